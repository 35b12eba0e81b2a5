"""The fused kernels at the ring sizes between the small ring and the benchmark's
(N = 2^13, 2^14, 2^15: 2, 4 and 8 tiles of 4096 words per limb), word for word against
the oracle through the C ABI (needs an MI355X).

Each case runs the benchmark's step on a ring of 12 + alpha primes (alpha = 4: three
key-switching digits at the top level, the last one partial below it; alpha = 3: four
digits; alpha = 8: two): the conv at
level 1 (hoisted baby steps: key inner products on the Q limbs, special-prime rows
through ModDown's first inverse stages) -> rescale -> ModRaise -> CoeffToSlot in three
groups, with the giant steps lazy (one ModDown per group, inner products fused with
the digits' tile pass) or one key switch each, and the conjugate split fused into the
last ModDown.  Channels fill the ring: C = N / 32^2 input and output channels of a
16 x 16 image.
"""
import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2312_04356_amd.workload import GpuWorkload  # noqa: E402
from tests.midsize import mid_workload  # noqa: E402
from tests.oracle_workload import OracleWorkload  # noqa: E402


def host_coeff(gctx, ct, n_polys=2):
    t = ct.data.clone()
    gctx.nj_to_coeff(t, ct.level, n_polys)
    torch.cuda.synchronize()
    return gctx.to_host(t)


def load(gctx, plan, t, pts):
    for idx, j in enumerate(plan.offsets(t)):
        gctx.nj_plan_set_diagonal(plan, t, idx, pts[j])


@pytest.mark.timeout(600)
@pytest.mark.parametrize("log_n,lazy,alpha", [(13, True, 4), (14, False, 4), (15, True, 4), (15, False, 4),
                                              (14, True, 3), (13, False, 3), (14, True, 8), (15, False, 8)])
def test_step_parity_midsize(log_n, lazy, alpha):
    O.set_threads(0)
    name = mid_workload(log_n, alpha)
    print("[midsize] N=2^%d lazy=%s alpha=%d: setup" % (log_n, lazy, alpha), flush=True)
    o = OracleWorkload(name, with_cts=True)
    g = GpuWorkload(name, with_cts=True, lazy=lazy)
    gctx = g.ctx
    assert g.q == o.ring.q and g.p == o.ring.p
    assert gctx.dnum == {3: 4, 4: 3, 8: 2}[alpha]
    assert sorted(g.conv_plan.offsets(0)) == sorted(o.conv_bsgs.js)
    load(gctx, g.conv_plan, 0, o.conv_pts)
    assert g.cts_plan.count() == len(o.cts) == 3
    for t, (_, pts) in enumerate(o.cts):
        load(gctx, g.cts_plan, t, pts)
    gs = g.galois_elements()
    assert sorted(gs) == sorted(set(o.galois_elements()))
    g.make_keys(gs)
    o.make_keys(gs)
    m = o.ring.to_rns(o.input_plaintext(), 1)
    x_o = o.encrypt_input(1)
    x_g = g.encrypt_input(1, m_dev=gctx.to_device(m))
    print("[midsize] N=2^%d lazy=%s alpha=%d: library" % (log_n, lazy, alpha), flush=True)
    y = gctx.empty_ct(0)
    gctx.nj_conv2d_cins(g.conv_plan, x_g, y)
    lvl = gctx.L - 3
    re, im = gctx.empty_ct(lvl), gctx.empty_ct(lvl)
    gctx.nj_coeff_to_slot(g.cts_plan, y, re, im)
    torch.cuda.synchronize()
    print("[midsize] N=2^%d lazy=%s alpha=%d: oracle" % (log_n, lazy, alpha), flush=True)
    y_o = o.ctx.conv2d_cins(x_o, o.conv_bsgs, o.conv_pts)
    assert np.array_equal(host_coeff(gctx, y), y_o), "conv output differs"
    w_re, w_im = o.ctx.coeff_to_slot(y_o, [p for p, _ in o.cts], [pts for _, pts in o.cts], lazy=lazy)
    got_re, got_im = host_coeff(gctx, re), host_coeff(gctx, im)
    assert got_re.shape == w_re.shape == (2, lvl + 1, g.N)
    assert np.array_equal(got_re, w_re), "Re differs in %d words" % np.count_nonzero(got_re != w_re)
    assert np.array_equal(got_im, w_im), "Im differs in %d words" % np.count_nonzero(got_im != w_im)
    assert re.level == im.level == lvl
