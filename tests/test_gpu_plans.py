"""Plan choices of the learned planner through the C ABI (needs an MI355X), word for word
against the oracle executing the same plan: CoeffToSlot with the depth and per-group
baby-step counts chosen (Sec. 2.6 leaves the BSGS split and the grouping of the DFT
stages free), with baby steps not hoisted, and the fused conv without hoisting."""
import numpy as np
import pytest

import oracle.plans as PL

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2312_04356_amd.workload import GpuWorkload  # noqa: E402
from tests.oracle_workload import OracleWorkload  # noqa: E402


def host_coeff(gctx, ct):
    t = ct.data.clone()
    gctx.nj_to_coeff(t, ct.level, 2)
    torch.cuda.synchronize()
    return gctx.to_host(t)


@pytest.mark.parametrize("groups,n1s,hoist", [(3, (4, 8, 2), False), (4, (2, 4, 8, 4), [True, False, True, False]),
                                              (2, (16, 4), True)])
def test_split_cts_plan_parity_small(groups, n1s, hoist):
    o = OracleWorkload("small", with_cts=False)
    g = GpuWorkload("small", with_cts=False)
    gctx, N, R = g.ctx, o.N, o.ring
    plan = gctx.nj_cts_plan_create_split(groups, n1s).set_lazy(True).set_hoist(hoist)
    ogroups = PL.cts_plan(N, groups, list(n1s))
    assert plan.count() == groups
    opts = []
    for t, (bs, diags) in enumerate(ogroups):
        assert sorted(plan.offsets(t)) == sorted(bs.js) and bs.n1 == n1s[t]
        pts = PL.encode_diagonals(diags, N, float(R.q[R.L - t]), R, R.L - t)
        for idx, j in enumerate(plan.offsets(t)):
            gctx.nj_plan_set_diagonal(plan, t, idx, pts[j])
        opts.append(pts)
    gs = sorted(set(plan.galois()))
    want_gs = {PL.galois_elt(r, N) for bs, _ in ogroups for r in bs.rotations()} | {2 * N - 1}
    assert set(gs) == want_gs
    g.make_keys(gs)
    o.make_keys(gs)
    m = R.to_rns(o.input_plaintext(), 0)
    x_o = o.encrypt_input(0)
    x_g = g.encrypt_input(0, m_dev=gctx.to_device(m))
    lvl = R.L - groups
    re, im = gctx.empty_ct(lvl), gctx.empty_ct(lvl)
    gctx.nj_coeff_to_slot(plan, x_g, re, im)
    w_re, w_im = o.ctx.coeff_to_slot(x_o, [bs for bs, _ in ogroups], opts, hoist=hoist, lazy=True)
    assert np.array_equal(host_coeff(gctx, re), w_re)
    assert np.array_equal(host_coeff(gctx, im), w_im)


def test_conv_without_hoisting_parity_small():
    o = OracleWorkload("small", with_cts=False)
    g = GpuWorkload("small", with_cts=False)
    gctx = g.ctx
    for idx, j in enumerate(g.conv_plan.offsets(0)):
        gctx.nj_plan_set_diagonal(g.conv_plan, 0, idx, o.conv_pts[j])
    g.conv_plan.set_hoist(False)
    gs = g.galois_elements()
    g.make_keys(gs)
    o.make_keys(gs)
    m = o.ring.to_rns(o.input_plaintext(), 1)
    x_o = o.encrypt_input(1)
    x_g = g.encrypt_input(1, m_dev=gctx.to_device(m))
    y = gctx.empty_ct(0)
    gctx.nj_conv2d_cins(g.conv_plan, x_g, y)
    want = o.ctx.conv2d_cins(x_o, o.conv_bsgs, o.conv_pts, hoist=False)
    assert np.array_equal(host_coeff(gctx, y), want)
    hoisted = o.ctx.conv2d_cins(x_o, o.conv_bsgs, o.conv_pts, hoist=True)
    assert not np.array_equal(hoisted, want)  # a different plan: different low bits


@pytest.mark.timeout(600)
def test_split_cts_plan_parity_full():
    """N = 2^16 (three digits): a depth-5 CoeffToSlot with chosen splits, lazy giant steps
    and hoisting on some groups only (plans the learned planner proposes), word for word"""
    import oracle as O
    O.set_threads(0)
    o = OracleWorkload("full", with_cts=False)
    g = GpuWorkload("full", with_cts=False)
    gctx, N, R = g.ctx, o.N, o.ring
    groups, n1s, hoist = 5, (2, 4, 4, 4, 4), [False, True, False, True, True]
    plan = gctx.nj_cts_plan_create_split(groups, n1s).set_lazy(True).set_hoist(hoist)
    ogroups = PL.cts_plan(N, groups, list(n1s))
    opts = []
    for t, (bs, diags) in enumerate(ogroups):
        assert sorted(plan.offsets(t)) == sorted(bs.js)
        pts = PL.encode_diagonals(diags, N, float(R.q[R.L - t]), R, R.L - t)
        for idx, j in enumerate(plan.offsets(t)):
            gctx.nj_plan_set_diagonal(plan, t, idx, pts[j])
        opts.append(pts)
    gs = sorted(set(plan.galois()))
    g.make_keys(gs)
    o.make_keys(gs)
    m = R.to_rns(o.input_plaintext(), 0)
    x_o = o.encrypt_input(0)
    x_g = g.encrypt_input(0, m_dev=gctx.to_device(m))
    lvl = R.L - groups
    re, im = gctx.empty_ct(lvl), gctx.empty_ct(lvl)
    gctx.nj_coeff_to_slot(plan, x_g, re, im)
    w_re, w_im = o.ctx.coeff_to_slot(x_o, [bs for bs, _ in ogroups], opts, hoist=hoist, lazy=True)
    assert np.array_equal(host_coeff(gctx, re), w_re)
    assert np.array_equal(host_coeff(gctx, im), w_im)
