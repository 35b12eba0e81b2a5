"""Lazy giant steps (one ModDown for the sum of a transform's giant-step inner
products) through the C ABI (needs an MI355X): CoeffToSlot bit-exact against the
oracle's lazy evaluation at N = 2^12, the benchmark's first CoeffToSlot group and a
transform of 31 giant steps (four chunks of key switches) bit-exact at N = 2^16,
batched equal to single calls, and the library's own lazy plans accurate at
N = 2^16."""
import numpy as np
import pytest

import oracle as O
import oracle.encoding as E
import oracle.plans as PL

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import synth  # noqa: E402
from paper_2312_04356_amd import Ct  # noqa: E402
from paper_2312_04356_amd.workload import GpuWorkload  # noqa: E402
from tests.oracle_workload import OracleWorkload  # noqa: E402


def host_coeff(gctx, t, level):
    t = t.clone()
    gctx.nj_to_coeff(t, level, 2)
    torch.cuda.synchronize()
    return gctx.to_host(t)


def cts_batch_vs_single(g, y, n):
    gctx = g.ctx
    lvl = gctx.L - g.w["cts_groups"]
    re, im = gctx.empty_batch(n, lvl), gctx.empty_batch(n, lvl)
    gctx.nj_coeff_to_slot_batch(g.cts_plan, y, n, re, im)
    torch.cuda.synchronize()
    for z in range(n):
        rz, iz = gctx.empty_ct(lvl), gctx.empty_ct(lvl)
        gctx.nj_coeff_to_slot(g.cts_plan, Ct(y.data[z], 0), rz, iz)
        assert torch.equal(rz.data, re.data[z]) and torch.equal(iz.data, im.data[z]), "ciphertext %d" % z
    return re, im


def test_lazy_coeff_to_slot_parity_small():
    o = OracleWorkload("small", with_cts=True)
    g = GpuWorkload("small", with_cts=True, lazy=True)
    gctx = g.ctx
    gs = g.cts_plan.galois()
    g.make_keys(gs)
    o.make_keys(gs)
    for t, (plan, pts) in enumerate(o.cts):
        for idx, j in enumerate(g.cts_plan.offsets(t)):
            gctx.nj_plan_set_diagonal(g.cts_plan, t, idx, pts[j])
    m = o.ring.to_rns(o.input_plaintext(), 0)
    x_o = o.encrypt_input(0)
    x_g = g.encrypt_input(0, m_dev=gctx.to_device(m))
    lvl = o.ring.L - len(o.cts)
    re, im = gctx.empty_ct(lvl), gctx.empty_ct(lvl)
    gctx.nj_coeff_to_slot(g.cts_plan, x_g, re, im)
    w_re, w_im = o.ctx.coeff_to_slot(x_o, [p for p, _ in o.cts], [pts for _, pts in o.cts], lazy=True)
    assert np.array_equal(host_coeff(gctx, re.data, lvl), w_re)
    assert np.array_equal(host_coeff(gctx, im.data, lvl), w_im)
    # before the rescale the two roundings differ (the rescale by q_L ~ 2^48 absorbs it)
    L = o.ring.L
    xr = gctx.empty_ct(L)
    gctx.nj_modraise(x_g, L, xr)
    lazy_out, plain_out = gctx.empty_ct(L), gctx.empty_ct(L)
    gctx.nj_plan_apply(g.cts_plan, 0, xr, lazy_out)
    g.cts_plan.set_lazy(False)
    gctx.nj_plan_apply(g.cts_plan, 0, xr, plain_out)
    g.cts_plan.set_lazy(True)
    xo = o.ctx.ct_modraise(x_o)
    plan0, pts0 = o.cts[0]
    assert np.array_equal(host_coeff(gctx, lazy_out.data, L), o.ctx.bsgs(L, xo, plan0, pts0, lazy=True))
    assert np.array_equal(host_coeff(gctx, plain_out.data, L), o.ctx.bsgs(L, xo, plan0, pts0, lazy=False))
    assert not torch.equal(lazy_out.data, plain_out.data)
    y = gctx.empty_batch(4, 0)
    for z in range(4):
        y.data[z].copy_(x_g.data)
    cts_batch_vs_single(g, y, 4)


def test_lazy_coeff_to_slot_group_parity_full():
    """N = 2^16 as the benchmark runs it: ModRaise of a level-0 ciphertext, then the
    first CoeffToSlot group (level 23, 32 diagonals, hoisted baby steps, lazy giant
    steps on the fused key-switch kernels), word for word against the oracle (about a
    minute of oracle time on one core)"""
    o = OracleWorkload("full", with_cts=True)
    g = GpuWorkload("full", with_cts=True, lazy=True)
    gctx = g.ctx
    plan0, pts0 = o.cts[0]
    gs = sorted({PL.galois_elt(r, o.N) for r in plan0.rotations()})
    assert set(gs) <= set(g.cts_plan.galois())
    g.make_keys(gs)
    o.make_keys(gs)
    for idx, j in enumerate(g.cts_plan.offsets(0)):
        gctx.nj_plan_set_diagonal(g.cts_plan, 0, idx, pts0[j])
    m = o.ring.to_rns(o.input_plaintext(), 0)
    x_o = o.encrypt_input(0)
    x_g = g.encrypt_input(0, m_dev=gctx.to_device(m))
    L = o.ring.L
    xr = gctx.empty_ct(L)
    gctx.nj_modraise(x_g, L, xr)
    out = gctx.empty_ct(L)
    gctx.nj_plan_apply(g.cts_plan, 0, xr, out)
    want = o.ctx.bsgs(L, o.ctx.ct_modraise(x_o), plan0, pts0, lazy=True)
    assert np.array_equal(host_coeff(gctx, out.data, L), want)


def test_lazy_many_giants_parity_full():
    """N = 2^16, level 1: a conv plan's structure (64 channels at W = 32, n1 = 2: one
    baby step, 31 giant steps, so the lazy giant steps run in four chunks that
    accumulate their inner products) with uniform random diagonals and input,
    word for word against the oracle's lazy evaluation"""
    rng = np.random.default_rng(23)
    o = OracleWorkload("full", with_cts=False)
    g = GpuWorkload("full", with_cts=False)
    gctx, N, q = g.ctx, g.N, g.q
    c, w0 = 64, 30
    taps = PL.taps_same(rng.uniform(-1, 1, (c, c, 3, 3)))
    plan = gctx.nj_conv_plan_create_taps(w0, c, c, taps, fuse=1, n1=2, level=1)
    lvl, W, C, ell, bi, bo = plan.layout()
    assert (lvl, W, C, bi, bo) == (1, 32, 64, 1, 1)
    js = plan.offsets(0)
    oplan = PL.Bsgs(N // 2, ell, [j * ell for j in js], n1=2)
    assert oplan.js == sorted(js) and len(oplan.giants) == 32
    pts = {j: np.stack([rng.integers(0, q[i], N, dtype=np.uint64) for i in range(2)]) for j in js}
    for idx, j in enumerate(js):
        gctx.nj_plan_set_diagonal(plan, 0, idx, pts[j])
    gs = plan.galois()
    assert sorted(gs) == sorted({PL.galois_elt(r, N) for r in oplan.rotations()})
    g.make_keys(gs)
    o.make_keys(gs)
    x = np.stack([np.stack([rng.integers(0, q[i], N, dtype=np.uint64) for i in range(2)]) for _ in range(2)])
    t = gctx.to_device(x.reshape(4, N))
    gctx.nj_to_eval(t, 1, 2)
    plan.set_lazy(True)
    y = gctx.empty_ct(1)
    gctx.nj_plan_apply(plan, 0, Ct(t, 1), y, 1)
    want = o.ctx.bsgs(1, x, oplan, pts, lazy=True)
    assert np.array_equal(host_coeff(gctx, y.data, 1), want)


def test_lazy_coeff_to_slot_full_accuracy_and_batch():
    g = GpuWorkload("full", with_cts=True, lazy=True)
    gctx = g.ctx
    g.make_keys()
    n = 3
    y = gctx.empty_batch(n, 0)
    for z in range(n):
        ct = g.encrypt_input(1)
        gctx.nj_conv2d_cins(g.conv_plan, ct, Ct(y.data[z], 0))
    re, im = cts_batch_vs_single(g, y, n)
    # slots: the bit-reversed halves of the ModRaised coefficients (m + q0 I) / scale
    q0 = g.q[0]
    c = host_coeff(gctx, y.data[0], 0)
    c0 = np.where(c[0][0] > q0 // 2, c[0][0].astype(np.int64) - np.int64(q0), c[0][0].astype(np.int64))
    c1 = np.where(c[1][0] > q0 // 2, c[1][0].astype(np.int64) - np.int64(q0), c[1][0].astype(np.int64))
    prod = np.zeros_like(c0)
    for i in np.nonzero(g.s)[0]:
        sh = np.roll(c1, i)
        sh[:i] = -sh[:i]
        prod += int(g.s[i]) * sh
    raw = (c0 + prod).astype(np.float64) / g.scale
    n2 = g.N // 2
    rev = np.array([E.bitrev(j, n2) for j in range(n2)])
    lvl = gctx.L - g.w["cts_groups"]
    for ct, want in ((re, raw[:n2][rev]), (im, raw[n2:][rev])):
        d = torch.empty((lvl + 1, g.N), dtype=torch.int64, device=gctx.device)
        gctx.nj_decrypt(Ct(ct.data[0], lvl), d)
        mm = O.centred_from_limbs(gctx.to_host(d)[:2], g.q[:2])
        zz = gctx.nj_decode_slots(np.array(mm, dtype=np.float64), g.scale)
        err = max(np.max(np.abs(zz.real - want)), np.max(np.abs(zz.imag)))
        print("lazy CoeffToSlot max abs slot error %.3e" % err)
        assert err < 1e-3
    assert synth.WORKLOADS["full"]["cts_groups"] == 3
