"""Downsampling flows' slot permutations through the C ABI (needs an MI355X): the
decomposition (one ciphertext, nj_conv2d_cins) and the densify (four ciphertexts,
nj_conv2d_block) word for word against the oracle at N = 2^12 with the oracle's
diagonals, and the library's own plans at N = 2^16 decrypting to the permuted slots."""
import numpy as np
import pytest

import oracle as O
import oracle.downsample as D
import oracle.plans as PL
from oracle.pipeline import block_bsgs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2312_04356_amd import Ct  # noqa: E402
from paper_2312_04356_amd.workload import GpuWorkload  # noqa: E402
from tests.oracle_workload import OracleWorkload  # noqa: E402

RNG = np.random.default_rng(43)


def host_coeff(gctx, ct):
    t = ct.data.clone()
    gctx.nj_to_coeff(t, ct.level, 2 * (t.numel() // (2 * (ct.level + 1) * gctx.N)))
    torch.cuda.synchronize()
    return gctx.to_host(t)


def random_ct(o, level):
    q = o.ring.q
    return np.stack([np.stack([RNG.integers(0, q[i], o.N, dtype=np.uint64) for i in range(level + 1)])
                     for _ in range(2)])


@pytest.mark.parametrize("half", [0, 1])
def test_decompose_parity_small(half):
    o = OracleWorkload("small", with_cts=False)
    g = GpuWorkload("small", with_cts=False)
    gctx, N, R, lvl = g.ctx, o.N, o.ring, 5
    W, C = 32, 4
    plan = gctx.nj_downsample_plan_create(0, W, C, half, lvl)
    bs, pts = D.decompose_plan(N, W, C, half)
    assert sorted(plan.offsets(0)) == sorted(bs.js) and len(bs.js) == W - 1
    enc = PL.encode_diagonals(pts, N, float(R.q[lvl]), R, lvl)
    for idx, j in enumerate(plan.offsets(0)):
        gctx.nj_plan_set_diagonal(plan, 0, idx, enc[j])
    gs = plan.galois()
    assert set(gs) == {PL.galois_elt(r, N) for r in bs.rotations()}
    g.make_keys(gs)
    o.make_keys(gs)
    x = random_ct(o, lvl)
    xt = gctx.to_device(x.reshape(2 * (lvl + 1), N))
    gctx.nj_to_eval(xt, lvl, 2)
    out = gctx.empty_ct(lvl - 1)
    gctx.nj_conv2d_cins(plan, Ct(xt, lvl, scale=2.0 ** 40), out)
    want = o.ctx.ct_rescale(lvl, o.ctx.bsgs(lvl, x, bs, enc))
    assert np.array_equal(host_coeff(gctx, out), want)


def test_densify_parity_small():
    o = OracleWorkload("small", with_cts=False)
    g = GpuWorkload("small", with_cts=False)
    gctx, N, R, lvl = g.ctx, o.N, o.ring, 4
    W, C, half = 32, 4, 0
    plan = gctx.nj_downsample_plan_create(1, W, C, half, lvl)
    _, _, _, bi, bo = plan.layout()[1:]
    assert (bi, bo) == (4, 1)
    bs, per = D.densify_plan(N, W, C, half)
    js = plan.offsets(0)
    assert sorted(js) == sorted(bs.js)
    nd = len(js)
    blocks = {}
    for m in range(4):
        enc = PL.encode_diagonals(per[m], N, float(R.q[lvl]), R, lvl)
        blocks[(0, m)] = enc
        for d, j in enumerate(js):
            if j in enc:
                gctx.nj_plan_set_diagonal(plan, 0, m * nd + d, enc[j])
    gs = plan.galois()
    g.make_keys(gs)
    o.make_keys(gs)
    xs = [random_ct(o, lvl) for _ in range(4)]
    xt = gctx.to_device(np.stack(xs).reshape(8 * (lvl + 1), N))
    gctx.nj_to_eval(xt, lvl, 8)
    out = gctx.empty_batch(1, lvl - 1)
    gctx.nj_conv2d_block(plan, Ct(xt, lvl, scale=2.0 ** 40), out)
    want = o.ctx.ct_rescale(lvl, block_bsgs(o.ctx, lvl, xs, bs, blocks, 1)[0])
    assert np.array_equal(host_coeff(gctx, out)[0], want)


def test_own_decompose_plan_full():
    """N = 2^16, W = 64, C = 16 (63 diagonals): the library's plan on an encrypted real
    slot vector decrypts to the permuted vector"""
    g = GpuWorkload("full", with_cts=False)
    gctx, N, lvl, half = g.ctx, g.N, 7, 0
    n = N // 2
    plan = gctx.nj_downsample_plan_create(0, 64, 16, half, lvl)
    assert len(plan.offsets(0)) == 63
    g.make_keys(plan.galois())
    z = RNG.uniform(-1, 1, n)
    coeffs = gctx.nj_encode_slots(z, g.scale)
    m = torch.empty((lvl + 1, N), dtype=torch.int64, device=gctx.device)
    gctx.nj_upload_plain(coeffs, lvl, m)
    import synth
    a, e = synth.enc_randomness(g.q[:lvl + 1], N, 9, 1)
    ct = gctx.nj_encrypt_sk(m, lvl, a, e, g.scale, gctx.empty_ct(lvl))
    out = gctx.empty_ct(lvl - 1)
    gctx.nj_conv2d_cins(plan, ct, out)
    d = torch.empty((lvl, N), dtype=torch.int64, device=gctx.device)
    gctx.nj_decrypt(out, d)
    vals = O.centred_from_limbs(gctx.to_host(d)[:2], g.q[:2])
    got = gctx.nj_decode_slots(np.array(vals, dtype=np.float64), out.scale).real
    want = z[D.half_slot_map(D.decompose_coeff_map(N, 64, 16), N, half)]
    err = np.max(np.abs(got - want))
    print("decompose at N=2^16: max abs slot error %.2e" % err)
    assert err < 1e-6
