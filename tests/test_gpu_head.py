"""The classifier head through the C ABI (needs an MI355X): the FC layer fused with the
whole StoC (Sec. 4.2.1) word for word against the oracle at N = 2^12 with the oracle's
diagonals, and with the library's own plan at N = 2^16 (512 -> 1000) decrypting to W x;
average pooling as depthwise convs (Sec. 3.3.5) at N = 2^16: 3x3 stride 2 on phase images
and the global 7 x 7 average, against plain FP64 pooling."""
import numpy as np
import pytest

import oracle as O
import oracle.encoding as E
import oracle.head as H
import oracle.plans as PL

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import synth  # noqa: E402
from paper_2312_04356_amd import Ct  # noqa: E402
from paper_2312_04356_amd.workload import GpuWorkload  # noqa: E402
from tests.oracle_workload import OracleWorkload  # noqa: E402

RNG = np.random.default_rng(47)


def host_coeff(gctx, ct):
    t = ct.data.clone()
    gctx.nj_to_coeff(t, ct.level, 2)
    torch.cuda.synchronize()
    return gctx.to_host(t)


def decrypt_coeffs(g, ct):
    d = torch.empty((ct.level + 1, g.N), dtype=torch.int64, device=g.ctx.device)
    g.ctx.nj_decrypt(ct, d)
    k = min(2, ct.level + 1)  # one limb at level 0 holds |m| < q_0 / 2 = 2^49
    return np.array(O.centred_from_limbs(g.ctx.to_host(d)[:k], g.q[:k]), dtype=np.float64) / ct.scale


def encrypt_coeffs(g, coeffs, level, sub):
    m = torch.empty((level + 1, g.N), dtype=torch.int64, device=g.ctx.device)
    g.ctx.nj_upload_plain(coeffs, level, m)
    a, e = synth.enc_randomness(g.q[:level + 1], g.N, 11, sub)
    return g.ctx.nj_encrypt_sk(m, level, a, e, g.scale, g.ctx.empty_ct(level))


def test_fc_parity_small():
    o = OracleWorkload("small", with_cts=False)
    g = GpuWorkload("small", with_cts=False)
    gctx, N, R, lvl = g.ctx, o.N, o.ring, 3
    n_in, n_out = 200, 300
    W = RNG.uniform(-1, 1, (n_out, n_in))
    plan = gctx.nj_fc_plan_create(W, lvl)
    bs, pts = H.fc_plan(N, n_in, n_out, W)
    assert sorted(plan.offsets(0)) == sorted(bs.js) and len(bs.js) == 512
    enc = PL.encode_diagonals(pts, N, float(R.q[lvl]), R, lvl)
    for idx, j in enumerate(plan.offsets(0)):
        gctx.nj_plan_set_diagonal(plan, 0, idx, enc[j])
    gs = plan.galois()
    g.make_keys(gs)
    o.make_keys(gs)
    x = np.stack([np.stack([RNG.integers(0, R.q[i], N, dtype=np.uint64) for i in range(lvl + 1)]) for _ in range(2)])
    xt = gctx.to_device(x.reshape(2 * (lvl + 1), N))
    gctx.nj_to_eval(xt, lvl, 2)
    out = gctx.empty_ct(lvl - 1)
    gctx.nj_conv2d_cins(plan, Ct(xt, lvl, scale=g.scale), out)
    assert np.array_equal(host_coeff(gctx, out), o.ctx.ct_rescale(lvl, o.ctx.bsgs(lvl, x, bs, enc)))


def test_fc_own_plan_full():
    """512 -> 1000 at N = 2^16 (period 1024): y_k at coefficient 32 k"""
    g = GpuWorkload("full", with_cts=False)
    gctx, N, lvl = g.ctx, g.N, 2
    n_in, n_out = 512, 1000
    W = RNG.uniform(-1, 1, (n_out, n_in)) / np.sqrt(n_in)
    x = RNG.uniform(-1, 1, n_in)
    plan = gctx.nj_fc_plan_create(W, lvl)
    g.make_keys(plan.galois())
    ct = encrypt_coeffs(g, gctx.nj_encode_slots(H.periodic_slots(x, n_in, n_out, N), g.scale), lvl, 1)
    out = gctx.empty_ct(lvl - 1)
    gctx.nj_conv2d_cins(plan, ct, out)
    dec = decrypt_coeffs(g, out)
    stride = N // (2 * 1024)
    err = np.max(np.abs(dec[np.arange(n_out) * stride] - W @ x))
    rest = np.ones(N, dtype=bool)
    rest[np.arange(n_out) * stride] = False
    print("FC 512->1000 at N=2^16: max abs error %.2e, off-position %.2e" % (err, np.max(np.abs(dec[rest]))))
    assert err < 2.0 ** -15 and np.max(np.abs(dec[rest])) < 2.0 ** -15


def read_layout(coeffs, W, C, w, nch):
    out = np.zeros((nch, w, w))
    for c in range(nch):
        rc = E.bitrev(c, C)
        for y in range(w):
            out[c, y] = coeffs[(y * W + np.arange(w)) * C + rc]
    return out


def test_average_pooling_full():
    g = GpuWorkload("full", with_cts=False)
    gctx = g.ctx
    # 3x3 stride 2 on 16 channels of 56 x 56: phase images (64 channels of 28 x 28, W = 32)
    C_img, w = 16, 56
    img = RNG.uniform(-1, 1, (C_img, w, w))
    plan = gctx.nj_conv_plan_create_layer(w, np.full((C_img, 3, 3), 1.0 / 9.0), stride=2, depthwise=True, level=1)
    lv, W, C, ell, bi, bo = plan.layout()
    assert (W, C, bi, bo) == (32, 64, 1, 1)
    ph = np.zeros((C, W, W))
    ph[:, :28, :28] = PL.polyphase(img)
    g.make_keys(plan.galois())
    ct = encrypt_coeffs(g, gctx.nj_encode_cins(ph.reshape(C, W * W), g.scale), 1, 2)
    out = gctx.empty_ct(0)
    gctx.nj_conv2d_cins(plan, ct, out)
    got = read_layout(decrypt_coeffs(g, out), W, C, 28, C_img)
    err = np.max(np.abs(got - H.avg_pool(img, 3, 2)))
    print("3x3/2 average pooling at N=2^16: max abs error %.2e" % err)
    assert err < 2.0 ** -15
    # global average of 7 x 7 images: the 'same' depthwise 7x7 conv of weights 1/49 read at
    # the centre pixel (W = 16 holds every output pixel's taps without wrap-around, C = 256)
    Cg, wg = 64, 7
    img = RNG.uniform(-1, 1, (Cg, wg, wg))
    plan = gctx.nj_conv_plan_create_layer(wg, np.full((Cg, wg, wg), 1.0 / 49.0), depthwise=True, level=1)
    lv, W, C, ell, bi, bo = plan.layout()
    assert (W, C) == (16, 256)
    ch = np.zeros((C, W, W))
    ch[:Cg, :wg, :wg] = img
    g.make_keys(plan.galois())
    ct = encrypt_coeffs(g, gctx.nj_encode_cins(ch.reshape(C, W * W), g.scale), 1, 3)
    out = gctx.empty_ct(0)
    gctx.nj_conv2d_cins(plan, ct, out)
    got = read_layout(decrypt_coeffs(g, out), W, C, wg, Cg)[:, 3, 3]
    err = np.max(np.abs(got - img.mean(axis=(1, 2))))
    print("global average pooling at N=2^16: max abs error %.2e" % err)
    assert err < 2.0 ** -15
