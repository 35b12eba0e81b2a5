"""Oracle pins for the conv variants: pointwise, stride 2 (polyphase decomposition),
depthwise (one PMult) and multi-ciphertext block convs, against plain FP64 convs."""
import numpy as np
import pytest

import oracle as O
import oracle.encoding as E
import oracle.plans as PL
from oracle.pipeline import Ctx, block_conv

RNG = np.random.default_rng(5)


def simulate_block(plan, bi, bo, diags, zs):
    outs = []
    for ob in range(bo):
        acc = 0
        for g in plan.giants:
            inner = 0
            for ib in range(bi):
                for j, (gg, i) in plan.split.items():
                    if gg == g and j in diags[(ob, ib)]:
                        inner = inner + diags[(ob, ib)][j] * E.rotl(zs[ib], plan.baby_rot(i))
            acc = acc + E.rotl(inner, plan.giant_rot(g))
        outs.append(acc)
    return outs


def read_layout(coeffs, W, C, w0):
    out = np.zeros((C, w0, w0))
    for c in range(C):
        rc = E.bitrev(c, C)
        for y in range(w0):
            out[c, y] = coeffs[(y * W + np.arange(w0)) * C + rc]
    return out


def run_fp64(img, taps, c_in, c_out, w0, N, fuse=True):
    W = PL.padded_width_taps(w0, taps)
    C = N // (W * W)
    ell = W * W // 2
    plan, bi, bo, diags = PL.block_conv_plan(taps, c_in, c_out, W, N, fuse)
    zs = []
    for ib in range(bi):
        ch = np.zeros((C, w0, w0))
        part = img[ib * C:(ib + 1) * C]
        ch[:part.shape[0]] = part
        zs.append(E.real_cins_slots(PL.image_to_slices(ch, W), ell))
    outs = simulate_block(plan, bi, bo, diags, zs)
    res = []
    for ob in range(bo):
        if fuse:
            f = E.slot_to_coeffs(outs[ob], N)
            res.append(read_layout(f, W, C, w0))
        else:  # CinS output: slice c holds DFT'(o_c)
            sl = outs[ob].reshape(C, ell)
            o = np.zeros((C, w0, w0))
            for c in range(C):
                # invert DFT' by least squares against the definition (small sizes only)
                M = E.omega(4 * ell) ** (np.outer(E.rot5(ell, 4 * ell), np.arange(2 * ell)) % (4 * ell))
                full = np.linalg.lstsq(np.vstack([M, np.conj(M)]), np.concatenate([sl[c], np.conj(sl[c])]),
                                       rcond=None)[0].real
                o[c] = full.reshape(W, W)[:w0, :w0]
            res.append(o)
    return np.concatenate(res)[:c_out]


def test_pointwise_conv():
    N, w0, C = 256, 8, 4
    img = RNG.uniform(-1, 1, (C, w0, w0))
    K = RNG.uniform(-1, 1, (C, C, 1, 1))
    got = run_fp64(img, PL.taps_same(K), C, C, w0, N)
    assert np.allclose(got, PL.conv2d_same(img, K), atol=1e-9)


def test_stride2_conv_by_polyphase_decomposition():
    N, w0 = 512, 8  # polyphase images 4x4 -> W = 8, C = 8 channels per ciphertext
    c_in, c_out = 2, 8
    img = RNG.uniform(-1, 1, (c_in, w0, w0))
    K = RNG.uniform(-1, 1, (c_out, c_in, 3, 3))
    taps = PL.taps_stride2(K)
    got = run_fp64(PL.polyphase(img), taps, 4 * c_in, c_out, w0 // 2, N)
    assert np.allclose(got, PL.conv2d_strided(img, K, 2), atol=1e-9)
    assert np.allclose(PL.conv2d_taps(PL.polyphase(img), taps, c_out), PL.conv2d_strided(img, K, 2))


def test_block_conv_two_by_two_blocks():
    N, w0 = 256, 6  # W = 8, C = 4 per ciphertext; 8 -> 8 channels = 2 x 2 blocks
    img = RNG.uniform(-1, 1, (8, w0, w0))
    K = RNG.uniform(-1, 1, (8, 8, 3, 3))
    got = run_fp64(img, PL.taps_same(K), 8, 8, w0, N)
    assert np.allclose(got, PL.conv2d_same(img, K), atol=1e-9)


def test_depthwise_is_one_diagonal_without_rotation():
    """Table 1: depthwise CinS conv = 1 PMult, 0 HRot (output stays CinS-encoded)"""
    N, w0, C = 256, 6, 4
    img = RNG.uniform(-1, 1, (C, w0, w0))
    K = RNG.uniform(-1, 1, (C, 3, 3))
    taps = PL.taps_depthwise(K)
    W = PL.padded_width_taps(w0, taps)
    plan, bi, bo, diags = PL.block_conv_plan(taps, C, C, W, N, fuse=False)
    assert len(diags[(0, 0)]) == 1 and plan.rotations() == []
    got = run_fp64(img, taps, C, C, w0, N, fuse=False)
    assert np.allclose(got, PL.conv2d_taps(img, taps, C), atol=1e-9)


def test_homomorphic_block_conv_decrypts_to_conv2d():
    """2 input and 2 output ciphertexts at N = 2^10, decrypted vs FP64 conv2d (2^-15)"""
    import synth
    N, w0 = 1024, 12  # W = 16, C = 4 per ciphertext
    q = O.gen_primes(10, 50, 1) + O.gen_primes(10, 48, 2, O.gen_primes(10, 50, 1))
    p = O.gen_primes(10, 50, 2, q)
    R = O.Ring(N, q, p)
    s = synth.ternary_secret(N, 32, 7)
    ctx = Ctx(R, s)
    img = RNG.uniform(-1, 1, (8, w0, w0))
    K = RNG.uniform(-1, 1, (8, 8, 3, 3))
    taps = PL.taps_same(K)
    W = PL.padded_width_taps(w0, taps)
    C, ell = N // (W * W), W * W // 2
    plan, bi, bo, diags = PL.block_conv_plan(taps, 8, 8, W, N)
    for r in plan.rotations():
        g = PL.galois_elt(r, N)
        a, e = synth.key_randomness(R.key_primes(), N, R.n_digits(R.L), 9, g)
        ctx.add_key(g, a, e)
    pts = {k: PL.encode_diagonals(v, N, float(q[1]), R, 1) for k, v in diags.items()}
    xs = []
    for ib in range(bi):
        z = E.real_cins_slots(PL.image_to_slices(img[ib * C:(ib + 1) * C], W), ell)
        m = R.to_rns(E.encode(z, N, 2.0 ** 40), 1)
        a, e = synth.enc_randomness(q[:2], N, 3, ib)
        xs.append(R.encrypt_sk(1, s, m, a, e))
    ys = block_conv(ctx, 1, xs, plan, pts, bo)
    want = PL.conv2d_same(img, K)
    for ob in range(bo):
        m = R.decrypt(0, s, ys[ob])
        vals = np.array(O.centred_from_limbs(m, q[:1]), dtype=np.float64) / 2.0 ** 40
        got = read_layout(vals, W, C, w0)
        assert np.max(np.abs(got - want[ob * C:(ob + 1) * C])) <= 2.0 ** -15
