"""Oracle pins for the downsampling flows' slot permutations (Sec. 5, Algorithm 2,
Appendix B): the coefficient maps against image-level definitions (phase images by
slicing, even pixels by slicing), the half maps against the CoeffToSlot slot order, the
0/1 diagonals against the permutation they encode, the decomposed stride-2 conv against
FP64 strided convolution, and the homomorphic evaluation against the permuted slots."""
import numpy as np
import pytest

import oracle as O
import oracle.downsample as D
import oracle.encoding as E
import oracle.plans as PL
import synth
from oracle.pipeline import Ctx

RNG = np.random.default_rng(17)


def layout(img, W, C, N):
    """coefficient vector of C images (C_img <= C channels, w x w) in the conv output layout"""
    a = np.zeros(N)
    for c in range(img.shape[0]):
        for y in range(img.shape[1]):
            for x in range(img.shape[2]):
                a[D.coeff_index(c, y, x, W, C)] = img[c, y, x]
    return a


def slots_of(a, N):
    """(real slots, imaginary slots) that CoeffToSlot leaves for coefficients a"""
    n = N // 2
    rev = np.array([E.bitrev(j, n) for j in range(n)])
    return a[:n][rev], a[n:][rev]


@pytest.mark.parametrize("N,W,C", [(1024, 16, 4), (4096, 32, 4), (4096, 16, 16)])
def test_decompose_map_gives_phase_images(N, W, C):
    img = RNG.uniform(-1, 1, (C, W, W))
    src = D.decompose_coeff_map(N, W, C)
    assert sorted(src) == list(range(N))  # a permutation
    got = layout(img, W, C, N)[src]
    want = layout(PL.polyphase(img), W // 2, 4 * C, N)
    assert np.array_equal(got, want)


def test_densify_map_gathers_even_pixels():
    N, W, C = 4096, 32, 4
    imgs = [RNG.uniform(-1, 1, (C, W, W)) for _ in range(4)]
    got = np.zeros(N)
    for m in range(4):
        src = D.densify_coeff_map(N, W, C, m)
        sel = src >= 0
        got[sel] = layout(imgs[m], W, C, N)[src[sel]]
    dense = np.zeros((4 * C, W // 2, W // 2))
    for m in range(4):
        for i in range(C):
            dense[4 * i + m] = imgs[m][i, 0::2, 0::2]
    assert np.array_equal(got, layout(dense, W // 2, 4 * C, N))


@pytest.mark.parametrize("kind", ["decompose", "densify"])
def test_half_maps_and_diagonals_reproduce_the_permutation(kind):
    N, W, C = 4096, 32, 4
    n = N // 2
    img = RNG.uniform(-1, 1, (C, W, W))
    srcs = [D.decompose_coeff_map(N, W, C)] if kind == "decompose" else [D.densify_coeff_map(N, W, C, m)
                                                                          for m in range(4)]
    for src in srcs:
        a = layout(img, W, C, N)
        b = np.zeros(N)
        b[src >= 0] = a[src[src >= 0]]
        for half in (0, 1):
            hm = D.half_slot_map(src, N, half)
            x = slots_of(a, N)[half]
            want = slots_of(b, N)[half]
            got = D.apply_diagonals(D.perm_diagonals(hm), x)
            assert np.array_equal(got, want)
            assert len(D.perm_diagonals(hm)) == (W - 1 if kind == "decompose" else W // 2)


def test_decomposed_stride2_conv_equals_strided_conv():
    """the phase images the permutation produces, convolved by the stride-2 taps at unit
    stride, give the stride-2 convolution (FP64)"""
    w0, ci, co = 16, 3, 2
    img = RNG.uniform(-1, 1, (ci, w0, w0))
    K = RNG.uniform(-1, 1, (co, ci, 3, 3))
    N, W, C = 1024, 16, 4
    pad = np.zeros((C, W, W))
    pad[:ci] = img
    ph_layout = layout(pad, W, C, N)[D.decompose_coeff_map(N, W, C)]
    ph = np.zeros((4 * C, W // 2, W // 2))
    for c in range(4 * C):
        for y in range(W // 2):
            for x in range(W // 2):
                ph[c, y, x] = ph_layout[D.coeff_index(c, y, x, W // 2, 4 * C)]
    got = PL.conv2d_taps(ph[:4 * ci, :w0 // 2, :w0 // 2], PL.taps_stride2(K), co)
    assert np.allclose(got, PL.conv2d_strided(img, K, 2), atol=1e-12)


def test_homomorphic_decompose_and_densify():
    """N = 2^10: the BSGS evaluation of the decomposition (one ciphertext) and of the
    densify (four ciphertexts) decrypt to the permuted slots"""
    N, W, C = 1024, 16, 4
    q, p = PL.chain_primes(10, 4, 2, 50, 48, 50, lambda ln, b, c, ex: O.gen_primes(ln, b, c, ex))
    R = O.Ring(N, q, p)
    s = synth.ternary_secret(N, 32, 5)
    ctx = Ctx(R, s)
    scale, lvl = 2.0 ** 40, 3
    n = N // 2

    def key(r):
        g = PL.galois_elt(r, N)
        if g not in ctx.keys:
            a, e = synth.key_randomness(R.key_primes(), N, R.n_digits(R.L), 6, g)
            ctx.add_key(g, a, e)

    def enc(z, sub):
        m = R.to_rns(E.encode(z, N, scale), lvl)
        a, e = synth.enc_randomness(q[:lvl + 1], N, 7, sub)
        return R.encrypt_sk(lvl, s, m, a, e)

    def dec(ct, level):
        m = np.array(O.centred_from_limbs(R.decrypt(level, s, ct), q[:level + 1]), dtype=np.float64)
        return E.decode(m, N, scale)

    half = 1
    bs, pts = D.decompose_plan(N, W, C, half)
    for r in bs.rotations():
        key(r)
    x = RNG.uniform(-1, 1, n)
    ct = enc(x, 1)
    enc_pts = PL.encode_diagonals(pts, N, float(q[lvl]), R, lvl)
    y = ctx.ct_rescale(lvl, ctx.bsgs(lvl, ct, bs, enc_pts))
    want = x[D.half_slot_map(D.decompose_coeff_map(N, W, C), N, half)]
    assert np.max(np.abs(dec(y, lvl - 1) - want)) < 1e-6
    # densify: four inputs through one BSGS structure (block matrix-vector product)
    from oracle.pipeline import block_bsgs
    bs, per = D.densify_plan(N, W, C, 0)
    for r in bs.rotations():
        key(r)
    xs = [RNG.uniform(-1, 1, n) for _ in range(4)]
    cts = [enc(v, 10 + m) for m, v in enumerate(xs)]
    blocks = {(0, m): PL.encode_diagonals(per[m], N, float(q[lvl]), R, lvl) for m in range(4)}
    out = ctx.ct_rescale(lvl, block_bsgs(ctx, lvl, cts, bs, blocks, 1)[0])
    want = np.zeros(n)
    for m in range(4):
        hm = D.half_slot_map(D.densify_coeff_map(N, W, C, m), N, 0)
        want[hm >= 0] = xs[m][hm[hm >= 0]]
    assert np.max(np.abs(dec(out, lvl - 1) - want)) < 1e-6
