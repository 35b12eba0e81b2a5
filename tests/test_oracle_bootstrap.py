"""Pins of the ModEval / StoC1 oracle: the Chebyshev interpolant against the function,
the Chebyshev division against numpy's Chebyshev arithmetic, StoC1's composed
diagonals against dense stage matrices, homomorphic ModEval against the FP64 model and
the true message, and a whole bootstrap (ModRaise, CoeffToSlot, ModEval, Re + i Im,
StoC1, the remaining StoC2 stages) returning the coefficients it started from."""
import numpy as np
import pytest
from numpy.polynomial import chebyshev as CH

import oracle as O
import oracle.bootstrap as B
import oracle.encoding as E
import oracle.plans as PL
import synth
from oracle.pipeline import Ctx

RNG = np.random.default_rng(17)
K, R_DA = 16, 3


def test_interpolant_matches_function():
    c = B.cheb_coeffs(K, R_DA)
    x = np.linspace(-1, 1, 2001)
    g = np.cos(2 * np.pi * (K * x - 0.25) / 8)
    assert np.max(np.abs(CH.chebval(x, c) - g)) < 1e-12
    # after the double angles: sin(2 pi K x)
    y = CH.chebval(x, c)
    for _ in range(R_DA):
        y = 2 * y * y - 1
    assert np.max(np.abs(y - np.sin(2 * np.pi * K * x))) < 1e-10


@pytest.mark.parametrize("G,d", [(32, 63), (16, 31), (8, 15), (8, 8), (16, 20)])
def test_chebyshev_division(G, d):
    c = RNG.normal(0, 1, d + 1)
    q, r = B.cheb_split(c, G)
    TG = np.zeros(G + 1)
    TG[G] = 1.0
    back = CH.chebadd(CH.chebmul(q, TG), r)
    assert len(r) == G
    assert np.allclose(back[:d + 1], c, atol=1e-12) and np.allclose(back[d + 1:], 0, atol=1e-12)


def test_stoc1_diagonals_equal_dense_stage_product():
    n, ell = 64, 16
    for d in (1, 2, 3):
        groups = B.stoc1_stage_groups(ell, d)
        assert [k for g in groups for k in g] == [1, 2, 4, 8]
        M = np.eye(n, dtype=complex)
        for k in [k for g in groups for k in g]:
            M = E.S_stage_dense(k, n) @ M
        z = RNG.normal(size=n) + 1j * RNG.normal(size=n)
        y = z
        for plan, diags in B.stoc1_plan(2 * n, ell, d):
            full = {(j * plan.u) % n: E.rotl(v, plan.split[j][0] * plan.n1 * plan.u) for j, v in diags.items()}
            y = E.apply_diagonals(full, y)
        assert np.allclose(y, M @ z)


class Small:
    """N = 2^11 ring with 21 ciphertext primes (q0 ~ 2^50, others ~ 2^48), alpha = 4,
    scale 2^40, sparse ternary secret of weight 32"""

    def __init__(self):
        self.N = N = 1 << 11
        q, p = PL.chain_primes(11, 21, 4, 50, 48, 50, lambda ln, b, c, ex: O.gen_primes(ln, b, c, ex))
        self.R = O.Ring(N, q, p)
        self.q = q
        self.s = synth.ternary_secret(N, 32, 77)
        self.ctx = Ctx(self.R, self.s)
        self.boot = B.Boot(self.ctx)
        self.scale = 2.0 ** 40

    def key(self, g):
        if g not in self.ctx.keys:
            a, e = synth.key_randomness(self.R.key_primes(), self.N, self.R.n_digits(self.R.L), 78,
                                        synth.RELIN_KEY_ID if g == "relin" else g)
            self.ctx.add_key(g, a, e)

    def enc(self, coeffs, level, sub):
        m = self.R.to_rns(coeffs, level)
        a, e = synth.enc_randomness(self.q[:level + 1], self.N, 79, sub)
        return self.R.encrypt_sk(level, self.s, m, a, e)

    def dec(self, x, level, scale):
        m = self.R.decrypt(level, self.s, x)
        return np.array(O.centred_from_limbs(m, self.q[:level + 1]), dtype=np.float64) / scale


@pytest.fixture(scope="module")
def sm():
    S = Small()
    S.key("relin")
    return S


@pytest.mark.parametrize("accumulate", [False, True])
def test_homomorphic_chebyshev_matches_chebval(sm, accumulate):
    """degree-63 series on encrypted x in [-1, 1] (slots), scale ~2^48, in both
    evaluation orders of the baby-step sums"""
    n = sm.N // 2
    xv = RNG.uniform(-1, 1, n)
    c = RNG.normal(0, 1, 64) / (1 + np.arange(64)) ** 2
    l1 = 19
    ct = (sm.enc(E.encode(xv, sm.N, 2.0 ** 48), l1, 0), l1, 2.0 ** 48)
    T = sm.boot.cheb_basis(ct)
    lam = l1 - 7
    out = sm.boot.eval_cheb(T, c, lam, float(sm.q[lam]), accumulate)
    got = E.decode(np.rint(sm.dec(out[0], out[1], 1.0)), sm.N, out[2])
    assert out[1] == lam
    assert np.max(np.abs(got.real - CH.chebval(xv, c))) < 1e-8


def test_eval_orders_agree_within_noise(sm):
    """the two evaluation orders of ModEval differ only in rounding: different low bits,
    the same message within 2^-20"""
    n = sm.N // 2
    P = sm.q[0] / sm.scale
    t = RNG.uniform(-1, 1, n) + P * RNG.integers(-6, 7, n)
    ct = (sm.enc(E.encode(t, sm.N, sm.scale), 20, 2), 20, sm.scale)
    c = B.cheb_coeffs(K, R_DA)
    a = sm.boot.eval_mod(ct, K, R_DA, c)
    b = sm.boot.eval_mod(ct, K, R_DA, c, accumulate=True)
    assert a[1] == b[1] and a[2] == b[2]
    assert not np.array_equal(a[0], b[0])
    za = E.decode(np.rint(sm.dec(a[0], a[1], 1.0)), sm.N, a[2]).real
    zb = E.decode(np.rint(sm.dec(b[0], b[1], 1.0)), sm.N, b[2]).real
    assert np.max(np.abs(za - zb)) < 2.0 ** -20


def test_eval_mod_recovers_message(sm):
    """slots t = m + P I (P = q0 / scale): ModEval returns m up to the sine's error and
    matches the FP64 model of the same chain"""
    n = sm.N // 2
    P = sm.q[0] / sm.scale
    m = RNG.uniform(-1, 1, n)
    I = RNG.integers(-6, 7, n)
    t = m + P * I
    l0 = 20
    ct = (sm.enc(E.encode(t, sm.N, sm.scale), l0, 1), l0, sm.scale)
    c = B.cheb_coeffs(K, R_DA)
    out = sm.boot.eval_mod(ct, K, R_DA, c)
    assert out[1] == l0 - 11
    got = E.decode(np.rint(sm.dec(out[0], out[1], 1.0)), sm.N, out[2]).real
    want_model = B.model(t, P, K, R_DA, c)
    print("ModEval: max |got - model| %.2e, max |got - m| %.2e" % (np.max(np.abs(got - want_model)),
                                                                 np.max(np.abs(got - m))))
    assert np.max(np.abs(got - want_model)) < 2.0 ** -15
    assert np.max(np.abs(got - m)) < 1e-4


def test_bootstrap_round_trip(sm):
    """coefficients c (scale 2^40, |c| < 1) at level 0 -> ModRaise -> CoeffToSlot (2
    groups) -> ModEval on Re and Im -> Re + i Im -> StoC1 (ell = 64, 2 groups) ->
    S_{n/2} ... S_ell (one transform) -> the same coefficients"""
    N, n, ell = sm.N, sm.N // 2, 64
    L = sm.R.L
    coeffs = RNG.uniform(-1, 1, N)
    x0 = sm.enc(np.rint(coeffs * sm.scale).astype(np.int64), 0, 2)
    groups = PL.cts_plan(N, 2)
    s2_strides = []
    k = ell
    while k < n:
        s2_strides.append(k)
        k *= 2
    st1 = B.stoc1_plan(N, ell, 2)
    M = None
    for k in s2_strides:
        D = E.stage_diagonals(k, n)
        M = D if M is None else E.compose(D, M, n)
    s2 = PL.Bsgs(n, ell, M.keys())
    s2_diags = PL.prerotate(s2, M)
    rots = set(s2.rotations())
    for bs, _ in groups + st1:
        rots |= set(bs.rotations())
    for r in sorted(rots):
        sm.key(PL.galois_elt(r, N))
    sm.key(2 * N - 1)
    cts_pts = []
    for g, (bs, diags) in enumerate(groups):
        cts_pts.append(PL.encode_diagonals(diags, N, float(sm.q[L - g]), sm.R, L - g))
    re, im = sm.ctx.coeff_to_slot(x0, [b for b, _ in groups], cts_pts)
    lvl = L - len(groups)
    c = B.cheb_coeffs(K, R_DA)
    er = sm.boot.eval_mod((re, lvl, sm.scale), K, R_DA, c)
    ei = sm.boot.eval_mod((im, lvl, sm.scale), K, R_DA, c)
    z = sm.boot.combine(er, ei)
    l = z[1]
    st1_pts = [(bs, PL.encode_diagonals(d, N, float(sm.q[l - g]), sm.R, l - g)) for g, (bs, d) in enumerate(st1)]
    y = sm.boot.stoc1(z, st1_pts)
    l = y[1]
    pts = PL.encode_diagonals(s2_diags, N, float(sm.q[l]), sm.R, l)
    out = sm.ctx.ct_rescale(l, sm.ctx.bsgs(l, y[0], s2, pts))
    got = sm.dec(out, l - 1, y[2])
    err = np.max(np.abs(got - coeffs))
    print("bootstrap round trip: level %d, max coefficient error %.2e" % (l - 1, err))
    assert err < 1e-4


@pytest.mark.parametrize("N,W,C,w0", [(1 << 12, 32, 4, 16), (1 << 16, 64, 16, 32), (1 << 11, 16, 8, 12)])
def test_layer_masks_mark_the_conv_output_pixels(N, W, C, w0):
    """the masks' ones are exactly the coefficients the conv output is read from,
    a[(y W + x) C + rev_C(c)] for y, x < w0, seen through CoeffToSlot's bit-reversed halves"""
    ind = np.zeros(N)
    for c in range(C):
        for y in range(w0):
            ind[(y * W + np.arange(w0)) * C + E.bitrev(c, C)] = 1.0
    n2 = N // 2
    rev = np.array([E.bitrev(j, n2) for j in range(n2)])
    mre, mim = B.layer_masks(N, W, C, w0)
    assert ind.sum() == C * w0 * w0 == mre.sum() + mim.sum()
    assert np.array_equal(mre, ind[:n2][rev]) and np.array_equal(mim, ind[n2:][rev])


def test_masked_square_layer_round_trip(sm):
    """Algorithm 1's tail on a bootstrapped ciphertext: coefficients c laid out as a conv
    output (W = 16, C = 8, w0 = 12) -> ModRaise -> CoeffToSlot -> ModEval, zero-padding
    masks, the square activation, Re + i Im, StoC1 -> the remaining StoC2 stages: the
    coefficients come back as c^2 on output pixels and 0 on padding"""
    N, n = sm.N, sm.N // 2
    W, C, w0 = 16, 8, 12
    ell = W * W // 2
    L = sm.R.L
    coeffs = RNG.uniform(-1, 1, N)
    x0 = sm.enc(np.rint(coeffs * sm.scale).astype(np.int64), 0, 3)
    groups = PL.cts_plan(N, 2)
    st1 = B.stoc1_plan(N, ell, 2)
    M = None
    k = ell
    while k < n:
        D = E.stage_diagonals(k, n)
        M = D if M is None else E.compose(D, M, n)
        k *= 2
    s2 = PL.Bsgs(n, ell, M.keys())
    s2_diags = PL.prerotate(s2, M)
    rots = set(s2.rotations())
    for bs, _ in groups + st1:
        rots |= set(bs.rotations())
    for r in sorted(rots):
        sm.key(PL.galois_elt(r, N))
    sm.key(2 * N - 1)
    cts_pts = [PL.encode_diagonals(d, N, float(sm.q[L - g]), sm.R, L - g) for g, (_, d) in enumerate(groups)]
    re, im = sm.ctx.coeff_to_slot(x0, [b for b, _ in groups], cts_pts)
    lvl = L - len(groups)
    le = lvl - 11  # ModEval output level: masks encoded at q_le
    mre, mim = B.layer_masks(N, W, C, w0)
    masks = tuple(sm.R.to_rns(E.encode(m, N, float(sm.q[le])), le) for m in (mre, mim))
    lp = le - 2  # after the mask and the square
    st1_pts = [(bs, PL.encode_diagonals(d, N, float(sm.q[lp - g]), sm.R, lp - g)) for g, (bs, d) in enumerate(st1)]
    y = sm.boot.slot_activation((re, lvl, sm.scale), (im, lvl, sm.scale), K, R_DA, B.cheb_coeffs(K, R_DA), masks, 1,
                                st1_pts, lp)
    assert y[1] == lp - 2
    l = y[1]
    pts = PL.encode_diagonals(s2_diags, N, float(sm.q[l]), sm.R, l)
    out = sm.ctx.ct_rescale(l, sm.ctx.bsgs(l, y[0], s2, pts))
    got = sm.dec(out, l - 1, y[2])
    p = np.arange(N) // C
    valid = (p // W < w0) & (p % W < w0)
    err = np.max(np.abs(got - np.where(valid, coeffs ** 2, 0.0)))
    print("masked square layer: level %d, max error %.2e" % (l - 1, err))
    assert err < 1e-3
