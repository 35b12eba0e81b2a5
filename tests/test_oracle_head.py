"""Oracle pins for the classifier head (Sec. 4.2.1, Sec. 3.3.5): the FC matrix fused with
the whole StoC against the slot encoding's definition (its output's coefficients are
W x), its cyclic diagonals against the matrix, the homomorphic evaluation against W x,
and average pooling as a depthwise conv against plain pooling."""
import numpy as np

import oracle as O
import oracle.encoding as E
import oracle.head as H
import oracle.plans as PL
import synth
from oracle.pipeline import Ctx

RNG = np.random.default_rng(19)


def test_fc_matrix_puts_wx_in_the_coefficients():
    N, n_in, n_out = 1024, 40, 56
    W = RNG.uniform(-1, 1, (n_out, n_in))
    x = RNG.uniform(-1, 1, n_in)
    npp = H.period(n_in, n_out)
    z = H.periodic_slots(x, n_in, n_out, N)
    M = H.fc_matrix(n_in, n_out, W)
    out = np.tile(M @ z[:npp], (N // 2) // npp)
    f = E.slot_to_coeffs_direct(out, N)  # the coefficient view, by the encoding's definition
    stride = N // (2 * npp)
    want = np.zeros(N)
    want[np.arange(n_out) * stride] = W @ x
    assert np.max(np.abs(f - want)) < 1e-9
    # the diagonals give the same product on the whole periodic vector
    d = H.fc_diagonals(N, n_in, n_out, W)
    assert len(d) == npp
    from oracle.downsample import apply_diagonals
    assert np.max(np.abs(apply_diagonals(d, z) - out)) < 1e-9


def test_fc_homomorphic():
    N, n_in, n_out = 1024, 30, 50
    q, p = PL.chain_primes(10, 4, 2, 50, 48, 50, lambda ln, b, c, ex: O.gen_primes(ln, b, c, ex))
    R = O.Ring(N, q, p)
    s = synth.ternary_secret(N, 32, 8)
    ctx = Ctx(R, s)
    scale, lvl = 2.0 ** 40, 2
    W = RNG.uniform(-1, 1, (n_out, n_in)) / np.sqrt(n_in)
    x = RNG.uniform(-1, 1, n_in)
    bs, pts = H.fc_plan(N, n_in, n_out, W)
    for r in bs.rotations():
        g = PL.galois_elt(r, N)
        if g not in ctx.keys:
            a, e = synth.key_randomness(R.key_primes(), N, R.n_digits(R.L), 9, g)
            ctx.add_key(g, a, e)
    m = R.to_rns(E.encode(H.periodic_slots(x, n_in, n_out, N), N, scale), lvl)
    a, e = synth.enc_randomness(q[:lvl + 1], N, 10, 0)
    ct = R.encrypt_sk(lvl, s, m, a, e)
    enc = PL.encode_diagonals(pts, N, float(q[lvl]), R, lvl)
    y = ctx.ct_rescale(lvl, ctx.bsgs(lvl, ct, bs, enc))
    dec = np.array(O.centred_from_limbs(R.decrypt(lvl - 1, s, y), q[:lvl]), dtype=np.float64) / scale
    stride = N // (2 * H.period(n_in, n_out))
    assert np.max(np.abs(dec[np.arange(n_out) * stride] - W @ x)) < 1e-6
    mask = np.ones(N, dtype=bool)
    mask[np.arange(n_out) * stride] = False
    assert np.max(np.abs(dec[mask])) < 1e-6


def test_average_pooling_as_depthwise_conv():
    """3x3 stride 2 via the phase images and the stride-2 depthwise taps; the global
    average as the 'same' depthwise conv read at the centre"""
    C, w = 3, 8
    img = RNG.uniform(-1, 1, (C, w, w))
    K4 = np.zeros((C, C, 3, 3))  # depthwise: one kernel of weights 1/9 per channel
    for c in range(C):
        K4[c, c] = 1.0 / 9.0
    got = PL.conv2d_taps(PL.polyphase(img), PL.taps_stride2(K4), C)
    assert np.allclose(got, H.avg_pool(img, 3, 2), atol=1e-12)
    Kg = np.full((C, w - 1, w - 1), 1.0 / (w - 1) ** 2)
    sub = img[:, :w - 1, :w - 1]
    full = PL.conv2d_taps(sub, PL.taps_depthwise(Kg), C)
    c0 = (w - 2) // 2
    assert np.allclose(full[:, c0, c0], sub.mean(axis=(1, 2)), atol=1e-12)
