"""Homomorphic pins of the oracle's fused conv + CoeffToSlot at N = 2^12 (the small workload).

The decrypted conv output is compared with the plain FP64 conv2d (bound 2^-15 at
scale 2^40); the CoeffToSlot output slots are compared with the bit-reversed
coefficients of the ModRaised plaintext (Sec. 2.4), computed directly in integers.
"""
import numpy as np
import pytest

import oracle as O
import oracle.encoding as E
from oracle.pipeline import Ctx
from tests.oracle_workload import OracleWorkload


@pytest.fixture(scope="module")
def wl():
    w = OracleWorkload("small")
    w.make_keys()
    return w


@pytest.fixture(scope="module")
def conv_out(wl):
    ct = wl.encrypt_input(1)
    return wl.ctx.conv2d_cins(ct, wl.conv_bsgs, wl.conv_pts, level=1, hoist=True)


def test_fused_conv_decrypts_to_conv2d(wl, conv_out):
    m = wl.ring.decrypt(0, wl.s, conv_out)
    vals = np.array(O.centred_from_limbs(m, wl.ring.q[:1]), dtype=np.float64) / wl.scale
    got = wl.read_conv_output(vals)
    err = np.max(np.abs(got - wl.conv_reference()))
    assert err <= 2.0 ** -15, err


def test_hoisted_and_plain_baby_steps_agree_within_noise(wl):
    ct = wl.encrypt_input(1)
    a = wl.ctx.bsgs(1, ct, wl.conv_bsgs, wl.conv_pts, hoist=True)
    b = wl.ctx.bsgs(1, ct, wl.conv_bsgs, wl.conv_pts, hoist=False)
    assert not np.array_equal(a, b)  # several correct results: the plan fixes the bits
    da = O.centred_from_limbs(wl.ring.decrypt(1, wl.s, a), wl.ring.q[:2])
    db = O.centred_from_limbs(wl.ring.decrypt(1, wl.s, b), wl.ring.q[:2])
    # both are at scale 2^40 q_1 before the rescale: they agree to 2^-20 of that scale
    assert max(abs(x - y) for x, y in zip(da, db)) < wl.scale * wl.ring.q[1] * 2.0 ** -20


def raw_modraised(wl, ct0):
    """c0 + c1 s over the integers with centred level-0 components = m + q0 I"""
    q0 = wl.ring.q[0]
    c = [np.where(ct0[k][0] > q0 // 2, ct0[k][0].astype(np.int64) - np.int64(q0), ct0[k][0].astype(np.int64))
         for k in range(2)]
    N = wl.N
    prod = np.zeros(N, dtype=np.int64)
    for i in np.nonzero(wl.s)[0]:
        sh = np.roll(c[1], i)
        sh[:i] = -sh[:i]
        prod += int(wl.s[i]) * sh
    return c[0] + prod


@pytest.mark.slow
def test_coeff_to_slot_gives_bit_reversed_coefficients(wl, conv_out):
    re, im = wl.ctx.coeff_to_slot(conv_out, [p for p, _ in wl.cts], [pts for _, pts in wl.cts])
    level = wl.ring.L - len(wl.cts)
    raw = raw_modraised(wl, conv_out).astype(np.float64) / wl.scale
    n = wl.N // 2
    rev = np.array([E.bitrev(j, n) for j in range(n)])
    for ct, want in ((re, raw[:n][rev]), (im, raw[n:][rev])):
        m = O.centred_from_limbs(wl.ring.decrypt(level, wl.s, ct)[:2], wl.ring.q[:2])
        z = E.decode(np.array(m, dtype=np.float64), wl.N, wl.scale)
        assert np.max(np.abs(z.imag)) < 1e-3
        assert np.max(np.abs(z.real - want)) < 1e-3, np.max(np.abs(z.real - want))
    # the q0 I multiples are really there (ModRaise is not the identity on the message)
    assert np.max(np.abs(raw)) > wl.ring.q[0] / wl.scale


def test_lazy_giant_steps_agree_within_noise(wl):
    """one ModDown for the sum of the giant steps' inner products: a different rounding
    (several correct results), the same plaintext up to a few units per coefficient"""
    plan, pts = wl.cts[0]
    x = wl.ctx.ct_modraise(wl.encrypt_input(0))
    L = wl.ring.L
    assert len([g for g in plan.giants if g]) > 1
    a = wl.ctx.bsgs(L, x, plan, pts, lazy=False)
    b = wl.ctx.bsgs(L, x, plan, pts, lazy=True)
    assert not np.array_equal(a, b)
    da = O.centred_from_limbs(wl.ring.decrypt(L, wl.s, a), wl.ring.q[:L + 1])
    db = O.centred_from_limbs(wl.ring.decrypt(L, wl.s, b), wl.ring.q[:L + 1])
    # before the rescale the scale is 2^40 q_L; rounding differs by far less than q_L
    assert max(abs(p - q) for p, q in zip(da, db)) < wl.ring.q[L] * 2.0 ** -20


@pytest.mark.slow
def test_lazy_coeff_to_slot_gives_bit_reversed_coefficients(wl, conv_out):
    re, im = wl.ctx.coeff_to_slot(conv_out, [p for p, _ in wl.cts], [pts for _, pts in wl.cts], lazy=True)
    level = wl.ring.L - len(wl.cts)
    raw = raw_modraised(wl, conv_out).astype(np.float64) / wl.scale
    n = wl.N // 2
    rev = np.array([E.bitrev(j, n) for j in range(n)])
    for ct, want in ((re, raw[:n][rev]), (im, raw[n:][rev])):
        m = O.centred_from_limbs(wl.ring.decrypt(level, wl.s, ct)[:2], wl.ring.q[:2])
        z = E.decode(np.array(m, dtype=np.float64), wl.N, wl.scale)
        assert np.max(np.abs(z.real - want)) < 1e-3 and np.max(np.abs(z.imag)) < 1e-3
