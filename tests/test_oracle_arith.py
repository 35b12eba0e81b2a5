"""Pins of the oracle's exact integer arithmetic against mathematics it does not use.

Each check uses an independent route: Python big integers, schoolbook products,
evaluation of a polynomial at a root of unity, CRT reconstruction, or the
defining inequality of the operation.
"""
import random

import numpy as np
import pytest

import oracle as O
from oracle.pipeline import Ctx, automorph_int

RNG = random.Random(7)


def fermat_probable_prime(n, bases=(2, 3, 5, 7, 11, 13, 17)):
    return all(pow(b, n - 1, n) == 1 for b in bases if b % n)


def schoolbook(a, b, q):
    n = len(a)
    c = [0] * n
    for i in range(n):
        for j in range(n):
            k = i + j
            if k < n:
                c[k] += int(a[i]) * int(b[j])
            else:
                c[k - n] -= int(a[i]) * int(b[j])
    return [x % q for x in c]


def rand_poly(n, q):
    return np.array([RNG.randrange(q) for _ in range(n)], dtype=np.uint64)


def small_ring(n=32, nq=4, alpha=2, bits=50):
    log_n = n.bit_length() - 1
    q = O.gen_primes(log_n, bits, nq)
    p = O.gen_primes(log_n, bits, alpha, exclude=q)
    return O.Ring(n, q, p)


# ------------------------------------------------------------------ primes

@pytest.mark.parametrize("log_n,bits", [(5, 50), (12, 50), (16, 48), (16, 50)])
def test_prime_chain(log_n, bits):
    ps = O.gen_primes(log_n, bits, 6)
    m = 2 << log_n
    for q in ps:
        assert q < 2 ** bits and q % m == 1 and fermat_probable_prime(q)
    # no candidate of the form k*2N+1 between consecutive chosen primes was skipped
    top = ((2 ** bits - 2) // m) * m + 1
    chosen = set(ps)
    t = top
    while t >= min(ps):
        if t not in chosen:
            assert not fermat_probable_prime(t), t
        t -= m
    assert ps == sorted(ps, reverse=True)


def test_is_prime_known_values():
    assert O.is_prime(2 ** 61 - 1) and O.is_prime(2 ** 31 - 1)
    assert not O.is_prime(2 ** 61 + 1)
    for carmichael in (561, 41041, 825265, 321197185, 5394826801, 232250619601):
        assert not O.is_prime(carmichael)
    assert not O.is_prime(3215031751)  # strong pseudoprime to bases 2,3,5,7


def test_mulmod_big_int():
    q = O.gen_primes(16, 50, 1)[0]
    for _ in range(2000):
        a, b = RNG.randrange(q), RNG.randrange(q)
        assert O.mulmod(a, b, q) == a * b % q


# ------------------------------------------------------- transforms, products

@pytest.mark.parametrize("n", [8, 16, 64])
def test_polymul_equals_schoolbook(n):
    q = O.gen_primes(n.bit_length() - 1, 50, 1)[0]
    for _ in range(3):
        a, b = rand_poly(n, q), rand_poly(n, q)
        assert [int(x) for x in O.polymul(a, b, q)] == schoolbook(a, b, q)


@pytest.mark.parametrize("n", [16, 1024, 4096])
def test_ntt_roundtrip_and_linearity(n):
    q = O.gen_primes(n.bit_length() - 1, 50, 1)[0]
    a, b = rand_poly(n, q), rand_poly(n, q)
    assert np.array_equal(O.ntt_inv(O.ntt_fwd(a, q), q), a)
    lhs = O.ntt_fwd((a + b) % np.uint64(q), q)
    rhs = (O.ntt_fwd(a, q) + O.ntt_fwd(b, q)) % np.uint64(q)
    assert np.array_equal(lhs, rhs)


def test_psi_is_primitive_2n_root():
    for n in (16, 4096, 65536):
        q = O.gen_primes(n.bit_length() - 1, 50, 1)[0]
        psi = int(O.lib.or_find_psi(n, q))
        assert pow(psi, n, q) == q - 1


def test_monomial_is_product_with_x_power():
    n, q = 16, O.gen_primes(4, 50, 1)[0]
    a = rand_poly(n, q)
    for k in (0, 1, 5, n, n + 3, 2 * n - 1):
        xk = [0] * n
        sign = -1 if (k // n) % 2 else 1
        xk[k % n] = sign % q
        assert [int(v) for v in O.monomial(a, k, q)] == schoolbook(a, xk, q)


# ------------------------------------------------------------- automorphism

def eval_at(a, x, q):
    return sum(int(c) * pow(x, i, q) for i, c in enumerate(a)) % q


def test_automorphism_is_substitution_x_to_x_g():
    n = 32
    q = O.gen_primes(5, 50, 1)[0]
    psi = int(O.lib.or_find_psi(n, q))
    a = rand_poly(n, q)
    for g in (5, 25, 2 * n - 1, 3 ** 3 % (2 * n)):
        b = O.automorph(a, g, q)
        for e in (1, 3, 7, 2 * n - 1):  # every primitive 2n-th root is psi^odd
            x = pow(psi, e, q)
            assert eval_at(b, x, q) == eval_at(a, pow(x, g, q), q)


def test_automorphism_composition_and_multiplicativity():
    n = 64
    q = O.gen_primes(6, 50, 1)[0]
    a, b = rand_poly(n, q), rand_poly(n, q)
    g, h = 5, 2 * n - 1
    assert np.array_equal(O.automorph(O.automorph(a, g, q), h, q), O.automorph(a, g * h % (2 * n), q))
    assert np.array_equal(O.automorph(O.polymul(a, b, q), g, q),
                          O.polymul(O.automorph(a, g, q), O.automorph(b, g, q), q))


# ------------------------------------------------------ RNS basis changes

def crt(vals, primes):
    Q = 1
    for p in primes:
        Q *= p
    x = 0
    for v, p in zip(vals, primes):
        h = Q // p
        x += int(v) * h * pow(h % p, -1, p)
    return x % Q, Q


def test_modup_is_crt_plus_small_multiple():
    R = small_ring(n=16, nq=6, alpha=3)
    level = 5
    x = np.stack([rand_poly(R.n, q) for q in R.q[:level + 1]])
    for j in range(R.n_digits(level)):
        ext = R.modup_digit(level, j, x)
        lo, hi = j * R.alpha, min((j + 1) * R.alpha, level + 1)
        dig = R.q[lo:hi]
        primes = R.ext_primes(level)
        for k in range(R.n):
            X, D = crt([x[i, k] for i in range(lo, hi)], dig)
            us = set()
            for t, pt in enumerate(primes):
                if lo <= t < hi:
                    assert int(ext[t, k]) == int(x[t, k])
                    continue
                u = (int(ext[t, k]) - X) * pow(D % pt, -1, pt) % pt
                us.add(u)
            assert len(us) == 1 and 0 <= us.pop() < hi - lo


def test_moddown_divides_by_p_up_to_small_multiple():
    R = small_ring(n=16, nq=4, alpha=3)
    level = 3
    primes = R.ext_primes(level)
    u = np.stack([rand_poly(R.n, t) for t in primes])
    out = R.moddown(level, u)
    P = 1
    for p in R.p:
        P *= p
    for k in range(R.n):
        Y, _ = crt([u[level + 1 + a, k] for a in range(R.alpha)], R.p)
        vs = set()
        for i in range(level + 1):
            qi = R.q[i]
            w = (int(u[i, k]) - int(out[i, k]) * P - Y) % qi
            vs.add(w * pow(P, -1, qi) % qi)
        assert len(vs) == 1 and 0 <= vs.pop() < R.alpha


def test_rescale_is_rounded_division():
    R = small_ring(n=16, nq=5, alpha=2)
    level = 4
    a = np.stack([rand_poly(R.n, q) for q in R.q[:level + 1]])
    out = R.rescale(level, a)
    ql = R.q[level]
    for k in range(R.n):
        A, Q = crt(a[:, k], R.q[:level + 1])
        if A > Q // 2:
            A -= Q
        B, Qp = crt(out[:, k], R.q[:level])
        if B > Qp // 2:
            B -= Qp
        assert 2 * abs(B * ql - A) <= ql


def test_modraise_is_centred_lift():
    R = small_ring(n=16, nq=5, alpha=2)
    a0 = rand_poly(R.n, R.q[0])
    out = R.modraise(a0)
    for k in range(R.n):
        v = int(a0[k])
        c = v - R.q[0] if v > R.q[0] // 2 else v
        X, Q = crt(out[:, k], R.q)
        assert (X - Q if X > Q // 2 else X) == c


# ------------------------------------------------------------- key switching

def make_ctx(R, seed=5):
    import synth
    s = synth.ternary_secret(R.n, min(16, R.n // 2), seed)
    return Ctx(R, s)


def add_key(ctx, g, seed=9):
    import synth
    R = ctx.ring
    a, e = synth.key_randomness(R.key_primes(), R.n, R.n_digits(R.L), seed, g if g != "relin" else 0)
    return ctx.add_key(g, a, e)


def dec_centred(ctx, level, ct):
    m = ctx.ring.decrypt(level, ctx.s, ct)
    return O.centred_from_limbs(m, ctx.ring.q[:level + 1])


@pytest.mark.parametrize("level", [0, 2, 4])
def test_keyswitch_decrypts_to_d_times_sprime(level):
    R = small_ring(n=32, nq=5, alpha=2)
    ctx = make_ctx(R)
    g = 5
    key = add_key(ctx, g)
    sp = automorph_int(ctx.s, g)
    d = np.stack([rand_poly(R.n, q) for q in R.q[:level + 1]])
    k0, k1 = R.keyswitch(level, d, key)
    # k0 + k1 s - d s' must be small (key noise only)
    lhs = R.decrypt(level, ctx.s, np.stack([k0, k1]))
    ds = R.to_rns(np.zeros(R.n, dtype=np.int64), level)
    for i, q in enumerate(R.q[:level + 1]):
        spq = np.mod(sp, q).astype(np.uint64)
        ds[i] = O.polymul(d[i], spq, q)
    diff = O.centred_from_limbs(R.sub(level, lhs, ds), R.q[:level + 1])
    assert max(abs(x) for x in diff) < 2 ** 30


def test_encrypt_decrypt_roundtrip():
    import synth
    R = small_ring(n=32, nq=3, alpha=2)
    ctx = make_ctx(R)
    m = np.array([RNG.randrange(-2 ** 40, 2 ** 40) for _ in range(R.n)], dtype=np.int64)
    a, e = synth.enc_randomness(R.q[:3], R.n, 3)
    ct = R.encrypt_sk(2, ctx.s, R.to_rns(m, 2), a, e)
    got = dec_centred(ctx, 2, ct)
    assert max(abs(int(x) - int(y)) for x, y in zip(got, m)) <= 30


def int_negacyclic(a, b):
    """a * b in Z[X]/(X^n + 1) on plain Python integers"""
    n = len(a)
    c = [0] * n
    for i in range(n):
        for j in range(n):
            if a[i] and b[j]:
                k = i + j
                if k < n:
                    c[k] += int(a[i]) * int(b[j])
                else:
                    c[k - n] -= int(a[i]) * int(b[j])
    return c


@pytest.mark.parametrize("level", [0, 2])
def test_public_key_encryption_noise_is_exact(level):
    """Sec. 2.1: pk = (-a s + e, a) decrypts to e, and Enc(m; pk) decrypts to exactly
    m + v e + e0 + e1 s (integer negacyclic products), at the top level and below"""
    import synth
    R = small_ring(n=32, nq=3, alpha=2)
    ctx = make_ctx(R)
    a, e = synth.pk_randomness(R.q, R.n, 11)
    pk = R.gen_public_key(ctx.s, a, e)
    assert dec_centred(ctx, R.L, pk) == [int(x) for x in e]
    m = [RNG.randrange(-2 ** 30, 2 ** 30) for _ in range(R.n)]
    v, e0, e1 = synth.pk_enc_randomness(R.n, 12, 0, h=8)
    ct = R.encrypt_pk(level, pk, R.to_rns(np.array(m, dtype=np.int64), level), v, e0, e1)
    ve, e1s = int_negacyclic(v, e), int_negacyclic(e1, ctx.s)
    want = [m[k] + ve[k] + int(e0[k]) + e1s[k] for k in range(R.n)]
    assert dec_centred(ctx, level, ct) == want
    # the second component is v pk1 + e1 = v a + e1 on the first level+1 limbs
    va = int_negacyclic(v, [int(x) for x in a[0]])
    assert [int(x) for x in ct[1][0]] == [(va[k] + int(e1[k])) % R.q[0] for k in range(R.n)]
