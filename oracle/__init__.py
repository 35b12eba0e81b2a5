"""Oracle: plain CPU RNS-CKKS reference for the fused CinS-conv + CoeffToSlot path.

TEST INFRASTRUCTURE ONLY.  Only `tests/`, `__graft_entry__.smoke()` and the
CPU-baseline leg of `bench.py` may import this package.  It shares no code with
the HIP library (`paper_2312_04356_amd`) and never imports it.

Layers:
  * `ckks_oracle.c` (built to `liboracle.so`): exact modular-integer arithmetic
    (primes, NTT-based polynomial product, automorphisms, ModUp/ModDown,
    key switching, rescale, ModRaise, encryption).
  * `encoding.py`: FP64 slot/CinS encodings and the DFT-factor matrices.
  * `plans.py`: the fused conv diagonals (K' = S'K) and CoeffToSlot stage groups.
  * `pipeline.py`: baby-step/giant-step evaluation and the fused pipeline.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "ckks_oracle.c")


def build():
    """Compile the C part of the oracle (gcc, plain C11)."""
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", _LIB_PATH, _SRC])


def _load():
    alt = os.environ.get("ORACLE_LIB")  # another build of ckks_oracle.c (e.g. with sanitizers)
    if alt:
        lib = ctypes.CDLL(alt)
    else:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
    u64, i32, vp = ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p
    sig = {
        "or_mulmod": (u64, [u64, u64, u64]),
        "or_set_threads": (None, [i32]),
        "or_get_threads": (i32, []),
        "or_powmod": (u64, [u64, u64, u64]),
        "or_is_prime": (i32, [u64]),
        "or_gen_primes": (i32, [i32, i32, i32, vp, i32, vp]),
        "or_find_psi": (u64, [i32, u64]),
        "or_ntt_fwd": (None, [vp, i32, u64]),
        "or_ntt_inv": (None, [vp, i32, u64]),
        "or_polymul": (None, [vp, vp, vp, i32, u64]),
        "or_automorph": (None, [vp, vp, i32, u64, u64]),
        "or_monomial": (None, [vp, vp, i32, i32, u64]),
        "or_modup_digit": (None, [vp, i32, i32, vp, vp]),
        "or_modup": (None, [vp, i32, vp, vp]),
        "or_moddown": (None, [vp, i32, vp, vp]),
        "or_keyswitch_ext": (None, [vp, i32, vp, u64, vp, vp, vp]),
        "or_key_ip": (None, [vp, i32, vp, u64, vp, vp, vp]),
        "or_keyswitch": (None, [vp, i32, vp, vp, vp, vp]),
        "or_switch_key": (None, [vp, vp, vp, vp, vp, vp]),
        "or_rescale": (None, [vp, i32, vp, vp]),
        "or_modraise": (None, [vp, i32, vp, vp]),
        "or_encrypt_sk": (None, [vp, i32, vp, vp, vp, vp, vp]),
        "or_encrypt_pk": (None, [vp, i32, vp, vp, vp, vp, vp, vp]),
        "or_decrypt": (None, [vp, i32, vp, vp, vp]),
        "or_poly_pmult": (None, [vp, i32, vp, vp, vp]),
        "or_poly_automorph": (None, [vp, i32, vp, u64, vp]),
        "or_poly_monomial": (None, [vp, i32, vp, i32, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _u64(a):
    a = np.ascontiguousarray(a, dtype=np.uint64)
    return a


def _i64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


# ---------------------------------------------------------------- scalars

def gen_primes(log_n, bits, count, exclude=()):
    ex = _u64(np.array(list(exclude) or [0], dtype=np.uint64))
    out = np.zeros(count, dtype=np.uint64)
    got = lib.or_gen_primes(log_n, bits, count, _p(ex), len(exclude), _p(out))
    if got != count:
        raise ValueError("not enough primes")
    return [int(x) for x in out]


def set_threads(n):
    """threads of the C part's limb loops (n <= 0: every host core); results do not
    depend on it"""
    lib.or_set_threads(int(n))


def get_threads():
    return int(lib.or_get_threads())


def is_prime(n):
    return bool(lib.or_is_prime(int(n)))


def mulmod(a, b, q):
    return int(lib.or_mulmod(int(a), int(b), int(q)))


# ----------------------------------------------------------- one-limb ops

def ntt_fwd(a, q):
    a = _u64(a).copy()
    lib.or_ntt_fwd(_p(a), a.size, int(q))
    return a


def ntt_inv(a, q):
    a = _u64(a).copy()
    lib.or_ntt_inv(_p(a), a.size, int(q))
    return a


def polymul(a, b, q):
    a, b = _u64(a), _u64(b)
    c = np.empty_like(a)
    lib.or_polymul(_p(a), _p(b), _p(c), a.size, int(q))
    return c


def automorph(a, g, q):
    a = _u64(a)
    out = np.empty_like(a)
    lib.or_automorph(_p(a), _p(out), a.size, int(g), int(q))
    return out


def monomial(a, k, q):
    a = _u64(a)
    out = np.empty_like(a)
    lib.or_monomial(_p(a), _p(out), a.size, int(k) % (2 * a.size), int(q))
    return out


# ---------------------------------------------------------------- the ring

class _Ring(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("L", ctypes.c_int), ("alpha", ctypes.c_int),
                ("q", ctypes.c_void_p), ("p", ctypes.c_void_p)]


class Ring:
    """RNS ring: degree n, ciphertext primes q_0..q_L, special primes p_0..p_{alpha-1}."""

    def __init__(self, n, q, p):
        self.n = int(n)
        self.q = [int(x) for x in q]
        self.p = [int(x) for x in p]
        self.L = len(self.q) - 1
        self.alpha = len(self.p)
        self._qa = _u64(np.array(self.q, dtype=np.uint64))
        self._pa = _u64(np.array(self.p, dtype=np.uint64))
        self._s = _Ring(self.n, self.L, self.alpha, _p(self._qa), _p(self._pa))

    @property
    def ptr(self):
        return ctypes.byref(self._s)

    def n_digits(self, level):
        return -(-(level + 1) // self.alpha)

    def ext_primes(self, level):
        return self.q[:level + 1] + self.p

    def key_primes(self):
        return self.q + self.p

    # -- per-polynomial ops (arrays [(l+1)][n] of canonical residues)
    def modup(self, level, x):
        x = _u64(x)
        out = np.empty((self.n_digits(level), level + 1 + self.alpha, self.n), dtype=np.uint64)
        lib.or_modup(self.ptr, level, _p(x), _p(out))
        return out

    def modup_digit(self, level, j, x):
        x = _u64(x)
        out = np.empty((level + 1 + self.alpha, self.n), dtype=np.uint64)
        lib.or_modup_digit(self.ptr, level, j, _p(x), _p(out))
        return out

    def moddown(self, level, u):
        u = _u64(u)
        out = np.empty((level + 1, self.n), dtype=np.uint64)
        lib.or_moddown(self.ptr, level, _p(u), _p(out))
        return out

    def keyswitch(self, level, d, key):
        d, key = _u64(d), _u64(key)
        o0 = np.empty((level + 1, self.n), dtype=np.uint64)
        o1 = np.empty_like(o0)
        lib.or_keyswitch(self.ptr, level, _p(d), _p(key), _p(o0), _p(o1))
        return o0, o1

    def key_ip(self, level, ext, g, key):
        """key inner product over Q_l u P without ModDown: (u0, u1), each [l+1+alpha][n]"""
        ext, key = _u64(ext), _u64(key)
        u0 = np.empty((level + 1 + self.alpha, self.n), dtype=np.uint64)
        u1 = np.empty_like(u0)
        lib.or_key_ip(self.ptr, level, _p(ext), int(g), _p(key), _p(u0), _p(u1))
        return u0, u1

    def keyswitch_ext(self, level, ext, g, key):
        ext, key = _u64(ext), _u64(key)
        o0 = np.empty((level + 1, self.n), dtype=np.uint64)
        o1 = np.empty_like(o0)
        lib.or_keyswitch_ext(self.ptr, level, _p(ext), int(g), _p(key), _p(o0), _p(o1))
        return o0, o1

    def switch_key(self, s, sp, a, e):
        s, sp, a, e = _i64(s), _i64(sp), _u64(a), _i64(e)
        dn = self.n_digits(self.L)
        key = np.empty((dn, 2, self.L + 1 + self.alpha, self.n), dtype=np.uint64)
        lib.or_switch_key(self.ptr, _p(s), _p(sp), _p(a), _p(e), _p(key))
        return key

    def rescale(self, level, a):
        a = _u64(a)
        out = np.empty((level, self.n), dtype=np.uint64)
        lib.or_rescale(self.ptr, level, _p(a), _p(out))
        return out

    def modraise(self, a0, top=None):
        top = self.L if top is None else top
        a0 = _u64(a0)
        out = np.empty((top + 1, self.n), dtype=np.uint64)
        lib.or_modraise(self.ptr, top, _p(a0), _p(out))
        return out

    def encrypt_sk(self, level, s, m, a, e):
        s, m, a, e = _i64(s), _u64(m), _u64(a), _i64(e)
        ct = np.empty((2, level + 1, self.n), dtype=np.uint64)
        lib.or_encrypt_sk(self.ptr, level, _p(s), _p(m), _p(a), _p(e), _p(ct))
        return ct

    def gen_public_key(self, s, a, e):
        """pk = (-a s + e, a) over all L+1 ciphertext primes (Sec. 2.1): the secret-key
        encryption of zero at the top level"""
        return self.encrypt_sk(self.L, s, np.zeros((self.L + 1, self.n), dtype=np.uint64), a, e)

    def encrypt_pk(self, level, pk, m, v, e0, e1):
        """Enc(m; pk) at `level` (Sec. 2.1): (v pk0 + e0 + m, v pk1 + e1) on the first
        level+1 limbs of pk, for small v, e0, e1 (coefficient form throughout)"""
        pk, m, v, e0, e1 = _u64(pk), _u64(m), _i64(v), _i64(e0), _i64(e1)
        assert pk.shape == (2, self.L + 1, self.n)
        ct = np.empty((2, level + 1, self.n), dtype=np.uint64)
        lib.or_encrypt_pk(self.ptr, level, _p(pk), _p(m), _p(v), _p(e0), _p(e1), _p(ct))
        return ct

    def decrypt(self, level, s, ct):
        s, ct = _i64(s), _u64(ct)
        out = np.empty((level + 1, self.n), dtype=np.uint64)
        lib.or_decrypt(self.ptr, level, _p(s), _p(ct), _p(out))
        return out

    def pmult(self, level, a, pt):
        a, pt = _u64(a), _u64(pt)
        out = np.empty((level + 1, self.n), dtype=np.uint64)
        lib.or_poly_pmult(self.ptr, level, _p(a), _p(pt), _p(out))
        return out

    def poly_automorph(self, level, a, g):
        a = _u64(a)
        out = np.empty((level + 1, self.n), dtype=np.uint64)
        lib.or_poly_automorph(self.ptr, level, _p(a), int(g), _p(out))
        return out

    def poly_monomial(self, level, a, k):
        a = _u64(a)
        out = np.empty((level + 1, self.n), dtype=np.uint64)
        lib.or_poly_monomial(self.ptr, level, _p(a), int(k) % (2 * self.n), _p(out))
        return out

    def add(self, level, a, b):
        qs = np.array(self.q[:level + 1], dtype=np.uint64)[:, None]
        s = _u64(a) + _u64(b)
        return np.where(s >= qs, s - qs, s)

    def sub(self, level, a, b):
        qs = np.array(self.q[:level + 1], dtype=np.uint64)[:, None]
        a, b = _u64(a), _u64(b)
        return np.where(a >= b, a - b, a + (qs - b))

    def to_rns(self, coeffs, level):
        """signed integer coefficients (int64 array or Python ints) -> residues [(l+1)][n]"""
        c = np.asarray(coeffs)
        out = np.empty((level + 1, self.n), dtype=np.uint64)
        for i in range(level + 1):
            if c.dtype == object:
                out[i] = np.array([int(v) % self.q[i] for v in c], dtype=np.uint64)
            else:
                out[i] = np.mod(c.astype(np.int64), np.int64(self.q[i])).astype(np.uint64)
        return out


def centred_from_limbs(res, primes):
    """CRT of residues [(k)][n] over the given primes -> list of centred Python ints."""
    res = np.asarray(res)
    k = len(primes)
    Q = 1
    for q in primes:
        Q *= int(q)
    out = []
    hats = []
    for i in range(k):
        h = Q // int(primes[i])
        hats.append((h, h * pow(h % int(primes[i]), -1, int(primes[i]))))
    for c in range(res.shape[1]):
        x = 0
        for i in range(k):
            x += int(res[i, c]) * hats[i][1]
        x %= Q
        if x > Q // 2:
            x -= Q
        out.append(x)
    return out
