"""Seeded synthetic inputs shared by the HIP path's tests/bench and the oracle.

This module holds random numbers and workload shapes only: no encoding, no
modular arithmetic of the method, nothing either side computes.  Every array
it returns is drawn from numpy's Philox counter-based generator (Salmon et al.,
"Parallel random numbers: as easy as 1, 2, 3", SC'11) keyed by an explicit
seed and a purpose number, so both sides receive identical inputs.

Purposes (the second key word):
  0 secret key        1 key-switching uniforms   2 key-switching errors
  3 encryption uniforms  4 encryption errors    5 image / weight data
  6 job mix          7 public-key uniforms   8 public-key error
  9 public-key encryption: v, e0, e1
"""
import numpy as np

(PURPOSE_SECRET, PURPOSE_KEY_A, PURPOSE_KEY_E, PURPOSE_ENC_A, PURPOSE_ENC_E, PURPOSE_DATA, PURPOSE_JOBS,
 PURPOSE_PK_A, PURPOSE_PK_E, PURPOSE_PK_ENC) = range(10)


def _gen(seed, purpose, sub=0):
    return np.random.Generator(np.random.Philox(key=[int(seed) & (2**64 - 1),
                                                     (int(purpose) << 32) | (int(sub) & 0xFFFFFFFF)]))


def uniform_residues(primes, n, seed, purpose, sub=0):
    """[len(primes)][n] uint64, row r uniform on [0, primes[r]) (rejection sampling)."""
    g = _gen(seed, purpose, sub)
    out = np.empty((len(primes), n), dtype=np.uint64)
    for r, q in enumerate(primes):
        q = int(q)
        bits = q.bit_length()
        mask = np.uint64((1 << bits) - 1)
        filled = 0
        row = out[r]
        while filled < n:
            need = n - filled
            cand = g.integers(0, 2**64 - 1, size=need + need // 8 + 16, dtype=np.uint64, endpoint=True) & mask
            cand = cand[cand < np.uint64(q)][:need]
            row[filled:filled + cand.size] = cand
            filled += cand.size
    return out


def ternary_secret(n, h, seed):
    """int8[n] with exactly h nonzero entries, each +1 or -1."""
    g = _gen(seed, PURPOSE_SECRET)
    pos = g.choice(n, size=h, replace=False)
    sgn = g.integers(0, 2, size=h) * 2 - 1
    s = np.zeros(n, dtype=np.int8)
    s[pos] = sgn
    return s


def cbd_error(n, seed, purpose, sub=0, eta=21):
    """int64[n]: centred binomial, popcount(eta bits) - popcount(eta bits); sigma = sqrt(eta/2)."""
    g = _gen(seed, purpose, sub)
    a = g.integers(0, 2, size=(n, eta), dtype=np.int8).sum(axis=1, dtype=np.int64)
    b = g.integers(0, 2, size=(n, eta), dtype=np.int8).sum(axis=1, dtype=np.int64)
    return a - b


def uniform_real(shape, seed, sub=0, lo=-1.0, hi=1.0):
    """float64 array of the given shape, U(lo, hi)."""
    g = _gen(seed, PURPOSE_DATA, sub)
    return g.uniform(lo, hi, size=shape)


# Workload shapes (conv layer and ring) used by tests and the benchmark.
WORKLOADS = {
    # N=2^12, 8 ciphertext primes + 2 special, one 3x3 conv 4->4 on 16x16, two CoeffToSlot levels
    "small": dict(log_n=12, n_q=8, alpha=2, q0_bits=50, q_bits=48, p_bits=50, log_scale=40, h=192,
                  c_in=4, c_out=4, w0=16, f=3, cts_groups=2, data_seed=1001, key_seed=2001),
    # N=2^16, 24 ciphertext primes + 8 special (three key-switching digits), 3x3 conv 16->16 on 32x32
    "full": dict(log_n=16, n_q=24, alpha=8, q0_bits=50, q_bits=48, p_bits=50, log_scale=40, h=192,
                 c_in=16, c_out=16, w0=32, f=3, cts_groups=3, data_seed=1002, key_seed=2002),
}


def key_randomness(primes, n, dnum, seed, key_id):
    """uniform a: [dnum][len(primes)][n] uint64 and errors e: [dnum][n] int64 for one switching key"""
    a = np.stack([uniform_residues(primes, n, seed, PURPOSE_KEY_A, int(key_id) * 64 + j) for j in range(dnum)])
    e = np.stack([cbd_error(n, seed, PURPOSE_KEY_E, int(key_id) * 64 + j) for j in range(dnum)])
    return a, e


def enc_randomness(primes, n, seed, sub=0):
    """uniform a: [len(primes)][n] uint64 and error e: [n] int64 for one secret-key encryption"""
    return uniform_residues(primes, n, seed, PURPOSE_ENC_A, sub), cbd_error(n, seed, PURPOSE_ENC_E, sub)


def pk_randomness(primes, n, seed):
    """uniform a: [len(primes)][n] uint64 and error e: [n] int64 of a public key"""
    return uniform_residues(primes, n, seed, PURPOSE_PK_A), cbd_error(n, seed, PURPOSE_PK_E)


def pk_enc_randomness(n, seed, sub=0, h=64):
    """(v, e0, e1) of one public-key encryption: v int64[n] ternary with h nonzero
    entries, e0 and e1 int64[n] centred binomial"""
    g = _gen(seed, PURPOSE_PK_ENC, 3 * int(sub))
    pos = g.choice(n, size=h, replace=False)
    v = np.zeros(n, dtype=np.int64)
    v[pos] = g.integers(0, 2, size=h) * 2 - 1
    return v, cbd_error(n, seed, PURPOSE_PK_ENC, 3 * int(sub) + 1), cbd_error(n, seed, PURPOSE_PK_ENC, 3 * int(sub) + 2)


RELIN_KEY_ID = 0  # Galois elements are odd, so 0 never collides


JOB_OPS = ("3x3", "3x3s2", "1x1", "dw3x3")
JOB_CHANNELS = {16: 56, 64: 28, 256: 14}  # channels per ciphertext -> image width (W = 64, 32, 16)


def job_mix(n, seed=1004, lo=7, hi=23):
    """n jobs (op, C, level): op uniform over JOB_OPS, C uniform over JOB_CHANNELS,
    level uniform on lo..hi"""
    g = _gen(seed, PURPOSE_JOBS)
    ops = g.integers(0, len(JOB_OPS), n)
    cs = g.integers(0, len(JOB_CHANNELS), n)
    lv = g.integers(lo, hi + 1, n)
    keys = sorted(JOB_CHANNELS)
    return [(JOB_OPS[o], keys[c], int(l)) for o, c, l in zip(ops, cs, lv)]
