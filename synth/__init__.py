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
import json
import os

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


# Parameter sets of the workloads, one JSON file each under synth/params/ (ring, chain,
# layer shape, seeds): small, full, larger, batched, plans.  WORKLOADS holds the two that
# tests and the benchmark build as a ring plus one conv layer.
_PARAMS_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "params")


def params(name):
    """the parameter set synth/params/<name>.json"""
    with open(os.path.join(_PARAMS_DIR, name + ".json")) as fh:
        doc = json.load(fh)
    doc.pop("description", None)
    return doc


WORKLOADS = {name: params(name) for name in ("small", "full")}


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
