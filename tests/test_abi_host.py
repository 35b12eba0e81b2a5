"""Host-side checks of the HIP library that need no GPU: exported symbols, the prime
chain, argument validation, and the library's FP64 encoder against the oracle's."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle as O
import oracle.encoding as E
import oracle.plans as PL
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "neujeans.h")

nj = pytest.importorskip("paper_2312_04356_amd")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(nj_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 30
    lib = ctypes.CDLL(nj.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(nj.EXPORTED), set(names) ^ set(nj.EXPORTED)


@pytest.mark.parametrize("name", ["small", "full"])
def test_prime_chain_matches_oracle(name):
    w = synth.WORKLOADS[name]
    got = nj.chain_primes(w["log_n"], w["n_q"], w["alpha"], w["q0_bits"], w["q_bits"], w["p_bits"])
    want = PL.chain_primes(w["log_n"], w["n_q"], w["alpha"], w["q0_bits"], w["q_bits"], w["p_bits"],
                           lambda ln, b, c, ex: O.gen_primes(ln, b, c, ex))
    assert got == want
    q, p = got
    assert all(x < 2 ** 50 for x in q + p) and len(set(q + p)) == len(q + p)


def test_gen_primes_rejects_bad_arguments():
    with pytest.raises(nj.NjError):
        nj.nj_gen_primes(12, 51, 1)
    with pytest.raises(nj.NjError):
        nj.nj_gen_primes(16, 20, 10 ** 6)


@pytest.mark.parametrize("log_n", [10, 12, 16])
def test_encoder_agrees_with_oracle_to_one_unit(log_n):
    N = 1 << log_n
    rng = np.random.default_rng(log_n)
    z = rng.uniform(-1, 1, N // 2) + 1j * rng.uniform(-1, 1, N // 2)
    scale = 2.0 ** 40
    mine = nj.nj_encode_slots(log_n, z, scale)
    theirs = E.encode(z, N, scale)
    diff = np.abs(mine - theirs)
    assert diff.max() <= 1
    assert np.count_nonzero(diff) <= N // 100
    back = nj.nj_decode_slots(log_n, mine.astype(np.float64), scale)
    assert np.max(np.abs(back - z)) < 1e-9


def test_real_cins_encoder_agrees_with_oracle():
    log_n, ell = 12, 512
    N = 1 << log_n
    C = N // (2 * ell)
    chans = np.random.default_rng(1).uniform(-1, 1, (C, 2 * ell))
    mine = nj.nj_encode_cins(log_n, chans, 2.0 ** 40)
    theirs = E.encode(E.real_cins_slots(chans, ell), N, 2.0 ** 40)
    assert np.abs(mine - theirs).max() <= 1


def test_encoder_rejects_bad_slice():
    with pytest.raises(nj.NjError):
        nj.nj_encode_cins(12, np.zeros((3, 100)), 1.0)


@pytest.mark.parametrize("log_n,W,C,w0", [(12, 32, 4, 16), (16, 64, 16, 32), (11, 16, 8, 12)])
def test_layer_masks_match_oracle(log_n, W, C, w0):
    """the library's zero-padding masks (host) against the oracle's"""
    import oracle.bootstrap as B
    got = nj.nj_layer_masks(log_n, W, C, w0)
    want = B.layer_masks(1 << log_n, W, C, w0)
    assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])


def _create_status(log_n, n_q, alpha):
    """status of nj_ctx_create for n_q + alpha primes of the chain rule (no GPU call is
    reached when the parameters are refused)"""
    q = nj.nj_gen_primes(log_n, 49, n_q)
    p = nj.nj_gen_primes(log_n, 49, alpha, q)
    qa, pa = np.array(q, dtype=np.uint64), np.array(p, dtype=np.uint64)
    prm = nj.NjParams(log_n, n_q, alpha, qa.ctypes.data, pa.ctypes.data, 2.0 ** 40)
    h = ctypes.c_void_p()
    return nj._lib.nj_ctx_create(ctypes.byref(prm), ctypes.byref(h))


@pytest.mark.parametrize("n_q,alpha", [(64, 8), (33, 16), (32, 2), (17, 1)])
def test_ctx_create_refuses_oversized_bases(n_q, alpha):
    """more ciphertext primes than the basis-conversion tables hold (n_q > 32), or more
    than 8 key-switching digits, is refused with NJ_EUNSUPPORTED before any device work"""
    assert _create_status(12, n_q, alpha) == -7
    assert "nj_ctx_create" in nj._lib.nj_last_error().decode()


def test_plan_model_file_is_complete():
    """the committed latency model (written by paper_2312_04356_amd/tune.py): parameters and
    standardisation of the 7-64-64-1 network, the feature names, the held-out error"""
    import json
    doc = json.load(open(os.path.join(ROOT, "paper_2312_04356_amd", "data", "plan_model_n65536.json")))
    assert len(doc["params"]) == nj.MLP_PARAMS and len(doc["norm"]) == nj.MLP_NORM
    assert len(doc["features"]) == nj.MLP_FEATURES
    assert all(v > 0 for v in doc["norm"][7:14]) and doc["n_timings"] >= 4500
    assert doc["heldout_rel_err"]["cts_d_not_3"]["n"] > 0


@pytest.mark.parametrize("stride,depthwise,f", [(1, False, 3), (1, False, 1), (2, False, 3), (2, False, 7),
                                                (2, False, 1), (1, True, 3)])
def test_library_conv_taps_match_oracle(stride, depthwise, f):
    """the library's tap decomposition of conv layers (stride 1, stride 2 on the phase
    layout, depthwise) equals the oracle's, which its CPU tests pin to FP64 convolution"""
    rng = np.random.default_rng(f * 10 + stride)
    K = rng.uniform(-1, 1, (3, f, f) if depthwise else (5, 3, f, f))
    got = sorted(nj.nj_conv_taps(K, stride, depthwise))
    if depthwise:
        want = PL.taps_depthwise(K)
    else:
        want = PL.taps_stride2(K) if stride == 2 else PL.taps_same(K)
    assert got == sorted(want)


def test_library_conv_taps_reject_bad_shapes():
    with pytest.raises(nj.NjError):
        nj.nj_conv_taps(np.zeros((2, 2, 2, 2)))  # even kernel
    with pytest.raises(nj.NjError):
        nj.nj_conv_taps(np.zeros((2, 2, 3, 3)), stride=3)
