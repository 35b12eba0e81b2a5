"""Values the paper prints: Table 1 (CinS conv op counts) and Table 5 (ciphertext sizes)."""
import json
import math
import os

import numpy as np
import pytest

import oracle.plans as PL

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def load(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


@pytest.mark.parametrize("log_n,w0", [(10, 7), (12, 16), (14, 16), (16, 32), (16, 16)])
def test_table1_conv_counts(log_n, w0):
    t = load("table1_cins_opcounts.json")["conv2d"]
    N = 1 << log_n
    W = PL.padded_width(w0, 3)
    C = N // (W * W)
    K = np.zeros((C, C, 3, 3))
    plan, diags = PL.conv_plan(K, W, N)
    env = {"C": C, "sqrt": math.sqrt}
    assert len(diags) == eval(t["pmult"], env) == eval(t["plaintexts"], env)
    if math.isqrt(C) ** 2 == C:
        assert len(plan.rotations()) == eval(t["hrot"], env)


def test_table5_ciphertext_sizes():
    t = load("table5_ct_sizes.json")
    N = 1 << t["log_n"]
    MiB = 2 ** 20
    # decryption: one level-0 ciphertext, 2 polynomials x 1 limb x N words of 8 bytes
    assert round(2 * 1 * N * 8 / MiB) == t["decryption_MB"]
    # encryption: real CinS input encrypted at level 1 (2 limbs)
    c, w, _ = t["input_image"]
    W = PL.padded_width(w, 3)
    per_ct = N // (W * W)
    n_ct = -(-c // per_ct)
    assert round(n_ct * 2 * 2 * N * 8 / MiB) == t["encryption_real_cins_MB"]
    # complex CinS packs N/2 values per ciphertext: twice the ciphertexts
    assert round(2 * n_ct * 2 * 2 * N * 8 / MiB) == t["encryption_complex_cins_MB"]
