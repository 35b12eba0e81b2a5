"""Oracle of the downsampling flows' slot permutations (Sec. 5, Algorithm 2; Appendix B).

TEST INFRASTRUCTURE ONLY (see the package docstring).

A downsampling (stride-2) conv either
  * decomposes its input first (Algorithm 2): each input ciphertext's image is rearranged
    into its four phase images I_i[a::2, b::2], which a unit-stride conv then combines
    (the stride-2 conv = the sum over phases of unit-stride convs of the phase images), so
    only the dense outputs are bootstrapped; or
  * runs as a unit-stride conv whose sparse outputs are bootstrapped and then densified
    (the earlier flow the paper compares with): the even pixels of four sparse outputs
    are gathered into one dense ciphertext.
Both rearrangements are fixed permutations of slots, evaluated as BSGS matrix-vector
products with 0/1 diagonals (Sec. 2.6).  The paper describes its matrix G_l through a
figure that is missing; here the permutation is derived from the layouts:
  * after CoeffToSlot, real slot j holds coefficient rev(j) and imaginary slot j
    coefficient N/2 + rev(j) (bit reversal over log2(N/2) bits);
  * the fused conv's output holds pixel (y, x) of channel c at coefficient
    (y W + x) C + rev_C(c) (W^2 C = N);
  * decompose: (W, C) -> (W/2, 4C) with channel 4 i + 2 b + a = I_i[a::2, b::2];
  * densify: four (W, C) images -> (W/2, 4C) with channel 4 i + m = I^(m)_i[0::2, 0::2].
Neither moves a value between the real and imaginary halves, so each half is its own
permutation.
"""
import numpy as np

from .encoding import bitrev
from .plans import Bsgs, prerotate


def coeff_index(c, y, x, W, C):
    """coefficient of pixel (y, x) of channel c in the fused conv's output layout"""
    return (y * W + x) * C + bitrev(c, C)


def decompose_coeff_map(N, W, C):
    """src[k'] = the input coefficient that output coefficient k' takes"""
    W2, C2 = W // 2, 4 * C
    src = np.full(N, -1, dtype=np.int64)
    for i in range(C):
        for a in (0, 1):
            for b in (0, 1):
                for y in range(W2):
                    for x in range(W2):
                        src[coeff_index(4 * i + 2 * b + a, y, x, W2, C2)] = coeff_index(i, 2 * y + a, 2 * x + b, W, C)
    return src


def densify_coeff_map(N, W, C, m):
    """src[k'] for the coefficients input m provides (-1 elsewhere)"""
    W2, C2 = W // 2, 4 * C
    src = np.full(N, -1, dtype=np.int64)
    for i in range(C):
        for y in range(W2):
            for x in range(W2):
                src[coeff_index(4 * i + m, y, x, W2, C2)] = coeff_index(i, 2 * y, 2 * x, W, C)
    return src


def half_slot_map(src, N, half):
    """output slot j of the half -> input slot of the same half (-1: none)"""
    n = N // 2
    out = np.full(n, -1, dtype=np.int64)
    for j in range(n):
        k = src[half * n + bitrev(j, n)]
        if k < 0:
            continue
        if k // n != half:
            raise ValueError("a slot would move between the real and imaginary halves")
        out[j] = bitrev(int(k % n), n)
    return out


def perm_diagonals(slot_map):
    """{r: 0/1 vector v_r} with out = sum_r v_r (.) (x <<< r), out[j] = x[slot_map[j]]"""
    n = len(slot_map)
    diags = {}
    for j, s in enumerate(slot_map):
        if s < 0:
            continue
        r = int((s - j) % n)
        diags.setdefault(r, np.zeros(n))[j] = 1.0
    return diags


def apply_diagonals(diags, x):
    """plain evaluation of sum_r v_r (.) (x <<< r)"""
    out = np.zeros(len(x), dtype=np.result_type(x, float))
    for r, v in diags.items():
        out = out + v * np.roll(x, -r)
    return out


def decompose_plan(N, W, C, half, n1=None):
    """(Bsgs, {j: pre-rotated diagonal}) of the decomposition of one half"""
    d = perm_diagonals(half_slot_map(decompose_coeff_map(N, W, C), N, half))
    plan = Bsgs(N // 2, 1, d.keys(), n1)
    return plan, prerotate(plan, d)


def densify_plan(N, W, C, half, n1=None):
    """(Bsgs, {m: {j: pre-rotated diagonal}}): one BSGS structure (the union of the four
    inputs' offsets) with each input's diagonals"""
    per = [perm_diagonals(half_slot_map(densify_coeff_map(N, W, C, m), N, half)) for m in range(4)]
    plan = Bsgs(N // 2, 1, sorted({r for d in per for r in d}), n1)
    return plan, {m: prerotate(plan, d) for m, d in enumerate(per)}
