"""Pins of the oracle's FP64 encodings, DFT factorisation and plan builders.

Checked against: the O(N^2) matrix definitions, products of dense matrices,
the ring product (schoolbook negacyclic convolution), numpy's inverse, the
closed forms of Appendix A, and scipy's 2-D correlation for conv2d.
"""
import numpy as np
import pytest
from scipy.signal import correlate2d

import oracle.encoding as E
import oracle.plans as PL

RNG = np.random.default_rng(3)


def rz(n):
    return RNG.uniform(-1, 1, n) + 1j * RNG.uniform(-1, 1, n)


# ---------------------------------------------------------------- slot encoding

@pytest.mark.parametrize("N", [8, 64, 256])
def test_slot_encoding_matches_matrix_definition(N):
    z = rz(N // 2)
    assert np.allclose(E.slot_to_coeffs(z, N), E.slot_to_coeffs_direct(z, N), atol=1e-12)
    assert np.allclose(E.coeffs_to_slot(E.slot_to_coeffs(z, N), N), z, atol=1e-12)


def test_slot_encoding_is_multiplicative():
    """<z1> <z2> = <z1 (.) z2> in R[X]/(X^N+1) (Sec. 2.2)"""
    N = 64
    z1, z2 = rz(N // 2), rz(N // 2)
    f = E.negacyclic_conv(E.slot_to_coeffs(z1, N), E.slot_to_coeffs(z2, N))
    assert np.allclose(E.coeffs_to_slot(f, N), z1 * z2, atol=1e-12)


def test_slot_rotation_by_automorphism():
    """X -> X^(5^r) rotates the slots left by r"""
    N = 64
    z = rz(N // 2)
    f = E.slot_to_coeffs(z, N)
    for r in (1, 3, 17):
        g = pow(5, r, 2 * N)
        h = np.zeros(N)
        for i in range(N):
            e = i * g % (2 * N)
            if e < N:
                h[e] += f[i]
            else:
                h[e - N] -= f[i]
        assert np.allclose(E.coeffs_to_slot(h, N), np.roll(z, -r), atol=1e-12)


def test_encode_rounds_half_even_and_decodes():
    N = 128
    z = rz(N // 2)
    c = E.encode(z, N, 2.0 ** 40)
    assert c.dtype == np.int64
    assert np.allclose(E.decode(c, N, 2.0 ** 40), z, atol=1e-9)


def test_coefficient_encoding_slots():
    """<m>_coeff with coefficients (Re m | Im m) has slots T_{N/2} P m = V m (Sec. 2.4)"""
    N = 32
    m = rz(N // 2)
    f = np.concatenate([m.real, m.imag])
    assert np.allclose(E.coeffs_to_slot(f, N), E.V_matrix(N) @ m, atol=1e-12)


# --------------------------------------------------------------- DFT factors

@pytest.mark.parametrize("N", [16, 64])
def test_T_equals_V_P(N):
    n = N // 2
    assert np.allclose(E.T_matrix(n), E.V_matrix(N) @ E.P_matrix(n), atol=1e-12)


@pytest.mark.parametrize("n", [4, 16, 32])
def test_butterfly_factorisation(n):
    """T_n = S_{n/2} ... S_1 (Eq. decomp)"""
    M = np.eye(n)
    k = 1
    while k < n:
        M = E.S_stage_dense(k, n) @ M
        k *= 2
    assert np.allclose(M, E.T_matrix(n), atol=1e-10)


@pytest.mark.parametrize("n,k", [(16, 1), (16, 4), (16, 8), (32, 2)])
def test_stage_diagonals_and_butterflies(n, k):
    S = E.S_stage_dense(k, n)
    assert np.allclose(E.diagonals_to_dense(E.stage_diagonals(k, n), n), S)
    assert np.allclose(E.diagonals_to_dense(E.stage_diagonals(k, n, True), n), np.linalg.inv(S))
    x = rz(n)
    assert np.allclose(E.apply_stage(x, k), S @ x)
    assert np.allclose(E.apply_stage(x, k, inverse=True), np.linalg.solve(S, x))


def test_diagonal_composition_is_matrix_product():
    n = 16
    A = E.stage_diagonals(4, n)
    B = E.stage_diagonals(2, n, True)
    C = E.compose(A, B, n)
    assert np.allclose(E.diagonals_to_dense(C, n), E.diagonals_to_dense(A, n) @ E.diagonals_to_dense(B, n))


def test_partial_dft_theorem():
    """Thm 1: S_{l<-1} = blockdiag(T_l) (C copies)"""
    n, ell = 32, 8
    M = np.eye(n)
    k = 1
    while k < ell:
        M = E.S_stage_dense(k, n) @ M
        k *= 2
    assert np.allclose(M, np.kron(np.eye(n // ell), E.T_matrix(ell)), atol=1e-10)


# ---------------------------------------------------------------- real CinS

@pytest.mark.parametrize("ell", [4, 16, 64])
def test_dft_prime_definitions(ell):
    m = RNG.uniform(-1, 1, (3, 2 * ell))
    assert np.allclose(E.dft_prime(m, ell), E.dft_prime_direct(m, ell), atol=1e-10)
    # Appendix A: DFT'(m) = T_l P_l fold(m)
    TP = E.T_matrix(ell) @ E.P_matrix(ell)
    assert np.allclose(E.dft_prime(m, ell), (TP @ E.fold(m, ell).T).T, atol=1e-10)


def test_real_dft_convolution_theorem():
    """Appendix A: DFT'(x) (.) DFT'(y) = DFT'(x *_{2l} y)"""
    ell = 8
    x, y = RNG.uniform(-1, 1, 2 * ell), RNG.uniform(-1, 1, 2 * ell)
    assert np.allclose(E.dft_prime(x, ell) * E.dft_prime(y, ell), E.dft_prime(E.negacyclic_conv(x, y), ell))


def test_cins_product_is_local_convolution():
    """Eq. nested_real_vector2 / Thm 3: <m>_CinS <m'>_CinS = <m *_local m'>_CinS in the ring"""
    N, ell = 64, 8
    C = N // (2 * ell)
    m, mp = RNG.uniform(-1, 1, (C, 2 * ell)), RNG.uniform(-1, 1, (C, 2 * ell))
    f = E.slot_to_coeffs(E.real_cins_slots(m, ell), N)
    fp = E.slot_to_coeffs(E.real_cins_slots(mp, ell), N)
    prod = E.negacyclic_conv(f, fp)
    local = np.stack([E.negacyclic_conv(m[c], mp[c]) for c in range(C)])
    assert np.allclose(prod, E.slot_to_coeffs(E.real_cins_slots(local, ell), N), atol=1e-10)


def test_slice_rotation():
    """Sec. 3.2.2: HRot by k l slots cycles the slices"""
    N, ell = 64, 8
    C = N // (2 * ell)
    m = RNG.uniform(-1, 1, (C, 2 * ell))
    z = E.real_cins_slots(m, ell)
    assert np.allclose(E.rotl(z, 2 * ell), E.real_cins_slots(np.roll(m, -2, axis=0), ell))


def test_stoc2_output_layout():
    """S_{N/2<-l} applied to real-CinS slots gives coefficient layout a[k C + rev_C(c)] = m_c[k]"""
    N, ell = 128, 8
    n = N // 2
    C = n // ell
    m = RNG.uniform(-1, 1, (C, 2 * ell))
    z = E.real_cins_slots(m, ell)
    k = ell
    while k < n:
        z = E.apply_stage(z, k)
        k *= 2
    f = E.slot_to_coeffs(z, N)
    want = np.zeros(N)
    for c in range(C):
        for j in range(2 * ell):
            want[j * C + E.bitrev(c, C)] = m[c, j]
    assert np.allclose(f, want, atol=1e-10)


# ------------------------------------------------------------------- conv plan

def test_conv2d_same_matches_scipy():
    img = RNG.uniform(-1, 1, (3, 7, 7))
    K = RNG.uniform(-1, 1, (2, 3, 3, 3))
    out = PL.conv2d_same(img, K)
    for o in range(2):
        want = sum(correlate2d(img[i], K[o, i], mode="same") for i in range(3))
        assert np.allclose(out[o], want)


@pytest.mark.parametrize("w0,f", [(5, 3), (6, 3), (4, 1), (7, 5)])
def test_kernel_polynomial_gives_conv(w0, f):
    """Fig. 1: zero-pad, flatten, negacyclic-convolve; valid outputs are the conv2d"""
    W = PL.padded_width(w0, f)
    img = RNG.uniform(-1, 1, (1, w0, w0))
    K = RNG.uniform(-1, 1, (1, 1, f, f))
    i = PL.image_to_slices(img, W)[0]
    o = E.negacyclic_conv(i, PL.kernel_poly(K[0, 0], W)).reshape(W, W)[:w0, :w0]
    assert np.allclose(o, PL.conv2d_same(img, K)[0])


def simulate_bsgs(plan, diags, z):
    """sum_g ( sum_i d'_{g n1+i} (.) (z <<< i u) ) <<< g n1 u  in FP64 slots"""
    out = 0
    for g in plan.giants:
        inner = 0
        for j, (gg, i) in plan.split.items():
            if gg == g:
                inner = inner + diags[j] * E.rotl(z, plan.baby_rot(i))
        out = out + E.rotl(inner, plan.giant_rot(g))
    return out


@pytest.mark.parametrize("N,w0,C", [(64, 3, 4), (256, 6, 4), (512, 5, 8), (1024, 7, 16)])
def test_fused_conv_diagonals_give_conv2d(N, w0, C):
    """BSGS with K^' = S'K^ diagonals on real-CinS input = conv2d in coefficient layout"""
    f = 3
    W = PL.padded_width(w0, f)
    assert N // (W * W) == C
    ell = W * W // 2
    img = RNG.uniform(-1, 1, (C, w0, w0))
    K = RNG.uniform(-1, 1, (C, C, f, f))
    plan, diags = PL.conv_plan(K, W, N)
    assert len(diags) == C  # Table 1: C plaintexts
    if int(np.sqrt(C)) ** 2 == C:
        assert len(plan.rotations()) == 2 * int(np.sqrt(C)) - 2  # Table 1: 2 sqrt(C) - 2 HRot
    z = E.real_cins_slots(PL.image_to_slices(img, W), ell)
    coeffs = E.slot_to_coeffs(simulate_bsgs(plan, diags, z), N)
    want = PL.conv2d_same(img, K)
    for c in range(C):
        got = np.array([coeffs[(y * W + x) * C + E.bitrev(c, C)] for y in range(w0) for x in range(w0)])
        assert np.allclose(got, want[c].reshape(-1), atol=1e-9)


@pytest.mark.parametrize("N,d", [(64, 2), (256, 3), (128, 1)])
def test_cts_groups_compose_to_inverse_dft(N, d):
    n = N // 2
    groups = PL.cts_plan(N, d)
    M = np.eye(n)
    for plan, diags in groups:
        # undo the BSGS pre-rotation to recover the group's matrix
        D = {}
        for j, v in diags.items():
            g, _ = plan.split[j]
            D[(j * plan.u) % n] = E.rotl(v, g * plan.n1 * plan.u)
        M = E.diagonals_to_dense(D, n) @ M
        # BSGS evaluation equals the dense product
        x = rz(n)
        assert np.allclose(simulate_bsgs(plan, diags, x), E.diagonals_to_dense(D, n) @ x)
    assert np.allclose(2 * M, np.linalg.inv(E.T_matrix(n)), atol=1e-10)


def test_cts_diagonal_counts():
    """structural diagonal counts: N=2^16 d=3 -> 32/63/63, N=2^12 d=2 -> 64/63"""
    assert [len(g) for g in PL.cts_stage_groups(2 ** 15, 3)] == [5, 5, 5]
    assert [len(g) for g in PL.cts_stage_groups(2 ** 11, 2)] == [6, 5]
    small = PL.cts_plan(2 ** 12, 2)
    assert [len(d) for _, d in small] == [64, 63]
    rot = [len(p.rotations()) for p, _ in small]
    assert rot == [14, 14]
