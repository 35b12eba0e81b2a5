"""Oracle FP64 encodings and DFT factor matrices (numpy, float64 / complex128).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Definitions followed (NeuJeans, arXiv 2312.04356):
  * Slot encoding, Sec. 2.2: zeta = exp(pi i / N), zeta_j = zeta^(5^j), 0 <= j < N/2;
    f = (1/N)(conj(U)^T z + U^T conj(z)), U[j][i] = zeta_j^i.  Decoding evaluates f at zeta_j.
  * Bit-reversed DFT matrix and its butterfly factorisation, Sec. 2.3 (Eq. decomp):
    T_n[i][j] = w_{4n}^(5^i rev_n(j)),  T_{N/2} = V P,  T_n = S_{n/2} ... S_1,
    S_k = blockdiag(B_k),  B_k = [[I, W_k], [I, -W_k]],  W_k = diag(w_{8k}^(5^i)), i < k.
  * Real CinS encoding, Sec. 3.3.1 and Appendix A:
    (DFT'_{2l} m)_j = sum_{k < 2l} m_k w_{4l}^(5^j k),  <m>_CinS = <(DFT'(m_1) | ... | DFT'(m_C))>_slot.
  * Matrix-vector products by cyclic diagonals, Sec. 2.6 (Eq. matvecmul):
    M x = sum_r diag(v_r) (x <<< r),  (x <<< r)[i] = x[(i + r) mod n].
"""
import numpy as np


def omega(m):
    """primitive m-th root of unity exp(2 pi i / m)"""
    return np.exp(2j * np.pi / m)


def rot5(count, modulus):
    """[5^j mod modulus for j < count]"""
    out = np.empty(count, dtype=np.int64)
    v = 1
    for j in range(count):
        out[j] = v
        v = v * 5 % modulus
    return out


def bitrev(j, n):
    bits = n.bit_length() - 1
    r = 0
    for _ in range(bits):
        r = (r << 1) | (j & 1)
        j >>= 1
    return r


# ------------------------------------------------------------------ slot encoding

def slot_to_coeffs(z, N):
    """f = (1/N)(conj(U)^T z + U^T conj(z)) via one length-2N FFT (library primitive as a step).

    FFT_{2N}(Z)[i] = sum_k Z[k] zeta^(-k i), with Z[5^j] = z_j and Z[-5^j] = conj(z_j).
    """
    z = np.asarray(z, dtype=np.complex128)
    assert z.shape == (N // 2,)
    e = rot5(N // 2, 2 * N)
    Z = np.zeros(2 * N, dtype=np.complex128)
    Z[e] = z
    Z[(2 * N - e) % (2 * N)] = np.conj(z)
    return np.real(np.fft.fft(Z)[:N]) / N


def slot_to_coeffs_direct(z, N):
    """The same map written as the matrix products of the definition (O(N^2); small N only)."""
    z = np.asarray(z, dtype=np.complex128)
    zeta = omega(2 * N)
    e = rot5(N // 2, 2 * N)
    U = zeta ** (np.outer(e, np.arange(N)) % (2 * N))
    f = (np.conj(U).T @ z + U.T @ np.conj(z)) / N
    return np.real(f)


def coeffs_to_slot(f, N):
    """z_j = f(zeta_j) = sum_i f_i zeta^(5^j i), via an inverse FFT of length 2N."""
    f = np.asarray(f, dtype=np.float64)
    F = np.fft.ifft(np.concatenate([f, np.zeros(N)])) * (2 * N)
    return F[rot5(N // 2, 2 * N)]


def encode(z, N, scale):
    """integer coefficients round_half_even(scale * f) as int64"""
    return np.rint(scale * slot_to_coeffs(z, N)).astype(np.int64)


def decode(coeffs, N, scale):
    return coeffs_to_slot(np.asarray(coeffs, dtype=np.float64) / scale, N)


# ------------------------------------------------------------------ DFT matrices

def V_matrix(N):
    e = rot5(N // 2, 2 * N)
    return omega(2 * N) ** (np.outer(e, np.arange(N // 2)) % (2 * N))


def P_matrix(n):
    P = np.zeros((n, n))
    for j in range(n):
        P[bitrev(j, n), j] = 1.0
    return P


def T_matrix(n):
    e = rot5(n, 4 * n)
    r = np.array([bitrev(j, n) for j in range(n)])
    return omega(4 * n) ** (np.outer(e, r) % (4 * n))


def W_diag(k):
    """diagonal of W_k: w_{8k}^(5^i), i < k"""
    return omega(8 * k) ** (rot5(k, 8 * k))


def B_block(k):
    W = np.diag(W_diag(k))
    I = np.eye(k)
    return np.block([[I, W], [I, -W]])


def S_stage_dense(k, n):
    return np.kron(np.eye(n // (2 * k)), B_block(k))


def apply_stage(x, k, inverse=False):
    """y = S_k x (or S_k^{-1} x) for a vector whose length is a multiple of 2k (butterflies)."""
    x = np.asarray(x, dtype=np.complex128)
    n = x.shape[-1]
    y = x.reshape(x.shape[:-1] + (n // (2 * k), 2, k))
    a, b = y[..., 0, :], y[..., 1, :]
    w = W_diag(k)
    if not inverse:
        out = np.stack([a + w * b, a - w * b], axis=-2)
    else:
        out = np.stack([0.5 * (a + b), 0.5 * (a - b) / w], axis=-2)
    return out.reshape(x.shape)


# --------------------------------------------------- cyclic-diagonal representation

def rotl(x, r):
    """(x <<< r)[i] = x[(i + r) mod n]"""
    return np.roll(x, -int(r), axis=-1)


def rotr(x, r):
    return np.roll(x, int(r), axis=-1)


def stage_diagonals(k, n, inverse=False):
    """{r: v_r} with S_k (or S_k^{-1}) = sum_r diag(v_r) (. <<< r), n-dimensional."""
    t = np.arange(n) % (2 * k)
    lo = t < k
    w = W_diag(k)
    wt = np.where(lo, 0, t - k)
    if not inverse:
        v0 = np.where(lo, 1.0 + 0j, -w[wt])
        vp = np.where(lo, w[np.minimum(t, k - 1)], 0)
        vm = np.where(lo, 0, 1.0 + 0j)
    else:
        v0 = np.where(lo, 0.5 + 0j, -0.5 / w[wt])
        vp = np.where(lo, 0.5 + 0j, 0)
        vm = np.where(lo, 0, 0.5 / w[wt])
    D = {}
    for r, v in ((0, v0), (k % n, vp), ((-k) % n, vm)):
        D[r] = D.get(r, 0) + v.astype(np.complex128)
    return D


def compose(A, B, n):
    """diagonals of A @ B: diag(a_r)(.<<<r) diag(b_s)(.<<<s) = diag(a_r * (b_s <<< r))(.<<<(r+s))"""
    C = {}
    for r, a in A.items():
        for s, b in B.items():
            t = (r + s) % n
            C[t] = C.get(t, 0) + a * rotl(b, r)
    return C


def apply_diagonals(D, x):
    return sum(v * rotl(x, r) for r, v in D.items())


def diagonals_to_dense(D, n):
    M = np.zeros((n, n), dtype=np.complex128)
    rows = np.arange(n)
    for r, v in D.items():
        M[rows, (rows + r) % n] += v
    return M


# --------------------------------------------------------------- real CinS

def dft_prime(m, ell):
    """(DFT'_{2l} m)_j = sum_{k<2l} m_k w_{4l}^(5^j k), j < l; via an inverse FFT of length 4l."""
    m = np.asarray(m, dtype=np.float64)
    assert m.shape[-1] == 2 * ell
    pad = np.zeros(m.shape[:-1] + (4 * ell,))
    pad[..., :2 * ell] = m
    F = np.fft.ifft(pad, axis=-1) * (4 * ell)
    return F[..., rot5(ell, 4 * ell)]


def dft_prime_direct(m, ell):
    m = np.asarray(m, dtype=np.float64)
    e = rot5(ell, 4 * ell)
    M = omega(4 * ell) ** (np.outer(e, np.arange(2 * ell)) % (4 * ell))
    return m @ M.T


def real_cins_slots(chans, ell):
    """chans: (C, 2l) real slices -> slot vector (DFT'(m_1) | ... | DFT'(m_C)) of length C*l"""
    return dft_prime(chans, ell).reshape(-1)


def fold(m, ell):
    """folded vector: m_i + sqrt(-1) m_{i+l}"""
    return m[..., :ell] + 1j * m[..., ell:]


def negacyclic_conv(x, y):
    """x *_n y in R[Y]/(Y^n + 1), schoolbook"""
    n = len(x)
    out = np.zeros(n)
    for i in range(n):
        for j in range(n):
            k = i + j
            if k < n:
                out[k] += x[i] * y[j]
            else:
                out[k - n] -= x[i] * y[j]
    return out
