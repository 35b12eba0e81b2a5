"""Oracle of the classifier head: the fully connected layer fused with the whole StoC
(Sec. 4.2.1) and average pooling as a depthwise conv (Sec. 3.3.5).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 4.2.1: slot encoding is CinS encoding with slices of length 1, so a fully connected
layer y = W x fuses with the entire StoC the way a conv fuses with StoC2.  Reading used
here: the features x (n_in of them) sit in the slots of a sparsely packed plaintext with
period n' (the smallest power of two >= n_in, n_out): the polynomial is g(X^{N/N'}),
N' = 2 n', whose slot j is z_j = g(zeta'^(5^j)), zeta' = exp(pi i / N'), j mod n'.
The fused matrix M' = V' E W S maps the n' slots so that the result's coefficients
g_k = y_k (k < n_out): V'[j][k] = zeta'^(5^j k) (the decoding of g's first n'
coefficients), E puts y there, S selects the first n_in slots.  As a transform on all N/2
slots it has the n' cyclic diagonals of M' repeated with period n'.

Average pooling (Sec. 3.3.5) is a depthwise conv whose kernels are the same for every
channel: k x k stride 2 with weights 1/k^2 on the phase images (Algorithm 2), and the
global average over a w x w image the 'same' depthwise w x w conv of weights 1/w^2 read
at the centre pixel.
"""
import numpy as np

from .encoding import omega, rot5
from .plans import Bsgs, prerotate


def period(n_in, n_out):
    p = 1
    while p < max(n_in, n_out):
        p *= 2
    return p


def fc_matrix(n_in, n_out, W):
    """M' (n' x n'), from the definition of the subring's decoding"""
    npp = period(n_in, n_out)
    e = rot5(npp, 4 * npp)
    V = omega(4 * npp) ** (np.outer(e, np.arange(n_out)) % (4 * npp))  # slots of coefficients 0..n_out-1
    M = np.zeros((npp, npp), dtype=np.complex128)
    M[:, :n_in] = V @ np.asarray(W, dtype=np.float64)
    return M


def fc_diagonals(N, n_in, n_out, W):
    """{r: length-N/2 diagonal} for r < n': v_r[j] = M'[j mod n'][(j + r) mod n']"""
    M = fc_matrix(n_in, n_out, W)
    npp, n = M.shape[0], N // 2
    rows = np.arange(n) % npp
    return {r: M[rows, (rows + r) % npp] for r in range(npp)}


def fc_plan(N, n_in, n_out, W, n1=None):
    d = fc_diagonals(N, n_in, n_out, W)
    plan = Bsgs(N // 2, 1, d.keys(), n1)
    return plan, prerotate(plan, d)


def periodic_slots(x, n_in, n_out, N):
    """the input slot vector: x in the first n_in slots of every period n'"""
    npp = period(n_in, n_out)
    z = np.zeros(npp, dtype=np.complex128)
    z[:n_in] = x
    return np.tile(z, (N // 2) // npp)


def avg_pool(img, k, stride):
    """plain FP64 average pooling, padding (k-1)/2 counted as zeros"""
    C, w, _ = img.shape
    p = (k - 1) // 2
    pad = np.zeros((C, w + 2 * p, w + 2 * p))
    pad[:, p:p + w, p:p + w] = img
    wo = (w + 2 * p - k) // stride + 1
    out = np.zeros((C, wo, wo))
    for u in range(k):
        for v in range(k):
            out += pad[:, u:u + stride * wo:stride, v:v + stride * wo:stride]
    return out / (k * k)
