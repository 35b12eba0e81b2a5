"""Oracle of the bootstrapping steps after CoeffToSlot: ModEval (modular reduction by a
Chebyshev interpolant and double angles) and StoC1 (the first log2(l) butterfly stages
of the DFT, S_{l <- 1}), plus the homomorphic multiplication they need.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 2.4 (bootstrapping): after ModRaise and CoeffToSlot the slots hold
t = m + (q_0 / Delta) I with a small integer vector I; ModEval recovers m.  The paper
defers ModEval to prior work; the reading used here: with period P = q_0 / s (s the
ciphertext scale) and x = t / (K P) in [-1, 1],
    m ~ (P / 2 pi) sin(2 pi t / P) = (P / 2 pi) D^r(g(x)),
    g(x) = cos(2 pi (K x - 1/4) / 2^r) as a Chebyshev interpolant of degree 63,
    D(y) = 2 y^2 - 1 (r = 3 double angles).
Algorithm 1 then combines Re + i Im and applies StoC1 = S_{l <- 1}
(Sec. 4.2: the remaining StoC2 stages are fused into the next conv).

Ciphertexts here are (x, level, scale): x [2][level+1][N] in coefficient form and the
scale tracked as a float64 computed by one fixed sequence of float64 operations, so
every integer constant (round(value * scale-ratio)) is a reproducible function of
the inputs.  Scale rules:
  * HMult (tensor, relinearisation with the key of s^2, rescale by q_l):
    scale = s_a * s_b / q_l.
  * const_mult(ct, c, lam, tau): drop to level lam+1, multiply by the integer
    round(c * tau * q_{lam+1} / s), rescale -> level lam, scale recorded as tau.
  * add_const(ct, c): add round(c * s) to the constant coefficient of c0.
  * sums combine ciphertexts recorded at the same scale.
Chebyshev evaluation, baby steps T_1..T_7 and giant steps T_8, T_16, T_32 (a sum
  sum_j c_j T_j of baby steps is, by default, the sum of the const_mult of each term;
  the option accumulate=True instead takes each term's integer
  round(c_j tau q_{lam+1} / s_j) at level lam + 1 and rescales the sum once):
  T_2j = 2 T_j^2 - 1;  T_{a+b} = 2 T_a T_b - T_{a-b} (T_{a-b} brought to the
  product's level and scale by const_mult with c = 1);
  p = q T_G + r with q_0 = c_G, q_j = 2 c_{G+j}, r_i = c_i - c_{2G-i} (the Chebyshev
  division by T_G, from T_{G+j} = 2 T_G T_j - T_{G-j}); q is evaluated one level up at
  scale tau q_{lam+1} / s_G so that q T_G lands at (lam, tau); degree < 8 is the
  linear combination sum c_j T_j + c_0.
"""
import math

import numpy as np
from numpy.polynomial import chebyshev as CH

from . import encoding as E
from .plans import Bsgs, prerotate

TWO48 = 2.0 ** 48


def cheb_split(c, G):
    """p = q T_G + r for p = sum c_k T_k of degree d, G <= d < 2G: q_0 = c_G,
    q_j = 2 c_{G+j}, r_i = c_i - c_{2G-i} (from T_{G+j} = 2 T_G T_j - T_{G-j})"""
    c = np.asarray(c, dtype=np.float64)
    d = len(c) - 1
    q = np.zeros(d - G + 1)
    q[0] = c[G]
    r = c[:G].copy()
    for j in range(1, d - G + 1):
        q[j] = 2.0 * c[G + j]
        r[G - j] -= c[G + j]
    return q, r


def cheb_coeffs(K, r, degree=63):
    """Chebyshev interpolant (first-kind nodes; numpy's routine as a step) of
    g(x) = cos(2 pi (K x - 1/4) / 2^r) on [-1, 1]"""
    return CH.chebinterpolate(lambda x: np.cos(2 * np.pi * (K * x - 0.25) / 2.0 ** r), degree)


def model(t, P, K, r, coeffs):
    """FP64 value of the same chain: (P / 2 pi) D^r(sum c_k T_k(t / (K P)))"""
    y = CH.chebval(np.asarray(t, dtype=np.float64) / (K * P), coeffs)
    for _ in range(r):
        y = 2 * y * y - 1
    return P / (2 * np.pi) * y


class Boot:
    """homomorphic steps on an oracle Ctx that holds the relinearisation key ('relin')"""

    def __init__(self, ctx):
        self.ctx = ctx
        self.R = ctx.ring
        self.N = ctx.N

    # ----------------------------------------------------------- primitives
    def drop(self, ct, level):
        x, l, s = ct
        assert level <= l
        return (x[:, :level + 1].copy(), level, s)

    def _const_poly(self, level, k):
        pt = np.zeros((level + 1, self.N), dtype=np.uint64)
        for i in range(level + 1):
            pt[i, 0] = int(k) % self.R.q[i]
        return pt

    def mul_int(self, ct, k):
        x, l, s = ct
        pt = self._const_poly(l, k)
        return (np.stack([self.R.pmult(l, x[0], pt), self.R.pmult(l, x[1], pt)]), l, s)

    def add_const(self, ct, c):
        x, l, s = ct
        k = int(np.rint(c * s))
        y = x.copy()
        for i in range(l + 1):
            y[0, i, 0] = (int(y[0, i, 0]) + k % self.R.q[i]) % self.R.q[i]
        return (y, l, s)

    def add(self, a, b):
        assert a[1] == b[1]
        return (self.ctx.ct_add(a[1], a[0], b[0]), a[1], a[2])

    def sub(self, a, b):
        assert a[1] == b[1]
        return (self.ctx.ct_sub(a[1], a[0], b[0]), a[1], a[2])

    def rescale(self, ct):
        x, l, s = ct
        return (self.ctx.ct_rescale(l, x), l - 1, s / float(self.R.q[l]))

    def hmult(self, a, b):
        """tensor product, relinearisation, rescale"""
        l = min(a[1], b[1])
        x, y = self.drop(a, l)[0], self.drop(b, l)[0]
        R = self.R
        d0 = R.pmult(l, x[0], y[0])
        d1 = R.add(l, R.pmult(l, x[0], y[1]), R.pmult(l, x[1], y[0]))
        d2 = R.pmult(l, x[1], y[1])
        k0, k1 = R.keyswitch(l, d2, self.ctx.keys["relin"])
        t = np.stack([R.add(l, d0, k0), R.add(l, d1, k1)])
        return (self.ctx.ct_rescale(l, t), l - 1, a[2] * b[2] / float(R.q[l]))

    def const_mult(self, ct, c, lam, tau):
        """c * ct at level lam, recorded scale tau; None when the constant rounds to 0"""
        x, l, s = ct
        assert lam < l
        q = float(self.R.q[lam + 1])
        k = int(np.rint(c * tau * q / s))
        if k == 0:
            return None
        y = self.mul_int(self.drop(ct, lam + 1), k)
        return (self.ctx.ct_rescale(lam + 1, y[0]), lam, tau)

    def zero(self, level, scale):
        return (np.zeros((2, level + 1, self.N), dtype=np.uint64), level, scale)

    # ------------------------------------------------------------ Chebyshev
    def sq_minus1(self, a):
        """2 a^2 - 1"""
        p = self.hmult(a, a)
        return self.add_const(self.add(p, p), -1.0)

    def prod_minus(self, a, b, c):
        """2 a b - c, c brought to the product's level and scale"""
        p = self.hmult(a, b)
        c2 = self.const_mult(c, 1.0, p[1], p[2])
        return self.sub(self.add(p, p), c2)

    def cheb_basis(self, x):
        T = {1: x}
        T[2] = self.sq_minus1(T[1])
        T[3] = self.prod_minus(T[1], T[2], T[1])
        T[4] = self.sq_minus1(T[2])
        T[5] = self.prod_minus(T[2], T[3], T[1])
        T[6] = self.sq_minus1(T[3])
        T[7] = self.prod_minus(T[3], T[4], T[1])
        T[8] = self.sq_minus1(T[4])
        T[16] = self.sq_minus1(T[8])
        T[32] = self.sq_minus1(T[16])
        return T

    def eval_cheb(self, T, c, lam, tau, accumulate=False):
        """sum_k c_k T_k at level lam, recorded scale tau.  Baby-step sums (degree < 8):
        by default every term c_j T_j is its own constant multiply and rescale; with
        accumulate=True the terms' integer multiples are summed at one level and the sum
        is rescaled once (an evaluation-order option the library offers as well)"""
        c = np.asarray(c, dtype=np.float64)
        d = len(c) - 1
        if d < 8 and not accumulate:
            acc = None
            for j in range(1, d + 1):
                if c[j] == 0.0:
                    continue
                t = self.const_mult(T[j], c[j], lam, tau)
                if t is not None:
                    acc = t if acc is None else self.add(acc, t)
            if acc is None:
                acc = self.zero(lam, tau)
            return self.add_const(acc, c[0])
        if d < 8:
            # sum_j k_j T_j at level lam + 1 with k_j = round(c_j tau q_{lam+1} / s_j) (each
            # term then stands at scale tau q_{lam+1}), one rescale for the whole sum
            q = float(self.R.q[lam + 1])
            acc = None
            for j in range(1, d + 1):
                if c[j] == 0.0:
                    continue
                k = int(np.rint(c[j] * tau * q / T[j][2]))
                if k == 0:
                    continue
                y = self.mul_int(self.drop(T[j], lam + 1), k)
                acc = y if acc is None else self.add(acc, y)
            if acc is None:
                acc = self.zero(lam, tau)
            else:
                acc = (self.ctx.ct_rescale(lam + 1, acc[0]), lam, tau)
            return self.add_const(acc, c[0])
        G = 32 if d >= 32 else (16 if d >= 16 else 8)
        q, r = cheb_split(c, G)
        tau_q = tau * float(self.R.q[lam + 1]) / T[G][2]
        Q = self.eval_cheb(T, q, lam + 1, tau_q, accumulate)
        prod = self.hmult(Q, T[G])
        rr = self.eval_cheb(T, r, lam, tau, accumulate)
        return (self.add(prod[0:2] + (tau,), rr)[0], lam, tau)

    # -------------------------------------------------------------- ModEval
    def eval_mod(self, ct, K, r, coeffs, accumulate=False):
        """ModEval of a CoeffToSlot output ct = (x, l0, s0); returns (x, l0 - 11, scale)
        encoding the slots' m (degree-63 interpolant, r = 3)"""
        x, l0, s0 = ct
        assert len(coeffs) == 64 and r == 3
        q0 = float(self.R.q[0])
        sx = float(K) * q0                          # the same integers read as x = t / (K P)
        k = int(np.rint(TWO48 * float(self.R.q[l0]) / sx))
        y = self.mul_int((x, l0, sx), k)
        y = (self.ctx.ct_rescale(l0, y[0]), l0 - 1, sx * k / float(self.R.q[l0]))
        T = self.cheb_basis(y)
        lam = y[1] - 7
        g = self.eval_cheb(T, coeffs, lam, float(self.R.q[lam]), accumulate)
        for _ in range(r):
            g = self.sq_minus1(g)
        return (g[0], g[1], g[2] * (2.0 * math.pi) * s0 / q0)

    # ------------------------------------------------- masks and activation
    def mask_mult(self, ct, mask_pt):
        """PMult by a slot mask encoded at scale q_l (coefficient form, l+1 limbs), then
        rescale by q_l: the recorded scale is unchanged"""
        x, l, s = ct
        y = np.stack([self.R.pmult(l, x[0], mask_pt), self.R.pmult(l, x[1], mask_pt)])
        return (self.ctx.ct_rescale(l, y), l - 1, s)

    def slot_activation(self, re, im, K, r, coeffs, masks, act, plan, plan_level):
        """Algorithm 1 after CoeffToSlot: ModEval on Re and Im; PMult by the zero-padding
        masks (masks = (pt_re, pt_im) or None); the activation (act 1: the square x^2 of
        AESPA, Sec. 2.5.2, by HMult; act 0: none); Re + i Im; StoC1 (plan from stoc1_plan,
        its first group at plan_level, the input dropped to it)"""
        er, ei = self.eval_mod(re, K, r, coeffs), self.eval_mod(im, K, r, coeffs)
        if masks is not None:
            er, ei = self.mask_mult(er, masks[0]), self.mask_mult(ei, masks[1])
        if act == 1:
            er, ei = self.hmult(er, er), self.hmult(ei, ei)
        z = self.combine(er, ei)
        assert z[1] >= plan_level
        return self.stoc1(self.drop(z, plan_level), plan)

    # --------------------------------------------------------------- StoC1
    def combine(self, re, im):
        """Re + i Im (i = X^{N/2} on the slots), at the lower level"""
        l = min(re[1], im[1])
        a, b = self.drop(re, l), self.drop(im, l)
        ib = self.ctx.ct_monomial(l, b[0], self.N // 2)
        return (self.ctx.ct_add(l, a[0], ib), l, a[2])

    def stoc1(self, ct, plan):
        """plan: [(Bsgs, pts)] from stoc1_plan, group g at level l - g"""
        x, l, s = ct
        for bs, pts in plan:
            x = self.ctx.ct_rescale(l, self.ctx.bsgs(l, x, bs, pts))
            l -= 1
        return (x, l, s)


def layer_masks(N, W, C, w0):
    """Algorithm 1's zero-padding masks (mask_Re, mask_Im; N/2 reals each).  The
    flattened conv (Sec. 2.5.1) leaves values at the padding positions; the fused conv's
    output holds channel rev_C(k mod C) of padded pixel p = floor(k / C),
    (y, x) = divmod(p, W), in coefficient k, and that pixel is an output pixel iff
    y, x < w0.  CoeffToSlot (T^-1, Sec. 2.3) puts coefficient rev_{N/2}(j) in slot j of
    the real part and coefficient N/2 + rev_{N/2}(j) in slot j of the imaginary part."""
    n2 = N // 2
    p = np.arange(N) // C
    valid = ((p // W < w0) & (p % W < w0)).astype(np.float64)
    rev = np.array([E.bitrev(j, n2) for j in range(n2)])
    return valid[:n2][rev], valid[n2:][rev]


def stoc1_stage_groups(ell, d):
    """strides 1, 2, ..., ell/2 (S_1 applied first) in d consecutive groups"""
    strides = []
    k = 1
    while k < ell:
        strides.append(k)
        k *= 2
    S = len(strides)
    sizes = [S // d + (1 if g < S % d else 0) for g in range(d)]
    out, pos = [], 0
    for sz in sizes:
        out.append(strides[pos:pos + sz])
        pos += sz
    return out


def stoc1_plan(N, ell, d, n1s=None):
    """[(Bsgs, {j: pre-rotated diagonal})] for S_{ell <- 1} in d groups"""
    n = N // 2
    out = []
    for gi, strides in enumerate(stoc1_stage_groups(ell, d)):
        M = None
        for k in strides:  # first stride applied first -> rightmost factor
            D = E.stage_diagonals(k, n)
            M = D if M is None else E.compose(D, M, n)
        plan = Bsgs(n, strides[0], M.keys(), None if n1s is None else n1s[gi])
        out.append((plan, prerotate(plan, M)))
    return out
