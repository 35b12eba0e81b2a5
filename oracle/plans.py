"""Oracle plan builders: fused conv diagonals and CoeffToSlot stage groups (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Fused conv (Sec. 3.3.2-3.3.4, Sec. 4, Eq. nested_conv):
  * each C_in/C_out kernel becomes a length-2l polynomial (W x W = 2l real slots,
    row-major, zero padding) so that the negacyclic product with the flattened
    input channel yields the 'same'-padded cross-correlation;
  * K^[o][i] = DFT'_{2l}(k_{o,i});  S' = S_{N/2<-l} = S_{N/4} ... S_l acts slice-wise,
    K^' = S' K^ (product of C x C matrices of length-l slices, Sec. 4.1-4.2);
  * cyclic diagonals d_k = (K^'[0][k] | K^'[1][1+k] | ... ), slice c holding
    K^'[c][(c+k) mod C];  the conv output is sum_k d_k (.) (ct <<< k l);
  * baby-step giant-step (Sec. 2.6): d'_{g n1 + i} = d_{g n1 + i} >>> g n1 l.
CoeffToSlot (Sec. 2.4): T_{N/2}^{-1} = S_1^{-1} ... S_{N/4}^{-1}; its stages, applied
  S_{N/4}^{-1} first, are grouped into d consecutive groups, one BSGS transform each;
  the 1/2 of the real/imaginary split is folded into the last group.
"""
import math

import numpy as np

from . import encoding as E


# ------------------------------------------------------------------ layouts

def padded_width(w0, f):
    """smallest power of two W with W >= w0 + (f-1)/2, so that wrap-around lands in padding"""
    p = (f - 1) // 2
    W = 1
    while W < w0 + p:
        W *= 2
    return W


def image_to_slices(img, W):
    """img: (C, w0, w0) -> (C, W*W) row-major, zero padded"""
    C, w0, _ = img.shape
    out = np.zeros((C, W, W))
    out[:, :w0, :w0] = img
    return out.reshape(C, W * W)


def kernel_poly(K, W):
    """k(Y) = sum_{u,v} K[u][v] Y^{-((u-p)W + (v-p))} mod (Y^{W^2} + 1), p = (f-1)/2"""
    f = K.shape[0]
    p = (f - 1) // 2
    n = W * W
    k = np.zeros(n)
    for u in range(f):
        for v in range(f):
            e = -((u - p) * W + (v - p))
            if e >= 0:
                k[e % n] += K[u, v]
            else:
                k[(e + n) % n] -= K[u, v]
    return k


def conv2d_same(img, K):
    """plain FP64 cross-correlation with 'same' zero padding: O[o] = sum_i K[o][i] * I[i]"""
    C_in, w0, _ = img.shape
    C_out, _, f, _ = K.shape
    p = (f - 1) // 2
    pad = np.zeros((C_in, w0 + 2 * p, w0 + 2 * p))
    pad[:, p:p + w0, p:p + w0] = img
    out = np.zeros((C_out, w0, w0))
    for u in range(f):
        for v in range(f):
            out += np.einsum("oi,iyx->oyx", K[:, :, u, v], pad[:, u:u + w0, v:v + w0])
    return out


# ------------------------------------------------------------- BSGS structure

class Bsgs:
    """Diagonal offsets j*u (j representatives centred in [-h, n/u - h)), baby size n1."""

    def __init__(self, n, u, offsets, n1=None):
        self.n, self.u = n, u
        h = (n // u) // 2
        reps = sorted({((int(r) // u + h) % (n // u)) - h for r in offsets})
        self.js = reps
        self.n1 = n1 if n1 is not None else int(math.ceil(math.sqrt(len(reps))))
        self.split = {j: (j // self.n1, j - (j // self.n1) * self.n1) for j in reps}

    @property
    def babies(self):
        return sorted({i for (_, i) in self.split.values()})

    @property
    def giants(self):
        return sorted({g for (g, _) in self.split.values()})

    def baby_rot(self, i):
        return (i * self.u) % self.n

    def giant_rot(self, g):
        return (g * self.n1 * self.u) % self.n

    def rotations(self):
        return sorted({self.baby_rot(i) for i in self.babies if i} | {self.giant_rot(g) for g in self.giants if g})


def galois_elt(r, N):
    """X -> X^(5^r mod 2N): left rotation of the slots by r"""
    return pow(5, r % (N // 2), 2 * N)


# ------------------------------------------------------------------- conv

def conv_plan(K, W, N, n1=None):
    """Fused conv + StoC2 diagonals (complex slot vectors), BSGS-pre-rotated.

    K: (C, C, f, f) with C = N / W^2.  Returns (Bsgs, {j: pre-rotated diagonal}).
    """
    n = N // 2
    ell = W * W // 2
    C = n // ell
    assert K.shape[0] == C and K.shape[1] == C
    Kh = np.zeros((C, C, ell), dtype=np.complex128)
    for o in range(C):
        for i in range(C):
            Kh[o, i] = E.dft_prime(kernel_poly(K[o, i], W), ell)
    # K^' = S' K^, column by column: S' = S_{n/2} ... S_l applies S_l first
    Kp = np.zeros_like(Kh)
    for i in range(C):
        col = Kh[:, i, :].reshape(-1)
        k = ell
        while k < n:
            col = E.apply_stage(col, k)
            k *= 2
        Kp[:, i, :] = col.reshape(C, ell)
    diags = {}
    for k in range(C):
        diags[k * ell] = np.concatenate([Kp[c, (c + k) % C] for c in range(C)])
    plan = Bsgs(n, ell, diags.keys(), n1)
    return plan, prerotate(plan, diags)


def prerotate(plan, diags):
    out = {}
    for r, d in diags.items():
        j = ((r // plan.u + (plan.n // plan.u) // 2) % (plan.n // plan.u)) - (plan.n // plan.u) // 2
        g, _ = plan.split[j]
        out[j] = E.rotr(d, g * plan.n1 * plan.u)
    return out


# --------------------------------------------------------------- CoeffToSlot

def cts_stage_groups(n, d):
    """strides in application order (n/2, n/4, ..., 1) split into d consecutive groups"""
    strides = []
    k = n // 2
    while k >= 1:
        strides.append(k)
        k //= 2
    S = len(strides)
    sizes = [S // d + (1 if g < S % d else 0) for g in range(d)]
    groups, pos = [], 0
    for s in sizes:
        groups.append(strides[pos:pos + s])
        pos += s
    return groups


def cts_plan(N, d, n1s=None):
    """[(Bsgs, {j: pre-rotated diagonal})] for each group, last group scaled by 1/2."""
    n = N // 2
    out = []
    groups = cts_stage_groups(n, d)
    for gi, strides in enumerate(groups):
        M = None
        for k in strides:  # first stride applied first -> rightmost factor
            D = E.stage_diagonals(k, n, inverse=True)
            M = D if M is None else E.compose(D, M, n)
        if gi == len(groups) - 1:
            M = {r: 0.5 * v for r, v in M.items()}
        plan = Bsgs(n, strides[-1], M.keys(), None if n1s is None else n1s[gi])
        out.append((plan, prerotate(plan, M)))
    return out


def encode_diagonals(diags, N, scale, ring, level):
    """{j: complex slot vector} -> {j: residues [(level+1)][N]} at the given scale"""
    return {j: ring.to_rns(E.encode(v, N, scale), level) for j, v in diags.items()}


def chain_primes(log_n, n_q, alpha, q0_bits, q_bits, p_bits, gen):
    """prime chain: q_0 (q0_bits), q_1..q_{n_q-1} (q_bits), p_0..p_{alpha-1} (p_bits), all distinct,
    each the next unused prime below 2^bits of the form k 2N + 1 (gen implements that rule)"""
    q0 = gen(log_n, q0_bits, 1, [])
    qs = gen(log_n, q_bits, n_q - 1, q0)
    ps = gen(log_n, p_bits, alpha, q0 + qs)
    return q0 + qs, ps


# ------------------------------------------------------- general conv layers
#
# A conv layer is a list of taps (o, i, dy, dx, w): output channel o receives
# w * I_i[y + dy][x + dx] (cross-correlation, zero outside the image).
#   * 3x3 / 1x1 stride 1, 'same' padding: dy = u - p, dx = v - p.
#   * stride 2 (Sec. 5, Algorithm 2; Appendix B): O[y][x] = sum K[u][v] I[2y+u-p][2x+v-p]
#     is the sum over phases (a, b) of unit-stride convs of the polyphase images
#     I^(a,b)[y][x] = I[2y+a][2x+b] with taps u - p = 2 dy + a, v - p = 2 dx + b.
# Channel counts above C = N/W^2 are split into C x C blocks (Sec. 3.3.4).

def taps_same(K):
    """K (C_out, C_in, f, f), stride 1 'same' -> taps"""
    co, ci, f, _ = K.shape
    p = (f - 1) // 2
    return [(o, i, u - p, v - p, float(K[o, i, u, v])) for o in range(co) for i in range(ci)
            for u in range(f) for v in range(f)]


def taps_stride2(K):
    """K (C_out, C_in, f, f), stride 2 -> taps on the polyphase input (4 C_in channels,
    channel 4 i + 2 b + a holds I_i[a::2, b::2]: the four phases of a channel adjacent,
    which keeps the slot permutation that rearranges an image into them to W - 1 cyclic
    diagonals)"""
    co, ci, f, _ = K.shape
    p = (f - 1) // 2
    out = []
    for o in range(co):
        for i in range(ci):
            for u in range(f):
                for v in range(f):
                    dy, a = divmod(u - p, 2)
                    dx, b = divmod(v - p, 2)
                    out.append((o, 4 * i + 2 * b + a, dy, dx, float(K[o, i, u, v])))
    return out


def taps_depthwise(K):
    """K (C, f, f) depthwise, stride 1 'same' -> taps (c, c, dy, dx, w)"""
    c, f, _ = K.shape
    p = (f - 1) // 2
    return [(ch, ch, u - p, v - p, float(K[ch, u, v])) for ch in range(c) for u in range(f) for v in range(f)]


def polyphase(img):
    """(C, w, w) -> (4C, w/2, w/2), channel 4 i + 2 b + a = img[i, a::2, b::2]"""
    C, w, _ = img.shape
    out = np.zeros((4 * C, w // 2, w // 2))
    for i in range(C):
        for a in (0, 1):
            for b in (0, 1):
                out[4 * i + 2 * b + a] = img[i, a::2, b::2]
    return out


def conv2d_taps(img, taps, c_out):
    """plain FP64 reference of a tap list"""
    C, w, _ = img.shape
    out = np.zeros((c_out, w, w))
    for (o, i, dy, dx, wt) in taps:
        sh = np.zeros((w, w))
        ys, xs = slice(max(0, -dy), min(w, w - dy)), slice(max(0, -dx), min(w, w - dx))
        yd, xd = slice(max(0, dy), min(w, w + dy)), slice(max(0, dx), min(w, w + dx))
        sh[ys, xs] = img[i][yd, xd]
        out[o] += wt * sh
    return out


def conv2d_strided(img, K, s):
    """plain FP64 strided cross-correlation with padding (f-1)/2"""
    C_in, w, _ = img.shape
    co, _, f, _ = K.shape
    p = (f - 1) // 2
    pad = np.zeros((C_in, w + 2 * p, w + 2 * p))
    pad[:, p:p + w, p:p + w] = img
    wo = (w + 2 * p - f) // s + 1
    out = np.zeros((co, wo, wo))
    for u in range(f):
        for v in range(f):
            out += np.einsum("oi,iyx->oyx", K[:, :, u, v], pad[:, u:u + s * wo:s, v:v + s * wo:s])
    return out


def padded_width_taps(w0, taps):
    """smallest power of two W with every tap's wrap-around landing in the padding"""
    reach = max([max(abs(t[2]), abs(t[3])) for t in taps] + [0])
    W = 1
    while W < w0 + reach:
        W *= 2
    return W


def kernel_poly_taps(taps, W):
    """k(Y) = sum w Y^{-(dy W + dx)} mod (Y^{W^2} + 1) for the taps of one (o, i) pair"""
    n = W * W
    k = np.zeros(n)
    for (dy, dx, wt) in taps:
        e = -(dy * W + dx)
        if e >= 0:
            k[e % n] += wt
        else:
            k[(e + n) % n] -= wt
    return k


def block_conv_plan(taps, c_in, c_out, W, N, fuse=True, n1=None):
    """Diagonals of a (possibly blocked) CinS conv: returns (Bsgs, bi, bo,
    {(ob, ib): {j: pre-rotated diagonal}}).  fuse = True multiplies StoC2 into the
    kernel matrix (K^' = S'K^); fuse = False keeps K^ (CinS output) and only the
    diagonals that are nonzero in some block."""
    n = N // 2
    ell = W * W // 2
    C = n // ell
    bi, bo = -(-c_in // C), -(-c_out // C)
    by = {}
    for (o, i, dy, dx, wt) in taps:
        by.setdefault((o, i), []).append((dy, dx, wt))
    blocks = {}
    for ob in range(bo):
        for ib in range(bi):
            Kh = np.zeros((C, C, ell), dtype=np.complex128)
            for o in range(C):
                for i in range(C):
                    t = by.get((ob * C + o, ib * C + i))
                    if t:
                        Kh[o, i] = E.dft_prime(kernel_poly_taps(t, W), ell)
            if fuse:
                for i in range(C):
                    col = Kh[:, i, :].reshape(-1)
                    k = ell
                    while k < n:
                        col = E.apply_stage(col, k)
                        k *= 2
                    Kh[:, i, :] = col.reshape(C, ell)
            diags = {}
            for k in range(C):
                d = np.concatenate([Kh[c, (c + k) % C] for c in range(C)])
                if fuse or np.any(d != 0):
                    diags[k * ell] = d
            blocks[(ob, ib)] = diags
    # one BSGS structure for every block: all C offsets when fused, else the
    # offsets that some block has
    offsets = sorted({r for diags in blocks.values() for r in diags})
    structure = Bsgs(n, ell, offsets, n1)
    diags_all = {key: prerotate(structure, diags) for key, diags in blocks.items()}
    return structure, bi, bo, diags_all
