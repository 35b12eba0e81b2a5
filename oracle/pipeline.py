"""Oracle homomorphic pipeline: rotations, BSGS transforms, fused conv, CoeffToSlot.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows, in the paper's order:
  * HRot (Sec. 2.1): left rotation of the slots by r is the automorphism
    X -> X^(5^r mod 2N) followed by key switching back to s.
  * BSGS (Sec. 2.6): sum_g ( sum_i d'_{g n1 + i} (.) (ct <<< i u) ) <<< g n1 u; the
    baby rotations are hoisted (one ModUp of c1, automorphism applied to the
    extended digits) when `hoist` is True, giant rotations are plain.
  * Fused conv (Algorithm 1, Sec. 4): BSGS at level 1 with K^' diagonals,
    then rescale to level 0.
  * CoeffToSlot (Sec. 2.4; Algorithm 1): ModRaise to the top level, one
    BSGS transform + rescale per stage group, then the real split
    Re = ct + conj(ct), Im = -X^{N/2} (ct - conj(ct)).
"""
import numpy as np

from .plans import galois_elt


def automorph_int(s, g):
    """s(X^g) for a small signed integer polynomial"""
    n = len(s)
    out = np.zeros(n, dtype=np.int64)
    for i in range(n):
        e = i * g % (2 * n)
        if e < n:
            out[e] += s[i]
        else:
            out[e - n] -= s[i]
    return out


def square_int(s):
    """s^2 in Z[X]/(X^n+1) for a ternary s (schoolbook over the nonzero support)"""
    n = len(s)
    nz = np.nonzero(s)[0]
    out = np.zeros(n, dtype=np.int64)
    for i in nz:
        for j in nz:
            k = i + j
            v = int(s[i]) * int(s[j])
            if k < n:
                out[k] += v
            else:
                out[k - n] -= v
    return out


class Ctx:
    """ring + secret + switching keys by Galois element (1 is never used; 'relin' for s^2)."""

    def __init__(self, ring, s):
        self.ring = ring
        self.N = ring.n
        self.s = np.asarray(s, dtype=np.int64)
        self.keys = {}

    def add_key(self, g, a, e):
        sp = square_int(self.s) if g == "relin" else automorph_int(self.s, g)
        self.keys[g] = self.ring.switch_key(self.s, sp, a, e)
        return self.keys[g]

    # ---------------------------------------------------------------- ct ops
    def ct_add(self, level, x, y):
        return np.stack([self.ring.add(level, x[0], y[0]), self.ring.add(level, x[1], y[1])])

    def ct_sub(self, level, x, y):
        return np.stack([self.ring.sub(level, x[0], y[0]), self.ring.sub(level, x[1], y[1])])

    def ct_pmult(self, level, x, pt):
        return np.stack([self.ring.pmult(level, x[0], pt), self.ring.pmult(level, x[1], pt)])

    def ct_rescale(self, level, x):
        return np.stack([self.ring.rescale(level, x[0]), self.ring.rescale(level, x[1])])

    def ct_modraise(self, x, top=None):
        return np.stack([self.ring.modraise(x[0][0], top), self.ring.modraise(x[1][0], top)])

    def ct_monomial(self, level, x, k):
        return np.stack([self.ring.poly_monomial(level, x[0], k), self.ring.poly_monomial(level, x[1], k)])

    def apply_galois(self, level, x, g):
        """(tau_g(c0), tau_g(c1)) switched back to s, plain (non-hoisted)"""
        c0 = self.ring.poly_automorph(level, x[0], g)
        d = self.ring.poly_automorph(level, x[1], g)
        k0, k1 = self.ring.keyswitch(level, d, self.keys[g])
        return np.stack([self.ring.add(level, c0, k0), k1])

    def rotate(self, level, x, r):
        r %= self.N // 2
        if r == 0:
            return x.copy()
        return self.apply_galois(level, x, galois_elt(r, self.N))

    def hoisted_rotations(self, level, x, rs):
        """{r: x <<< r} sharing one ModUp of c1"""
        ext = self.ring.modup(level, x[1])
        out = {}
        for r in rs:
            r %= self.N // 2
            if r == 0:
                out[r] = x.copy()
                continue
            g = galois_elt(r, self.N)
            k0, k1 = self.ring.keyswitch_ext(level, ext, g, self.keys[g])
            c0 = self.ring.poly_automorph(level, x[0], g)
            out[r] = np.stack([self.ring.add(level, c0, k0), k1])
        return out

    def bsgs(self, level, x, plan, pts, hoist=True, lazy=False):
        """sum_j pts[j] (.) (x <<< j u), evaluated baby-step giant-step.  lazy: the giant
        rotations' key inner products are summed over Q_l u P and share one ModDown
        (their rotated c0 parts are summed alongside)"""
        babies = plan.babies
        if hoist:
            rot = self.hoisted_rotations(level, x, [plan.baby_rot(i) for i in babies])
            baby = {i: rot[plan.baby_rot(i) % (self.N // 2)] for i in babies}
        else:
            baby = {i: self.rotate(level, x, plan.baby_rot(i)) for i in babies}
        acc = None
        inners = {}
        for g in plan.giants:
            inner = None
            for j, (gg, i) in sorted(plan.split.items()):
                if gg != g:
                    continue
                t = self.ct_pmult(level, baby[i], pts[j])
                inner = t if inner is None else self.ct_add(level, inner, t)
            inners[g] = inner
        if lazy:
            return self._giants_lazy(level, plan, inners)
        for g in plan.giants:
            inner = inners[g]
            if g != 0:
                inner = self.rotate(level, inner, plan.giant_rot(g))
            acc = inner if acc is None else self.ct_add(level, acc, inner)
        return acc

    def _giants_lazy(self, level, plan, inners):
        R = self.ring
        ext_q = np.array(R.ext_primes(level), dtype=np.uint64)[:, None]
        u0s = u1s = c0s = None
        for g in plan.giants:
            if g == 0:
                continue
            ge = galois_elt(plan.giant_rot(g), self.N)
            c0 = R.poly_automorph(level, inners[g][0], ge)
            d = R.poly_automorph(level, inners[g][1], ge)
            u0, u1 = R.key_ip(level, R.modup(level, d), 1, self.keys[ge])
            if u0s is None:
                u0s, u1s, c0s = u0, u1, c0
            else:
                u0s, u1s = (u0s + u0) % ext_q, (u1s + u1) % ext_q
                c0s = R.add(level, c0s, c0)
        if u0s is None:
            return inners[0]
        out = np.stack([R.add(level, c0s, R.moddown(level, u0s)), R.moddown(level, u1s)])
        return self.ct_add(level, inners[0], out) if 0 in inners else out

    # ------------------------------------------------------------ the path
    def conv2d_cins(self, x, plan, pts, level=1, hoist=True, lazy=False):
        y = self.bsgs(level, x, plan, pts, hoist, lazy)
        return self.ct_rescale(level, y)

    def conj_split(self, level, x):
        c = self.apply_galois(level, x, 2 * self.N - 1)
        re = self.ct_add(level, x, c)
        im = self.ct_monomial(level, self.ct_sub(level, x, c), 3 * self.N // 2)
        return re, im

    def coeff_to_slot(self, x0, groups, group_pts, hoist=True, lazy=False):
        """x0: level-0 ct [2][1][N].  groups: [Bsgs]; group_pts[g]: {j: pt} at level L-g.
        hoist: one flag, or one per group."""
        x = self.ct_modraise(x0)
        level = self.ring.L
        hs = list(hoist) if isinstance(hoist, (list, tuple)) else [hoist] * len(groups)
        for plan, pts, h in zip(groups, group_pts, hs):
            x = self.bsgs(level, x, plan, pts, h, lazy)
            x = self.ct_rescale(level, x)
            level -= 1
        return self.conj_split(level, x)


def block_bsgs(ctx, level, xs, plan, pts, bo, hoist=True):
    """Block matrix-vector product of Sec. 3.3.4 with BSGS: out_ob = sum_ib K^(ob,ib) x_ib.
    Baby rotations of every input ciphertext are computed once (hoisted ModUp per
    input); for each output block and giant step the inner sum runs over all input
    blocks and baby steps, then one giant rotation is applied to it.
    pts[(ob, ib)][j]: integer plaintext of diagonal j of block (ob, ib)."""
    babies = []
    for x in xs:
        if hoist:
            rot = ctx.hoisted_rotations(level, x, [plan.baby_rot(i) for i in plan.babies])
            babies.append({i: rot[plan.baby_rot(i) % (ctx.N // 2)] for i in plan.babies})
        else:
            babies.append({i: ctx.rotate(level, x, plan.baby_rot(i)) for i in plan.babies})
    outs = []
    for ob in range(bo):
        acc = None
        for g in plan.giants:
            inner = None
            for ib in range(len(xs)):
                for j, (gg, i) in sorted(plan.split.items()):
                    if gg != g or j not in pts[(ob, ib)]:
                        continue
                    t = ctx.ct_pmult(level, babies[ib][i], pts[(ob, ib)][j])
                    inner = t if inner is None else ctx.ct_add(level, inner, t)
            if g != 0:
                inner = ctx.rotate(level, inner, plan.giant_rot(g))
            acc = inner if acc is None else ctx.ct_add(level, acc, inner)
        outs.append(acc)
    return outs


def block_conv(ctx, level, xs, plan, pts, bo, hoist=True):
    """conv layer of Sec. 3.3 (fused with StoC2 when its plan is): block BSGS, then rescale"""
    return [ctx.ct_rescale(level, y) for y in block_bsgs(ctx, level, xs, plan, pts, bo, hoist)]
