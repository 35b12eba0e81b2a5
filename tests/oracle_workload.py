"""Builds an oracle context for a named synthetic workload (tests and CPU baseline only)."""
import numpy as np

import oracle as O
import oracle.encoding as E
import oracle.plans as PL
import synth
from oracle.pipeline import Ctx


class OracleWorkload:
    def __init__(self, name, with_cts=True, n1=None, cts_split=True):
        """cts_split: the CoeffToSlot groups' baby-step counts from the workload's
        "cts_n1" (else, or when False, the default split)"""
        w = dict(synth.WORKLOADS[name])
        self.w = w
        self.N = N = 1 << w["log_n"]
        q, p = PL.chain_primes(w["log_n"], w["n_q"], w["alpha"], w["q0_bits"], w["q_bits"], w["p_bits"],
                               lambda ln, b, c, ex: O.gen_primes(ln, b, c, ex))
        self.ring = O.Ring(N, q, p)
        self.scale = 2.0 ** w["log_scale"]
        self.s = synth.ternary_secret(N, w["h"], w["key_seed"])
        self.ctx = Ctx(self.ring, self.s)
        self.W = PL.padded_width(w["w0"], w["f"])
        self.ell = self.W * self.W // 2
        self.C = N // (self.W * self.W)
        self.img = synth.uniform_real((w["c_in"], w["w0"], w["w0"]), w["data_seed"], 0)
        self.K = synth.uniform_real((w["c_out"], w["c_in"], w["f"], w["f"]), w["data_seed"], 1)
        self.conv_bsgs, conv_diags = PL.conv_plan(self.K, self.W, N, n1)
        self.conv_pts = PL.encode_diagonals(conv_diags, N, float(q[1]), self.ring, 1)
        self.cts = []
        if with_cts:
            L = self.ring.L
            n1s = w.get("cts_n1") if cts_split else None
            for g, (plan, diags) in enumerate(PL.cts_plan(N, w["cts_groups"], n1s)):
                lvl = L - g
                self.cts.append((plan, PL.encode_diagonals(diags, N, float(q[lvl]), self.ring, lvl)))

    def rotations(self):
        rs = set(self.conv_bsgs.rotations())
        for plan, _ in self.cts:
            rs |= set(plan.rotations())
        return sorted(rs)

    def galois_elements(self):
        gs = [PL.galois_elt(r, self.N) for r in self.rotations()]
        if self.cts:
            gs.append(2 * self.N - 1)
        return gs

    def make_keys(self, gs=None):
        R = self.ring
        for g in (self.galois_elements() if gs is None else gs):
            a, e = synth.key_randomness(R.key_primes(), self.N, R.n_digits(R.L), self.w["key_seed"], g)
            self.ctx.add_key(g, a, e)

    def input_plaintext(self):
        z = E.real_cins_slots(PL.image_to_slices(self.img, self.W), self.ell)
        return E.encode(z, self.N, self.scale)

    def encrypt_input(self, level=1):
        m = self.ring.to_rns(self.input_plaintext(), level)
        a, e = synth.enc_randomness(self.ring.q[:level + 1], self.N, self.w["data_seed"], 0)
        return self.ring.encrypt_sk(level, self.s, m, a, e)

    def conv_reference(self):
        return PL.conv2d_same(self.img, self.K)

    def read_conv_output(self, coeffs):
        """coefficient layout a[(y W + x) C + rev_C(c)] -> (C, w0, w0)"""
        w0, W, C = self.w["w0"], self.W, self.C
        out = np.zeros((C, w0, w0))
        for c in range(C):
            rc = E.bitrev(c, C)
            for y in range(w0):
                idx = (y * W + np.arange(w0)) * C + rc
                out[c, y] = np.asarray(coeffs, dtype=np.float64)[idx]
        return out
