"""Sets up a named synthetic workload on the GPU through the library's ABI.

Context with the chain primes, secret key, switching keys for the fused conv and
CoeffToSlot plans, and the real-CinS encrypted input image.  All randomness comes
from `synth` (seeded Philox); all arithmetic runs in libneujeans.
"""
import numpy as np

import synth

from . import Ctx, chain_primes


def padded_width(w0, f):
    p = (f - 1) // 2
    W = 1
    while W < w0 + p:
        W *= 2
    return W


class GpuWorkload:
    def __init__(self, name, with_cts=True, conv_n1=0, lazy=False, cts_split=True):
        """cts_split: the CoeffToSlot groups' baby-step counts from the workload's
        "cts_n1" (else, or when False, the library's default split)"""
        import torch
        self.torch = torch
        w = dict(synth.WORKLOADS[name])
        self.name, self.w = name, w
        self.N = 1 << w["log_n"]
        self.q, self.p = chain_primes(w["log_n"], w["n_q"], w["alpha"], w["q0_bits"], w["q_bits"], w["p_bits"])
        self.scale = 2.0 ** w["log_scale"]
        self.ctx = Ctx(w["log_n"], self.q, self.p, self.scale)
        self.s = synth.ternary_secret(self.N, w["h"], w["key_seed"])
        self.ctx.nj_set_secret(self.s)
        self.W = padded_width(w["w0"], w["f"])
        self.ell = self.W * self.W // 2
        self.C = self.N // (self.W * self.W)
        self.img = synth.uniform_real((w["c_in"], w["w0"], w["w0"]), w["data_seed"], 0)
        self.K = synth.uniform_real((w["c_out"], w["c_in"], w["f"], w["f"]), w["data_seed"], 1)
        self.conv_plan = self.ctx.nj_conv_plan_create(w["w0"], w["f"], self.K, conv_n1)
        self.cts_plan = None
        if with_cts:
            n1s = w.get("cts_n1") if cts_split else None
            self.cts_plan = (self.ctx.nj_cts_plan_create_split(w["cts_groups"], n1s) if n1s
                             else self.ctx.nj_cts_plan_create(w["cts_groups"]))
        if lazy and self.cts_plan is not None:
            self.cts_plan.set_lazy(True)
        self.keys_made = set()

    def galois_elements(self):
        gs = set(self.conv_plan.galois())
        if self.cts_plan is not None:
            gs |= set(self.cts_plan.galois())
        return sorted(gs)

    def make_keys(self, gs=None):
        primes = self.q + self.p
        for g in (self.galois_elements() if gs is None else gs):
            if g in self.keys_made:
                continue
            a, e = synth.key_randomness(primes, self.N, self.ctx.dnum, self.w["key_seed"], g)
            self.ctx.nj_gen_switch_key(g, a, e)
            self.keys_made.add(g)

    def image_slices(self):
        out = np.zeros((self.C, self.W, self.W))
        w0 = self.w["w0"]
        out[:self.img.shape[0], :w0, :w0] = self.img
        return out.reshape(self.C, self.W * self.W)

    def encrypt_input(self, level=1, m_dev=None):
        """real-CinS encoded image, encrypted at `level` (plaintext from the library's encoder
        unless device residues m_dev are given)"""
        if m_dev is None:
            coeffs = self.ctx.nj_encode_cins(self.image_slices(), self.scale)
            m_dev = self.torch.empty((level + 1, self.N), dtype=self.torch.int64, device=self.ctx.device)
            self.ctx.nj_upload_plain(coeffs, level, m_dev)
        a, e = synth.enc_randomness(self.q[:level + 1], self.N, self.w["data_seed"], 0)
        ct = self.ctx.empty_ct(level)
        return self.ctx.nj_encrypt_sk(m_dev, level, a, e, self.scale, ct)
