"""The N = 2^12 bootstrapping ring shared by the GPU bootstrapping tests: 21 + 4 primes,
a weight-32 secret, the same keys on the oracle's side and the library's (needs a GPU)."""
import numpy as np
import torch

import oracle as O
import oracle.bootstrap as B
import oracle.encoding as E
import oracle.plans as PL
import synth
from oracle.pipeline import Ctx as OCtx
from paper_2312_04356_amd import Ctx, chain_primes

SCALE = 2.0 ** 40


class Rig:
    """the same ring, secret and keys on both sides: by default N = 2^12 with 21 + 4
    primes and a weight-32 secret; Rig(16, 24, 8, 192) is the benchmark's N = 2^16 ring"""

    def __init__(self, log_n=12, n_q=21, n_p=4, h=32):
        print("\n[setup] bootstrap ring N=2^%d, %d + %d primes" % (log_n, n_q, n_p), flush=True)
        self.N = N = 1 << log_n
        q, p = PL.chain_primes(log_n, n_q, n_p, 50, 48, 50, lambda ln, b, c, ex: O.gen_primes(ln, b, c, ex))
        assert (q, p) == tuple(list(map(int, v)) for v in chain_primes(log_n, n_q, n_p, 50, 48, 50))
        self.q, self.p = q, p
        self.R = O.Ring(N, q, p)
        self.s = synth.ternary_secret(N, h, 77)
        self.o = OCtx(self.R, self.s)
        self.boot = B.Boot(self.o)
        self.g = Ctx(log_n, q, p, SCALE)
        self.g.nj_set_secret(self.s)
        self.keys = set()
        self.key("relin")

    def key(self, g):
        if g in self.keys:
            return
        kid = synth.RELIN_KEY_ID if g == "relin" else g
        a, e = synth.key_randomness(self.q + self.p, self.N, self.R.n_digits(self.R.L), 78, kid)
        self.o.add_key(g, a, e)
        self.g.nj_gen_switch_key(0 if g == "relin" else g, a, e)
        self.keys.add(g)

    def enc(self, values, level, scale, sub):
        """slot vector -> (oracle ct, device ct)"""
        coeffs = E.encode(values, self.N, scale)
        m = self.R.to_rns(coeffs, level)
        a, e = synth.enc_randomness(self.q[:level + 1], self.N, 79, sub)
        x = self.R.encrypt_sk(level, self.s, m, a, e)
        ct = self.g.empty_ct(level)
        self.g.nj_encrypt_sk(self.g.to_device(m), level, a, e, scale, ct)
        return x, ct

    def coeff(self, ct):
        t = ct.data.clone()
        self.g.nj_to_coeff(t, ct.level, 2)
        torch.cuda.synchronize()
        return self.g.to_host(t)

    def dec_slots(self, ct):
        d = torch.empty((ct.level + 1, self.N), dtype=torch.int64, device=self.g.device)
        self.g.nj_decrypt(ct, d)
        m = np.array(O.centred_from_limbs(self.g.to_host(d)[:min(3, ct.level + 1)], self.q[:min(3, ct.level + 1)]),
                     dtype=np.float64)
        return E.decode(m, self.N, ct.scale)
