"""A ResNet-18-shaped network on a 224 x 224 x 3 input, end to end through the library at
N = 2^16 (the analog of Table 2's NeuJeans column, timing only: synthetic weights).

Every conv is a fused CinS conv (Sec. 4: K' = S'K, block convs of Sec. 3.3.4) at level 1
followed by bootstrapping as in Algorithm 1: CoeffToSlot, ModEval of Re and Im, the
zero-padding masks, the square activation (AESPA, Sec. 2.5.2), Re + i Im, StoC1.  Every
stride-2 layer uses the decomposed flow (Algorithm 2, Sec. 5): the bootstrapping before
it rearranges each ciphertext's image into phase images (nj_downsample_plan_create) before
StoC1, and the stride-2 conv is a unit-stride conv over the phase channels.

  stem    conv1 7x7/2 3 -> 64 (224 -> 112; the client encrypts the input's phase images,
          3 ciphertexts), square; then 3x3/2 average pooling as a stride-2 depthwise conv
          (Sec. 3.3.5) on the decomposed conv1 output (112 -> 56), no activation
  stage 1 2 blocks of 2 x (3x3 64 @ 56), identity shortcuts
  stages 2-4  first block: 3x3/2 and 3x3, shortcut 1x1/2; second block: 2 x 3x3,
          identity shortcut (128 @ 28, 256 @ 14, 512 @ 7)
A shortcut joins its block's second conv output in coefficient form at level 0, before
that output's bootstrapping: the identity as the fused conv of the identity kernel
(depthwise 1x1 of ones, fused with StoC2), the downsampling shortcut as its 1x1/2 conv
on the same phase images as the block's first conv.  Weights U(-1, 1) / sqrt(f^2 c_in)
(synthetic, seed 1005), input U(-1, 1).  Phases are timed by HIP events around each
library call (one call at a time), in Table 2's rows.

    python -m paper_2312_04356_amd.network --out gpurun_out/resnet18.json [--md gpurun_out/resnet18.md]
"""
import argparse
import json
import math
import time

import numpy as np

import synth

from . import Ct, nj_layer_masks
from .workload import GpuWorkload

K_MOD, R_DA = 32, 3
LVL_MASK = 9     # ModEval output level (CoeffToSlot 23 -> 20, ModEval 20 -> 9)
LVL_DEC = 7      # decomposition plans (after mask and square)
LVL_STOC = 4     # StoC1 plans (3 groups -> level 1, the conv level)
N_LOG = 16


def padded(w0, reach):
    W = 1
    while W < w0 + reach:
        W *= 2
    return W


class Net:
    def __init__(self, seed=1005):
        import torch
        self.torch = torch
        self.g = GpuWorkload("full", with_cts=True, lazy=True)
        self.c = self.g.ctx
        self.N = self.g.N
        self.seed = seed
        self.sub = 0
        a, e = synth.key_randomness(self.g.q + self.g.p, self.N, self.c.dnum, self.g.w["key_seed"],
                                    synth.RELIN_KEY_ID)
        self.c.nj_gen_switch_key(0, a, e)
        self.ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
        self.times, self.counts = {}, {}
        self.masks, self.stoc1, self.dec = {}, {}, {}
        self.plans = []

    # ------------------------------------------------------------ helpers
    def weights(self, shape, fan_in):
        self.sub += 1
        return synth.uniform_real(shape, self.seed, self.sub) / math.sqrt(fan_in)

    def timed(self, phase, fn):
        t = self.torch
        t.cuda.synchronize()
        self.ev[0].record()
        out = fn()
        self.ev[1].record()
        t.cuda.synchronize()
        self.times[phase] = self.times.get(phase, 0.0) + self.ev[0].elapsed_time(self.ev[1])
        self.counts[phase] = self.counts.get(phase, 0) + 1
        return out

    def mask(self, W, C, w0):
        key = (W, C, w0)
        if key not in self.masks:
            c, pts = self.c, []
            for mk in nj_layer_masks(N_LOG, W, C, w0):
                t = self.torch.empty((LVL_MASK + 1, self.N), dtype=self.torch.int64, device=c.device)
                c.nj_upload_plain(c.nj_encode_slots(mk, float(self.g.q[LVL_MASK])), LVL_MASK, t)
                c.nj_to_eval(t, LVL_MASK, 1)
                pts.append(t)
            self.masks[key] = pts
        return self.masks[key]

    def stoc1_plan(self, W):
        if W not in self.stoc1:
            self.stoc1[W] = self.c.nj_stoc1_plan_create(W * W // 2, 3, LVL_STOC)
        return self.stoc1[W]

    def dec_plans(self, W, C):
        if (W, C) not in self.dec:
            self.dec[(W, C)] = [self.c.nj_downsample_plan_create(0, W, C, h, LVL_DEC) for h in (0, 1)]
        return self.dec[(W, C)]

    def conv_plan(self, w0, K, stride=1, depthwise=False):
        p = self.c.nj_conv_plan_create_layer(w0, K, stride=stride, depthwise=depthwise, level=1)
        self.plans.append(p)
        return p

    # ------------------------------------------------------------ the layer steps
    def conv(self, plan, xs):
        """block conv of CinS inputs (list of level >= 1 cts) -> list of level-0 outputs"""
        c = self.c
        _, W, C, ell, bi, bo = plan.layout()
        assert len(xs) == bi, (len(xs), bi)
        x = c.empty_batch(bi, 1)
        for k, ct in enumerate(xs):
            if ct.level == 1:
                x.data[k].copy_(ct.data)
            else:
                c.nj_drop_level(ct, 1, Ct(x.data[k], 1))
        x.scale = xs[0].scale
        y = c.empty_batch(bo, 0)
        self.timed("Conv2d", lambda: c.nj_conv2d_block(plan, x, y))
        return [Ct(y.data[k], 0, scale=y.scale) for k in range(bo)]

    def add(self, ys, zs):
        c = self.c
        outs = []
        for y, z in zip(ys, zs):
            o = c.empty_ct(0)
            self.timed("ETC", lambda: c.nj_add(y, z, o))
            outs.append(o)
        return outs

    def bootstrap(self, ys, W, C, w0, act, decompose):
        """level-0 conv outputs -> CinS inputs of the next layer (level 1)"""
        c, L = self.c, self.c.L
        lo = L - 3
        mre, mim = self.mask(W, C, w0)
        dec = self.dec_plans(W, C) if decompose else None
        st1 = self.stoc1_plan(W // 2 if decompose else W)
        outs = []
        for y in ys:
            re, im = c.empty_ct(lo), c.empty_ct(lo)
            self.timed("CtoS+ModEval", lambda: c.nj_coeff_to_slot(self.g.cts_plan, y, re, im))
            halves = []
            for part, mk in ((re, mre), (im, mim)):
                e = c.empty_ct(LVL_MASK)
                self.timed("CtoS+ModEval", lambda: c.nj_eval_mod(part, K_MOD, R_DA, None, e))
                t, m = c.empty_ct(LVL_MASK), c.empty_ct(LVL_MASK - 1)

                def masked():
                    c.nj_pmult(e, mk, t)
                    t.scale = e.scale * float(self.g.q[LVL_MASK])  # masks encoded at q_l keep the scale
                    return c.nj_rescale(t, m)
                self.timed("Activation", masked)
                if act:
                    sq = c.empty_ct(LVL_MASK - 2)
                    self.timed("Activation", lambda: c.nj_hmult(m, m, sq))
                else:
                    sq = c.empty_ct(LVL_MASK - 2)
                    c.nj_drop_level(m, LVL_MASK - 2, sq)
                if dec is not None:
                    d = c.empty_ct(LVL_DEC - 1)
                    self.timed("Decomp", lambda: c.nj_conv2d_cins(dec[len(halves)], sq, d))
                    sq = d
                halves.append(sq)
            z = c.empty_ct(halves[0].level)
            self.timed("StoC", lambda: c.nj_combine(halves[0], halves[1], z))
            if z.level > LVL_STOC:
                zz = c.empty_ct(LVL_STOC)
                c.nj_drop_level(z, LVL_STOC, zz)
                z = zz
            out = c.empty_ct(LVL_STOC - 3)
            self.timed("StoC", lambda: c.nj_stoc1(st1, z, out))
            outs.append(out)
        self.counts["bootstraps"] = self.counts.get("bootstraps", 0) + len(ys)
        return outs

    # ------------------------------------------------------------ the network
    def build(self):
        """plans of every layer (timed separately from inference)"""
        P = {}
        P["conv1"] = self.conv_plan(224, self.weights((64, 3, 7, 7), 49 * 3), stride=2)
        P["pool"] = self.conv_plan(112, np.full((64, 3, 3), 1.0 / 9.0), stride=2, depthwise=True)
        for s, (ch, w0) in enumerate(((64, 56), (128, 28), (256, 14), (512, 7))):
            ci = 64 if s == 0 else ch // 2
            win = w0 if s == 0 else 2 * w0
            if s == 0:
                P["s0b0a"] = self.conv_plan(w0, self.weights((ch, ci, 3, 3), 9 * ci))
            else:
                P["s%db0a" % s] = self.conv_plan(win, self.weights((ch, ci, 3, 3), 9 * ci), stride=2)
                P["s%dsc" % s] = self.conv_plan(win, self.weights((ch, ci, 1, 1), ci), stride=2)
            P["s%db0b" % s] = self.conv_plan(w0, self.weights((ch, ch, 3, 3), 9 * ch))
            P["s%db1a" % s] = self.conv_plan(w0, self.weights((ch, ch, 3, 3), 9 * ch))
            P["s%db1b" % s] = self.conv_plan(w0, self.weights((ch, ch, 3, 3), 9 * ch))
            P["s%did" % s] = self.conv_plan(w0, np.ones((ch, 1, 1)), depthwise=True)
        self.P = P
        # keys of every rotation the plans, StoC1, the decompositions and CoeffToSlot use
        for W, C in ((128, 4), (64, 16), (32, 64), (16, 256)):
            self.dec_plans(W, C)
        for W in (64, 32, 16, 8):
            self.stoc1_plan(W)
        gs = set(self.g.cts_plan.galois())
        for p in list(P.values()) + list(self.stoc1.values()) + [d for v in self.dec.values() for d in v]:
            gs |= set(p.galois())
        self.g.make_keys(sorted(gs))
        return len(gs)

    def input_cts(self):
        """the client's encryption: the input's phase images (12 channels at 112 x 112,
        W = 128, C = 4: three ciphertexts) in real CinS at level 1"""
        c = self.c
        img = synth.uniform_real((3, 224, 224), self.seed, 0)
        ph = np.zeros((12, 112, 112))
        for i in range(3):
            for a in (0, 1):
                for b in (0, 1):
                    ph[4 * i + 2 * b + a] = img[i, a::2, b::2]
        W, C = 128, 4
        outs = []
        for k in range(3):
            ch = np.zeros((C, W, W))
            ch[:, :112, :112] = ph[4 * k:4 * k + 4]
            coeffs = c.nj_encode_cins(ch.reshape(C, W * W), self.g.scale)
            m = self.torch.empty((2, self.N), dtype=self.torch.int64, device=c.device)
            c.nj_upload_plain(coeffs, 1, m)
            a, e = synth.enc_randomness(self.g.q[:2], self.N, self.seed, 100 + k)
            outs.append(c.nj_encrypt_sk(m, 1, a, e, self.g.scale, c.empty_ct(1)))
        return outs

    def infer(self, xs):
        P = self.P
        self.times, self.counts = {}, {}
        # stem: conv1 (W = 128, C = 4 outputs: 16 ciphertexts), decomposed for the pooling
        y = self.conv(P["conv1"], xs)
        x = self.bootstrap(y, 128, 4, 112, act=True, decompose=True)
        y = self.conv(P["pool"], x)  # 3x3/2 average pooling: 56 x 56, 4 ciphertexts
        x = self.bootstrap(y, 64, 16, 56, act=False, decompose=False)
        for s, (ch, w0) in enumerate(((64, 56), (128, 28), (256, 14), (512, 7))):
            W = padded(w0, 1)
            C = self.N // (W * W)
            # block 0
            if s == 0:
                h = self.bootstrap(self.conv(P["s0b0a"], x), W, C, w0, act=True, decompose=False)
                sc = self.conv(P["s0id"], x)
            else:
                h = self.bootstrap(self.conv(P["s%db0a" % s], x), W, C, w0, act=True, decompose=False)
                sc = self.conv(P["s%dsc" % s], x)
            x = self.bootstrap(self.add(self.conv(P["s%db0b" % s], h), sc), W, C, w0, act=True, decompose=False)
            # block 1; the last bootstrapping of a stage decomposes for the next stride-2 layer
            h = self.bootstrap(self.conv(P["s%db1a" % s], x), W, C, w0, act=True, decompose=False)
            sc = self.conv(P["s%did" % s], x)
            x = self.bootstrap(self.add(self.conv(P["s%db1b" % s], h), sc), W, C, w0, act=True, decompose=s < 3)
        return x


def summary(res, command):
    rows = ["CtoS+ModEval", "StoC", "Conv2d", "Activation", "Decomp", "ETC"]
    lines = ["# ResNet-18-shaped network at N = 2^16, end to end (Table 2 analog, timing only)", "",
             "Command (repository root): `%s`" % command, "",
             "One MI355X; 224 x 224 x 3 synthetic input, synthetic weights; every conv fused with StoC2, every "
             "output ciphertext bootstrapped (Algorithm 1), stride-2 layers by the decomposed flow (Algorithm 2). "
             "HIP-event time per library call, summed by Table 2's rows.", "",
             "| phase | seconds | calls |", "|---|---|---|"]
    for r in rows:
        lines.append("| %s | %.3f | %d |" % (r, res["ms_by_phase"].get(r, 0.0) / 1e3, res["calls"].get(r, 0)))
    lines += ["| **total** | **%.3f** | |" % (res["ms"] / 1e3), "",
              "Bootstrapped ciphertexts: %d.  Wall time of the inference (host included): %.3f s.  Setup (plans of "
              "%d layers, %d rotation keys): %.1f s.  The paper's NeuJeans ResNet18-AESPA total on an A100 with "
              "HEaaN is 5.35 s (Table 2; context, different hardware and library)."
              % (res["bootstraps"], res["wall_ms"] / 1e3, res["layers"], res["keys"], res["setup_s"])]
    return "\n".join(lines) + "\n"


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--out", required=True)
    ap.add_argument("--md", default=None)
    ap.add_argument("--runs", type=int, default=2, help="inferences (the first warms up)")
    args = ap.parse_args()
    t0 = time.time()
    net = Net()
    nk = net.build()
    xs = net.input_cts()
    setup = time.time() - t0
    print("[network] setup %.1f s, %d keys" % (setup, nk), flush=True)
    res = None
    for r in range(args.runs):
        net.torch.cuda.synchronize()
        t1 = time.perf_counter()
        out = net.infer(xs)
        net.torch.cuda.synchronize()
        wall = (time.perf_counter() - t1) * 1e3
        res = {"ms_by_phase": dict(net.times), "calls": dict(net.counts), "ms": sum(net.times.values()),
               "wall_ms": wall, "bootstraps": net.counts.get("bootstraps", 0), "outputs": len(out),
               "output_level": out[0].level, "layers": len(net.P), "keys": nk, "setup_s": setup}
        print("[network] run %d: %.3f s in the calls, %.3f s wall, %d bootstraps" %
              (r, res["ms"] / 1e3, wall / 1e3, res["bootstraps"]), flush=True)
    with open(args.out, "w") as fh:
        json.dump(res, fh, indent=1)
    if args.md:
        with open(args.md, "w") as fh:
            fh.write(summary(res, "python -m paper_2312_04356_amd.network --out gpurun_out/resnet18.json --md "
                                  "gpurun_out/resnet18_e2e_n65536.md"))


if __name__ == "__main__":
    main()
