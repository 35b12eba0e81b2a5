"""A ResNet-18-shaped network on a 224 x 224 x 3 input, end to end through the library at
N = 2^16 (the analog of Table 2's NeuJeans column with synthetic weights): the time of
every phase, and the decrypted output against the same network computed in FP64.

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
on the same phase images as the block's first conv.  Weights U(-1, 1) (synthetic, seed
1005), each conv's (and each shortcut's) scaled so that its output on this input has rms
0.2 (the role BN folding plays in a trained network); input U(-1, 1).  Phases are timed by HIP events around each
library call (one call at a time), in Table 2's rows.

    python -m paper_2312_04356_amd.network --out results/resnet18.json [--md results/resnet18.md]
"""
import argparse
import json
import math
import sys
import time

import numpy as np

import synth

from . import Ct, nj_layer_masks
from .workload import GpuWorkload

K_MOD, R_DA = 32, 3
RMS_OUT = 0.2    # rms of every conv's output on the input (weights scaled to it)
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

    def mask(self, W, C, w0, r):
        """Algorithm 1's zero-padding masks times r (the scale correction below)"""
        key = (W, C, w0, r)
        if key not in self.masks:
            c, pts = self.c, []
            for mk in nj_layer_masks(N_LOG, W, C, w0):
                t = self.torch.empty((LVL_MASK + 1, self.N), dtype=self.torch.int64, device=c.device)
                c.nj_upload_plain(c.nj_encode_slots(r * mk, float(self.g.q[LVL_MASK])), LVL_MASK, t)
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

    def calib(self, K, x, stride=1, depthwise=False):
        """K scaled so that its conv's FP64 output on x has rms RMS_OUT (the role BN
        folding plays in a trained network: square activations neither vanish nor blow
        up), and that output"""
        z = conv_fp64(x, K, stride, depthwise)
        g = RMS_OUT / np.sqrt(np.mean(z ** 2))
        return K * g, z * g

    def layer(self, name, w0, K, B, stride=1, depthwise=False):
        """the plan of a conv whose output (or the residual sum it enters) is bounded by
        B: the weights are divided by B, which the masks after ModEval restore (Algorithm
        1), so ModEval sees |m / B| <= 1"""
        self.P[name] = self.conv_plan(w0, K / B, stride, depthwise)
        self.K[name] = (K, stride, depthwise)

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

    def bootstrap(self, ys, W, C, w0, act, decompose, B=1.0):
        """level-0 conv outputs -> CinS inputs of the next layer (level 1).  ModEval's
        output scale is a fixed multiple of its input's, so each layer would drift the
        scale; the masks carry the correction instead: they are encoded times
        r = T' / (ModEval's scale) and the masked result is read at scale T', the scale
        from which the square (or, without activation, the level drop) lands on the
        input scale T.  Every layer then returns T, and a residual sum adds two
        ciphertexts at one scale.  The masks also carry B, the bound folded into the
        layer's weights."""
        c, L = self.c, self.c.L
        lo = L - 3
        T = self.g.scale
        T_pre = math.sqrt(T * float(self.g.q[LVL_MASK - 1])) if act else T
        dec = self.dec_plans(W, C) if decompose else None
        st1 = self.stoc1_plan(W // 2 if decompose else W)
        outs = []
        for y in ys:
            re, im = c.empty_ct(lo), c.empty_ct(lo)
            self.timed("CtoS+ModEval", lambda: c.nj_coeff_to_slot(self.g.cts_plan, y, re, im))
            halves = []
            for half, part in enumerate((re, im)):
                e = c.empty_ct(LVL_MASK)
                self.timed("CtoS+ModEval", lambda: c.nj_eval_mod(part, K_MOD, R_DA, None, e))
                mk = self.mask(W, C, w0, B * T_pre / e.scale)[half]
                t, m = c.empty_ct(LVL_MASK), c.empty_ct(LVL_MASK - 1)

                def masked():
                    c.nj_pmult(e, mk, t)
                    t.scale = e.scale * float(self.g.q[LVL_MASK])  # masks encoded at q_l keep the scale
                    return c.nj_rescale(t, m)
                self.timed("Activation", masked)
                m.scale = T_pre  # the integers hold value * mask * r * e.scale = value * mask * T_pre
                sq = c.empty_ct(LVL_MASK - 2)
                if act:
                    self.timed("Activation", lambda: c.nj_hmult(m, m, sq))
                    sq.scale = T  # T_pre^2 / q_l, equal to T up to the last bit of a double
                else:
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
        self.P, self.K, self.B = {}, {}, {}
        self.img = synth.uniform_real((3, 224, 224), self.seed, 0)

        def bound(z):
            return 2.0 ** math.ceil(math.log2(max(1.05 * float(np.max(np.abs(z))), 1e-3)))
        K, z = self.calib(self.weights((64, 3, 7, 7), 49 * 3), self.img, 2)
        self.B["conv1"] = bound(z)
        self.layer("conv1", 224, K, self.B["conv1"], stride=2)
        x = z ** 2
        K = np.full((64, 3, 3), 1.0 / 9.0)
        z = conv_fp64(x, K, 2, True)
        self.B["pool"] = bound(z)
        self.layer("pool", 112, K, self.B["pool"], stride=2, depthwise=True)
        x = z
        for s, (ch, w0) in enumerate(((64, 56), (128, 28), (256, 14), (512, 7))):
            ci = 64 if s == 0 else ch // 2
            win = w0 if s == 0 else 2 * w0
            st = 1 if s == 0 else 2
            # block 0: its shortcut is the identity kernel in stage 0, 1x1 stride 2 later
            Ka, za = self.calib(self.weights((ch, ci, 3, 3), 9 * ci), x, st)
            if s == 0:
                Ks, zs = self.calib(np.ones((ch, 1, 1)), x, 1, True)
            else:
                Ks, zs = self.calib(self.weights((ch, ci, 1, 1), ci), x, 2)
            Kb, zb = self.calib(self.weights((ch, ch, 3, 3), 9 * ch), za ** 2)
            self.B["s%db0a" % s], self.B["s%db0" % s] = bound(za), bound(zb + zs)
            self.layer("s%db0a" % s, win, Ka, self.B["s%db0a" % s], stride=st)
            self.layer("s%dsc" % s, win if s else w0, Ks, self.B["s%db0" % s], stride=st, depthwise=s == 0)
            self.layer("s%db0b" % s, w0, Kb, self.B["s%db0" % s])
            x = (zb + zs) ** 2
            # block 1: the identity kernel as shortcut
            Ka, za = self.calib(self.weights((ch, ch, 3, 3), 9 * ch), x)
            Ks, zs = self.calib(np.ones((ch, 1, 1)), x, 1, True)
            Kb, zb = self.calib(self.weights((ch, ch, 3, 3), 9 * ch), za ** 2)
            self.B["s%db1a" % s], self.B["s%db1" % s] = bound(za), bound(zb + zs)
            self.layer("s%db1a" % s, w0, Ka, self.B["s%db1a" % s])
            self.layer("s%did" % s, w0, Ks, self.B["s%db1" % s], depthwise=True)
            self.layer("s%db1b" % s, w0, Kb, self.B["s%db1" % s])
            x = (zb + zs) ** 2
        # the identity kernel fused with StoC2, unscaled: reads the last output back
        self.readout = self.conv_plan(7, np.ones((512, 1, 1)), depthwise=True)
        P = self.P
        # keys of every rotation the plans, StoC1, the decompositions and CoeffToSlot use
        for W, C in ((128, 4), (64, 16), (32, 64), (16, 256)):
            self.dec_plans(W, C)
        for W in (64, 32, 16, 8):
            self.stoc1_plan(W)
        gs = set(self.g.cts_plan.galois())
        for p in list(P.values()) + [self.readout] + list(self.stoc1.values()) + [d for v in self.dec.values()
                                                                                  for d in v]:
            gs |= set(p.galois())
        self.g.make_keys(sorted(gs))
        return len(gs)

    def input_cts(self):
        """the client's encryption: the input's phase images (12 channels at 112 x 112,
        W = 128, C = 4: three ciphertexts) in real CinS at level 1"""
        c = self.c
        img = self.img
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
        B = self.B
        y = self.conv(P["conv1"], xs)
        x = self.bootstrap(y, 128, 4, 112, act=True, decompose=True, B=B["conv1"])
        y = self.conv(P["pool"], x)  # 3x3/2 average pooling: 56 x 56, 4 ciphertexts
        x = self.bootstrap(y, 64, 16, 56, act=False, decompose=False, B=B["pool"])
        for s, (ch, w0) in enumerate(((64, 56), (128, 28), (256, 14), (512, 7))):
            W = padded(w0, 1)
            C = self.N // (W * W)
            # block 0
            h = self.bootstrap(self.conv(P["s%db0a" % s], x), W, C, w0, act=True, decompose=False,
                               B=B["s%db0a" % s])
            sc = self.conv(P["s%dsc" % s], x)
            x = self.bootstrap(self.add(self.conv(P["s%db0b" % s], h), sc), W, C, w0, act=True, decompose=False,
                               B=B["s%db0" % s])
            # block 1; the last bootstrapping of a stage decomposes for the next stride-2 layer
            h = self.bootstrap(self.conv(P["s%db1a" % s], x), W, C, w0, act=True, decompose=False,
                               B=B["s%db1a" % s])
            sc = self.conv(P["s%did" % s], x)
            x = self.bootstrap(self.add(self.conv(P["s%db1b" % s], h), sc), W, C, w0, act=True, decompose=s < 3,
                               B=B["s%db1" % s])
        return x


def conv_fp64(x, K, stride=1, depthwise=False):
    """'same' zero-padded cross-correlation with the given stride (output width
    ceil(w / stride)), K [c_out][c_in][f][f] or depthwise [c][f][f], in FP64"""
    f = K.shape[-1]
    p = (f - 1) // 2
    ci, w, _ = x.shape
    wo = (w + stride - 1) // stride
    xp = np.pad(x, ((0, 0), (p, p), (p, p)))
    taps = [xp[:, u:u + stride * wo:stride, v:v + stride * wo:stride] for u in range(f) for v in range(f)]
    if depthwise:
        return sum(K[:, u, v, None, None] * taps[u * f + v] for u in range(f) for v in range(f))
    cols = np.stack(taps, axis=1).reshape(ci * f * f, wo * wo)
    return (K.reshape(K.shape[0], ci * f * f) @ cols).reshape(K.shape[0], wo, wo)


def forward_fp64(net):
    """the network in FP64 on the same input and weights: conv, square, the pooling,
    the residual sums, as the homomorphic inference computes them"""
    def cv(name, x):
        K, stride, dw = net.K[name]
        return conv_fp64(x, K, stride, dw)
    x = cv("conv1", net.img) ** 2
    x = cv("pool", x)
    for s in range(4):
        h = cv("s%db0a" % s, x) ** 2
        sc = cv("s%dsc" % s, x)
        x = (cv("s%db0b" % s, h) + sc) ** 2
        h = cv("s%db1a" % s, x) ** 2
        x = (cv("s%db1b" % s, h) + cv("s%did" % s, x)) ** 2
    return x


def decode_output(net, xs):
    """the last layer's output (512 channels at 7 x 7) brought to coefficient layout by
    the identity plan fused with StoC2, decrypted and read at (y W + x) C + rev_C(c)"""
    c = net.c
    ys = net.conv(net.readout, xs)
    _, W, C, _, _, _ = net.readout.layout()
    bits = C.bit_length() - 1
    rev = np.array([int(format(k, "0%db" % bits)[::-1], 2) for k in range(C)])
    q0 = float(net.g.q[0])
    out = []
    for k, y in enumerate(ys):
        d = net.torch.empty((1, net.N), dtype=net.torch.int64, device=c.device)
        c.nj_decrypt(y, d)
        v = c.to_host(d)[0].astype(np.float64)
        v[v > q0 / 2] -= q0
        v /= y.scale
        idx = (np.arange(7)[:, None] * W + np.arange(7)[None, :])[None] * C + rev[:, None, None]
        out.append(v[idx])
    return np.concatenate(out)[:512]


def summary(res, command):
    rows = ["CtoS+ModEval", "StoC", "Conv2d", "Activation", "Decomp", "ETC"]
    lines = ["# ResNet-18-shaped network at N = 2^16, end to end (Table 2 analog, synthetic weights)", "",
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
    if "output_vs_fp64" in res:
        e = res["output_vs_fp64"]
        lines += ["", "The decrypted output of the last layer (512 channels at 7 x 7) against the same network "
                  "computed in FP64 (same input and weights, square activations, 'same' strided convs, average "
                  "pooling, residual sums): max abs error %.2e (rms %.2e) for values up to %.3f (rms %.3f)."
                  % (e["max_abs_err"], e["rms_err"], e["max_abs_value"], e["rms_value"])]
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
    got = decode_output(net, out)
    want = forward_fp64(net)
    res["output_vs_fp64"] = {"max_abs_err": float(np.max(np.abs(got - want))),
                             "rms_err": float(np.sqrt(np.mean((got - want) ** 2))),
                             "max_abs_value": float(np.max(np.abs(want))),
                             "rms_value": float(np.sqrt(np.mean(want ** 2)))}
    print("[network] output (512 x 7 x 7) vs the FP64 forward pass: max abs error %.2e, max |value| %.3f" %
          (res["output_vs_fp64"]["max_abs_err"], res["output_vs_fp64"]["max_abs_value"]), flush=True)
    with open(args.out, "w") as fh:
        json.dump(res, fh, indent=1)
    if args.md:
        with open(args.md, "w") as fh:
            fh.write(summary(res, "python -m paper_2312_04356_amd.network " + " ".join(sys.argv[1:])))


if __name__ == "__main__":
    main()
