"""Plan selection study at N = 2^16: time BSGS transforms of many structures (random
diagonals, timing keys), train the latency model on the GPU, and compare its choice of
baby-step count n1 with exhaustive timing and the default n1 = ceil(sqrt(#diagonals))
on the 20 convolutions of a ResNet-18-shaped network (224 x 224 input).

    python -m paper_2312_04356_amd.tune --out gpurun_out/tune.json [--samples 5000]

Every timing runs in libneujeans (nj_time_plan); the model is trained and evaluated
by its HIP kernels (nj_mlp_*).  Layers are described by the structure their fused
conv transform has in the library's layout: C = N / W^2 channels per ciphertext
(all C diagonals after fusing StoC2), bi input and bo output ciphertexts.
"""
import argparse
import json
import math
import time

import numpy as np

from . import Ctx, Mlp, chain_primes

LOG_N, N_Q, ALPHA = 16, 24, 8

# (name, C, bi, bo): conv1 7x7/2 on the 12 polyphase channels of the 3-channel
# 224 x 224 input (W = 128); 3x3 at 56 (W = 64); each stage: 3x3/2 on polyphase inputs,
# 3x3, 1x1/2 downsample (only the (0, 0) phase is read), 2 x 3x3
RESNET18 = ([("conv1 7x7/2 3->64", 4, 3, 16)] + [("3x3 64@56 #%d" % i, 16, 4, 4) for i in range(4)] +
            [("3x3/2 64->128", 64, 4, 2), ("3x3 128@28", 64, 2, 2), ("1x1/2 64->128", 64, 1, 2),
             ("3x3 128@28 #2", 64, 2, 2), ("3x3 128@28 #3", 64, 2, 2),
             ("3x3/2 128->256", 256, 2, 1), ("3x3 256@14", 256, 1, 1), ("1x1/2 128->256", 256, 1, 1),
             ("3x3 256@14 #2", 256, 1, 1), ("3x3 256@14 #3", 256, 1, 1),
             ("3x3/2 256->512", 1024, 1, 1), ("3x3 512@7", 1024, 1, 1), ("1x1/2 256->512", 1024, 1, 1),
             ("3x3 512@7 #2", 1024, 1, 1), ("3x3 512@7 #3", 1024, 1, 1)])
EVAL_LEVEL = 1


def pow2_upto(c):
    return [1 << k for k in range(int(math.log2(c)) + 1)]


def conv_offsets(C):
    return list(range(C))


def log(msg):
    print(msg, flush=True)


class Timer:
    def __init__(self, ctx, reps):
        self.ctx, self.reps, self.cache = ctx, reps, {}

    def conv(self, C, n1, bi, bo, level):
        key = ("conv", C, n1, bi, bo, level)
        if key not in self.cache:
            n = (1 << LOG_N) // 2
            plan = self.ctx.nj_plan_create_random(level, n // C, conv_offsets(C), n1, bi, bo, seed=len(self.cache))
            self.cache[key] = (plan.features(level), self.ctx.nj_time_plan(plan, level, reps=self.reps))
            del plan
        return self.cache[key]

    def transform(self, u, offsets, n1, level, tag):
        key = ("lt", tag, n1, level)
        if key not in self.cache:
            plan = self.ctx.nj_plan_create_random(level, u, offsets, n1, 1, 1, seed=len(self.cache))
            self.cache[key] = (plan.features(level), self.ctx.nj_time_plan(plan, level, reps=self.reps))
            del plan
        return self.cache[key]


def plan_bytes(C, bi, bo, level):
    return bi * bo * C * (level + 1) * (1 << LOG_N) * 8


def sample_configs(rng, n, held_out):
    """random (C, n1, bi, bo, level) conv structures, at most 4 GB of diagonals"""
    shapes = [(1, 1), (1, 2), (2, 1), (2, 2), (4, 2), (4, 4), (3, 16), (2, 4)]
    out, seen = [], set()
    tries = 0
    while len(out) < n and tries < 50 * n:
        tries += 1
        C = int(rng.choice([4, 16, 64, 256, 1024]))
        n1 = int(rng.choice(pow2_upto(C)))
        bi, bo = shapes[rng.integers(len(shapes))]
        level = int(rng.integers(1, N_Q))
        if plan_bytes(C, bi, bo, level) > 4e9 or bi * bo * C > 4096:
            continue
        key = (C, n1, bi, bo, level)
        if key in seen or (level == EVAL_LEVEL and (C, bi, bo) in held_out):
            continue
        seen.add(key)
        out.append(key)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--out", required=True)
    ap.add_argument("--samples", type=int, default=5000)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--epochs", type=int, default=300)
    ap.add_argument("--seed", type=int, default=1005)
    args = ap.parse_args()
    t0 = time.time()
    q, p = chain_primes(LOG_N, N_Q, ALPHA, 50, 48, 50)
    ctx = Ctx(LOG_N, q, p, 2.0 ** 40)
    ctx.nj_timing_keys(16)
    timer = Timer(ctx, args.reps)
    rng = np.random.default_rng(args.seed)
    held_out = {(C, bi, bo) for _, C, bi, bo in RESNET18}
    # CoeffToSlot stage groups (3 groups) as extra structures for training
    cts = ctx.nj_cts_plan_create(3)
    n = (1 << LOG_N) // 2
    cts_lts = []
    for t in range(cts.count()):
        f = cts.features(ctx.L - t, t)
        cts_lts.append((n >> int(f[1]), cts.offsets(t)))
    del cts
    configs = sample_configs(rng, args.samples, held_out)
    log("[tune] %d conv structures to time" % len(configs))
    X, y = [], []
    for i, (C, n1, bi, bo, level) in enumerate(configs):
        f, ms = timer.conv(C, n1, bi, bo, level)
        X.append(f), y.append(math.log(ms))
        if (i + 1) % 250 == 0:
            log("[tune] timed %d / %d (%.0f s)" % (i + 1, len(configs), time.time() - t0))
    for g, (u, offs) in enumerate(cts_lts):
        for n1 in pow2_upto(64):
            for level in range(ctx.L - 2, ctx.L + 1):
                f, ms = timer.transform(u, offs, n1, level, "cts%d" % g)
                X.append(f), y.append(math.log(ms))
    X, y = np.array(X, dtype=np.float32), np.array(y, dtype=np.float32)
    log("[tune] %d timings in %.0f s" % (len(y), time.time() - t0))
    # model: 80 / 20 split for the held-out error, then the full set for selection
    perm = rng.permutation(len(y))
    cut = int(0.8 * len(y))
    m = Mlp(seed=args.seed)
    tr_loss = m.train(X[perm[:cut]], y[perm[:cut]], epochs=args.epochs, batch=256, lr=1e-3, seed=args.seed)
    pred = m.predict(X[perm[cut:]])
    rel = np.abs(np.exp(pred - y[perm[cut:]]) - 1.0)
    log("[tune] held-out latency error: median %.1f%%, 90th pct %.1f%%" % (100 * np.median(rel),
                                                                         100 * np.percentile(rel, 90)))
    m = Mlp(seed=args.seed)
    full_loss = m.train(X, y, epochs=args.epochs, batch=256, lr=1e-3, seed=args.seed)
    # per layer: every candidate n1 timed (exhaustive), the model's pick, the default
    layers = []
    tot = {"default": 0.0, "mlp": 0.0, "best": 0.0}
    for name, C, bi, bo in RESNET18:
        cands = pow2_upto(C)
        meas = {n1: timer.conv(C, n1, bi, bo, EVAL_LEVEL) for n1 in cands}
        feats = np.array([meas[n1][0] for n1 in cands], dtype=np.float32)
        ms = {n1: meas[n1][1] for n1 in cands}
        guess = dict(zip(cands, np.exp(m.predict(feats))))
        best = min(cands, key=lambda k: ms[k])
        pick = min(cands, key=lambda k: guess[k])
        dflt_n1 = int(math.ceil(math.sqrt(C)))
        dflt = timer.conv(C, dflt_n1, bi, bo, EVAL_LEVEL)[1]
        layers.append({"layer": name, "C": C, "bi": bi, "bo": bo, "default_n1": dflt_n1, "default_ms": dflt,
                       "best_n1": best, "best_ms": ms[best], "mlp_n1": pick, "mlp_ms": ms[pick],
                       "mlp_predicted_ms": float(guess[pick]), "candidates": {str(k): ms[k] for k in cands}})
        tot["default"] += dflt
        tot["mlp"] += ms[pick]
        tot["best"] += ms[best]
        log("[tune] %-18s C=%4d %dx%-2d default n1=%-3d %.3f ms | best n1=%-4d %.3f ms | model n1=%-4d %.3f ms"
            % (name, C, bi, bo, dflt_n1, dflt, best, ms[best], pick, ms[pick]))
    # CoeffToSlot depth: d stage groups (d levels), each group's transform timed at its
    # level with the library's default split; the model predicts the sum
    cts_d = []
    for d in (2, 3, 4, 5):
        plan = ctx.nj_cts_plan_create(d)
        feats = np.array([plan.features(ctx.L - t, t) for t in range(d)], dtype=np.float32)
        meas = sum(ctx.nj_time_plan(plan, ctx.L - t, t=t, reps=args.reps) for t in range(d))
        guess = float(np.exp(m.predict(feats)).sum())
        cts_d.append({"groups": d, "levels_used": d, "measured_ms": meas, "predicted_ms": guess,
                      "diagonals": [int(f[2]) for f in feats]})
        log("[tune] CoeffToSlot d=%d: measured %.3f ms, model %.3f ms, diagonals %s"
            % (d, meas, guess, [int(f[2]) for f in feats]))
        del plan
    ctx.nj_timing_keys(0)
    report = {"cts_depth": cts_d, "ring": {"log_n": LOG_N, "n_q": N_Q, "alpha": ALPHA}, "eval_level": EVAL_LEVEL,
              "n_timings": int(len(y)), "train_mse_std_units": tr_loss, "full_train_mse_std_units": full_loss,
              "heldout_rel_err_median": float(np.median(rel)), "heldout_rel_err_p90": float(np.percentile(rel, 90)),
              "totals_ms": tot, "mlp_vs_best": tot["mlp"] / tot["best"], "default_vs_best": tot["default"] / tot["best"],
              "layers": layers, "seconds": time.time() - t0}
    with open(args.out, "w") as fh:
        json.dump(report, fh, indent=1)
    log("[tune] totals: default %.2f ms, model %.2f ms, exhaustive best %.2f ms (model/best %.3f, default/best %.3f)"
        % (tot["default"], tot["mlp"], tot["best"], report["mlp_vs_best"], report["default_vs_best"]))


if __name__ == "__main__":
    main()
