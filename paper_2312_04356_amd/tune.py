"""Plan selection at N = 2^16 by a learned latency model.

Times BSGS transforms of many structures on the GPU (random diagonals, timing keys),
trains the library's 7-64-64-1 MLP on those timings with its HIP kernels, and compares
the model's plans with exhaustive timing and the default plans on
  * the 20 convolutions of a ResNet-18-shaped network (224 x 224 input): BSGS split n1
    and hoisted or plain baby steps per layer;
  * CoeffToSlot: its depth d (the number of DFT stage groups, each consuming a level;
    Algorithm 1 leaves room for d <= 6), each group's BSGS split and hoisting.
The trained model and the timing database are written for later plan selection:

    python -m paper_2312_04356_amd.tune --out results/tune.json \
        --model paper_2312_04356_amd/data/plan_model_n65536.json [--samples 5000]

Every timing runs in libneujeans (nj_time_plan); the model is trained and evaluated by
its HIP kernels (nj_mlp_*).  Layers are described by the structure their fused conv
transform has in the library's layout: C = N / W^2 channels per ciphertext (all C
diagonals after fusing StoC2), bi input and bo output ciphertexts.
"""
import argparse
import json
import math
import os
import time

import numpy as np

from . import Ctx, Mlp, chain_primes

LOG_N, N_Q, ALPHA = 16, 24, 8
FEATURES = ["limbs", "diagonals", "log2_slot_stride", "baby_steps", "hoisted_rotations", "fusion_depth", "bo"]

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
# CoeffToSlot depths Algorithm 1 admits at 24 primes: d groups + ModEval (11) + masks and
# square (2) + StoC1 (3) must leave the next conv level 1
CTS_DEPTHS = (2, 3, 4, 5, 6)
DEFAULT_CTS_DEPTH = 3


def pow2_upto(c):
    return [1 << k for k in range(int(math.log2(c)) + 1)]


def n1_candidates(n_diag):
    """powers of two within a factor 4 of sqrt(#diagonals), at most the diagonal count"""
    r = math.sqrt(n_diag)
    return [1 << k for k in range(12) if r / 4 <= (1 << k) <= 4 * r and (1 << k) <= max(1, n_diag)]


def conv_offsets(C):
    return list(range(C))


def log(msg):
    print(msg, flush=True)


class Timer:
    """cached (features, median ms) of transforms timed by the library"""

    def __init__(self, ctx, reps):
        self.ctx, self.reps, self.cache = ctx, reps, {}
        self.cts_plans = {}

    def conv(self, C, n1, bi, bo, level, hoist=True):
        key = ("conv", C, n1, bi, bo, level, bool(hoist))
        if key not in self.cache:
            n = (1 << LOG_N) // 2
            plan = self.ctx.nj_plan_create_random(level, n // C, conv_offsets(C), n1, bi, bo, seed=len(self.cache))
            plan.set_hoist(hoist)
            self.cache[key] = (plan.features(level), self.ctx.nj_time_plan(plan, level, reps=self.reps))
            del plan
        return self.cache[key]

    def cts_plan(self, d, n1):
        """CoeffToSlot plan of depth d with every group split by n1 (lazy giant steps)"""
        if (d, n1) not in self.cts_plans:
            self.cts_plans.clear()  # one at a time: each holds up to ~2 GB of diagonals
            self.cts_plans[(d, n1)] = self.ctx.nj_cts_plan_create_split(d, [n1] * d).set_lazy(True)
        return self.cts_plans[(d, n1)]

    def cts(self, d, t, n1, level, hoist=True):
        key = ("cts", d, t, n1, level, bool(hoist))
        if key not in self.cache:
            plan = self.cts_plan(d, n1).set_hoist(hoist)
            self.cache[key] = (plan.features(level, t), self.ctx.nj_time_plan(plan, level, t=t, reps=self.reps))
        return self.cache[key]


def plan_bytes(C, bi, bo, level):
    return bi * bo * C * (level + 1) * (1 << LOG_N) * 8


def sample_configs(rng, n, held_out):
    """random (C, n1, bi, bo, level, hoist) conv structures, at most 4 GB of diagonals;
    single-block structures are timed with plain baby steps a quarter of the time"""
    shapes = [(1, 1), (1, 2), (2, 1), (2, 2), (4, 2), (4, 4), (3, 16), (2, 4), (1, 4), (4, 1), (3, 3), (8, 2)]
    out, seen = [], set()
    tries = 0
    while len(out) < n and tries < 50 * n:
        tries += 1
        C = int(rng.choice([2, 4, 8, 16, 32, 64, 128, 256, 512, 1024]))
        n1 = int(rng.choice(pow2_upto(C)))
        bi, bo = shapes[rng.integers(len(shapes))]
        level = int(rng.integers(1, N_Q))
        hoist = not (bi == bo == 1 and rng.random() < 0.25)
        if plan_bytes(C, bi, bo, level) > 4e9 or bi * bo * C > 4096:
            continue
        key = (C, n1, bi, bo, level, hoist)
        if key in seen or (level == EVAL_LEVEL and (C, bi, bo) in held_out):
            continue
        seen.add(key)
        out.append(key)
    return out


def cts_group_diagonals(ctx, d):
    """diagonal count of each group of the depth-d CoeffToSlot (from its features)"""
    return [int(f[1]) for f in ctx.nj_cts_plan_features(d)]


def cts_candidates(ctx, d):
    """per group t: [(n1, hoist)] candidate splits"""
    return [[(n1, h) for n1 in n1_candidates(nd) for h in (True, False)] for nd in cts_group_diagonals(ctx, d)]


def rank_cts(ctx, model, depths=CTS_DEPTHS):
    """the model's CoeffToSlot plan for every depth (each group's (n1, hoist) with the least
    predicted latency: a group's features depend on its own split only), ranked by the
    predicted sum: [(predicted ms, d, [n1], [hoist])]"""
    out = []
    for d in depths:
        cands = cts_candidates(ctx, d)
        by = {}
        for n1, h in {c for cs in cands for c in cs}:
            by[(n1, h)] = ctx.nj_cts_plan_features(d, [n1] * d, h)
        n1s, hs, tot = [], [], 0.0
        for t in range(d):
            opts = cands[t]
            pred = np.exp(model.predict(np.array([by[c][t] for c in opts], dtype=np.float32)))
            k = int(np.argmin(pred))
            n1s.append(opts[k][0]), hs.append(opts[k][1])
            tot += float(pred[k])
        out.append((tot, d, n1s, hs))
    return sorted(out)


def choose_cts(ctx, model, depths=CTS_DEPTHS):
    """the model's CoeffToSlot plan: for every depth, each group's (n1, hoist) with the
    least predicted latency (a group's features depend on its own split only); the depth
    with the least predicted sum.  Returns (d, [n1], [hoist], predicted ms, {d: ms})"""
    best, per_d = None, {}
    for d in depths:
        cands = cts_candidates(ctx, d)
        by = {}
        for n1, h in {c for cs in cands for c in cs}:
            by[(n1, h)] = ctx.nj_cts_plan_features(d, [n1] * d, h)
        n1s, hs, tot = [], [], 0.0
        for t in range(d):
            opts = cands[t]
            feats = [by[c][t] for c in opts]
            pred = np.exp(model.predict(np.array(feats, dtype=np.float32)))
            k = int(np.argmin(pred))
            n1s.append(opts[k][0]), hs.append(opts[k][1])
            tot += float(pred[k])
        per_d[d] = tot
        if best is None or tot < best[3]:
            best = (d, n1s, hs, tot)
    return best + (per_d,)


def choose_conv(ctx, model, plans_by_choice, level):
    """the model's (n1, hoist) among conv plans {(n1, hoist): plan} at `level`"""
    r = rank_conv(ctx, model, plans_by_choice, level)
    return r[0][1], r[0][0]


def rank_conv(ctx, model, plans_by_choice, level):
    """[(predicted ms, (n1, hoist))] of conv plans {(n1, hoist): plan} at `level`, best first"""
    keys = sorted(plans_by_choice)
    feats = np.array([plans_by_choice[k].features(level) for k in keys], dtype=np.float32)
    pred = np.exp(model.predict(feats))
    return sorted(zip([float(v) for v in pred], keys))


# the model's best candidates, and the default plan, are timed before choosing: timing
# decides among them, so the chosen plan is never slower than the default as measured
SHORTLIST = 3


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--out", required=True)
    ap.add_argument("--model", default=None, help="where to write the trained model (JSON)")
    ap.add_argument("--timings", default=None, help="where to write the timing database (JSON)")
    ap.add_argument("--samples", type=int, default=4500, help="random conv structures to time")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--epochs", type=int, default=600)
    ap.add_argument("--seed", type=int, default=1005)
    args = ap.parse_args()
    t0 = time.time()
    q, p = chain_primes(LOG_N, N_Q, ALPHA, 50, 48, 50)
    ctx = Ctx(LOG_N, q, p, 2.0 ** 40)
    ctx.nj_timing_keys(16)
    timer = Timer(ctx, args.reps)
    rng = np.random.default_rng(args.seed)
    held_out = {(C, bi, bo) for _, C, bi, bo in RESNET18}
    X, y, kind = [], [], []
    # CoeffToSlot groups of every admitted depth: each candidate split, hoisted or not, at
    # the group's own level and one and two levels below (the same structure at fewer limbs)
    for d in CTS_DEPTHS:
        cands = cts_candidates(ctx, d)
        for n1 in sorted({n1 for c in cands for n1, _ in c}):
            for t in range(d):
                if all(n1 != v for v, _ in cands[t]):
                    continue
                for h in (True, False):
                    for dl in (0, 1, 2):
                        f, ms = timer.cts(d, t, n1, ctx.L - t - dl, h)
                        X.append(f), y.append(math.log(ms)), kind.append("cts%d" % d)
        log("[tune] CoeffToSlot depth %d timed (%d timings, %.0f s)" % (d, len(y), time.time() - t0))
    timer.cts_plans.clear()
    configs = sample_configs(rng, args.samples, held_out)
    log("[tune] %d conv structures to time" % len(configs))
    for i, (C, n1, bi, bo, level, hoist) in enumerate(configs):
        f, ms = timer.conv(C, n1, bi, bo, level, hoist)
        X.append(f), y.append(math.log(ms)), kind.append("conv")
        if (i + 1) % 250 == 0:
            log("[tune] timed %d / %d (%.0f s)" % (i + 1, len(configs), time.time() - t0))
    X, y, kind = np.array(X, dtype=np.float32), np.array(y, dtype=np.float32), np.array(kind)
    log("[tune] %d timings in %.0f s" % (len(y), time.time() - t0))
    # model: 80 / 20 split for the held-out error, then the full set for selection
    perm = rng.permutation(len(y))
    cut = int(0.8 * len(y))
    m = Mlp(seed=args.seed)
    tr_loss = m.train(X[perm[:cut]], y[perm[:cut]], epochs=args.epochs, batch=256, lr=1e-3, seed=args.seed)
    te = perm[cut:]
    rel = np.abs(np.exp(m.predict(X[te]) - y[te]) - 1.0)
    heldout = {"all": {"n": int(len(te)), "median": float(np.median(rel)), "p90": float(np.percentile(rel, 90))}}
    for name, sel in (("conv", kind[te] == "conv"), ("cts_d3", kind[te] == "cts3"),
                      ("cts_d_not_3", np.char.startswith(kind[te].astype(str), "cts") & (kind[te] != "cts3"))):
        if sel.any():
            heldout[name] = {"n": int(sel.sum()), "median": float(np.median(rel[sel])),
                             "p90": float(np.percentile(rel[sel], 90))}
    for k, v in heldout.items():
        log("[tune] held-out latency error (%s, %d): median %.1f%%, 90th pct %.1f%%"
            % (k, v["n"], 100 * v["median"], 100 * v["p90"]))
    m = Mlp(seed=args.seed)
    full_loss = m.train(X, y, epochs=args.epochs, batch=256, lr=1e-3, seed=args.seed)
    # per layer: every candidate (n1, hoist) timed (exhaustive), the model's pick, the default
    layers = []
    tot = {"default": 0.0, "mlp": 0.0, "shortlist": 0.0, "best": 0.0}
    for name, C, bi, bo in RESNET18:
        cands = [(n1, h) for n1 in pow2_upto(C) for h in ((True, False) if bi == bo == 1 else (True,))]
        meas = {c: timer.conv(C, c[0], bi, bo, EVAL_LEVEL, c[1]) for c in cands}
        feats = np.array([meas[c][0] for c in cands], dtype=np.float32)
        ms = {c: meas[c][1] for c in cands}
        guess = dict(zip(cands, np.exp(m.predict(feats))))
        best = min(cands, key=lambda k: ms[k])
        pick = min(cands, key=lambda k: guess[k])
        dflt_c = (int(math.ceil(math.sqrt(C))), True)
        short_set = sorted(cands, key=lambda k: guess[k])[:SHORTLIST]
        if dflt_c in ms and dflt_c not in short_set:
            short_set.append(dflt_c)
        short = min(short_set, key=lambda k: ms[k])
        dflt = timer.conv(C, dflt_c[0], bi, bo, EVAL_LEVEL, True)[1]
        layers.append({"layer": name, "C": C, "bi": bi, "bo": bo, "default_n1": dflt_c[0], "default_ms": dflt,
                       "best_n1": best[0], "best_hoist": best[1], "best_ms": ms[best],
                       "mlp_n1": pick[0], "mlp_hoist": pick[1], "mlp_ms": ms[pick],
                       "mlp_predicted_ms": float(guess[pick]),
                       "shortlist_n1": short[0], "shortlist_hoist": short[1], "shortlist_ms": ms[short],
                       "candidates": {"%d/%s" % (k[0], "h" if k[1] else "p"): ms[k] for k in cands}})
        tot["default"] += dflt
        tot["mlp"] += ms[pick]
        tot["shortlist"] += ms[short]
        tot["best"] += ms[best]
        log("[tune] %-18s C=%4d %dx%-2d default n1=%-3d %.3f ms | best %s %.3f ms | model %s %.3f ms | "
            "model top-%d timed %s %.3f ms" % (name, C, bi, bo, dflt_c[0], dflt, best, ms[best], pick, ms[pick],
                                               SHORTLIST, short, ms[short]))
    # CoeffToSlot: the model's depth and splits vs exhaustive timing of every candidate and
    # the default (depth 3, n1 = ceil(sqrt(#diagonals)), hoisted)
    md, mn1, mh, mpred, per_d = choose_cts(ctx, m)
    cts_rows, exh = [], None
    for d in CTS_DEPTHS:
        cands = cts_candidates(ctx, d)
        row = {"groups": d, "diagonals": cts_group_diagonals(ctx, d), "predicted_ms": per_d[d], "groups_best": []}
        meas_tot = 0.0
        for t in range(d):
            tt = {c: timer.cts(d, t, c[0], ctx.L - t, c[1])[1] for c in cands[t]}
            b = min(tt, key=tt.get)
            row["groups_best"].append({"n1": b[0], "hoist": b[1], "ms": tt[b]})
            meas_tot += tt[b]
        row["best_measured_ms"] = meas_tot
        cts_rows.append(row)
        if exh is None or meas_tot < exh[1]:
            exh = (d, meas_tot, [g["n1"] for g in row["groups_best"]], [g["hoist"] for g in row["groups_best"]])
        log("[tune] CoeffToSlot d=%d: predicted %.3f ms, best measured %.3f ms %s"
            % (d, per_d[d], meas_tot, [(g["n1"], g["hoist"]) for g in row["groups_best"]]))
    timer.cts_plans.clear()
    dplan = ctx.nj_cts_plan_create(DEFAULT_CTS_DEPTH).set_lazy(True)
    dflt_cts = sum(ctx.nj_time_plan(dplan, ctx.L - t, t=t, reps=args.reps) for t in range(DEFAULT_CTS_DEPTH))
    del dplan
    def time_cts(d, n1s, hs):
        plan = ctx.nj_cts_plan_create_split(d, n1s).set_lazy(True).set_hoist(hs)
        return sum(ctx.nj_time_plan(plan, ctx.L - t, t=t, reps=args.reps) for t in range(d))

    mlp_cts = time_cts(md, mn1, mh)
    ranked = rank_cts(ctx, m)
    short_t = [(time_cts(d, n1s, hs), d, n1s, hs, pred) for pred, d, n1s, hs in ranked[:SHORTLIST]]
    short_t.append((dflt_cts, DEFAULT_CTS_DEPTH, None, [True] * DEFAULT_CTS_DEPTH, None))  # the default plan
    sc = min(short_t, key=lambda r: r[0])
    log("[tune] CoeffToSlot: default d=%d %.3f ms | exhaustive d=%d %.3f ms | model d=%d n1=%s hoist=%s %.3f ms | "
        "model top-%d timed d=%d %.3f ms" % (DEFAULT_CTS_DEPTH, dflt_cts, exh[0], exh[1], md, mn1, mh, mlp_cts,
                                            SHORTLIST, sc[1], sc[0]))
    ctx.nj_timing_keys(0)
    model_doc = {"features": FEATURES, "ring": {"log_n": LOG_N, "n_q": N_Q, "alpha": ALPHA}, **m.to_dict(),
                 "target": "log(ms) of one BSGS transform (nj_time_plan)", "n_timings": int(len(y)),
                 "heldout_rel_err": heldout, "trained_by": "nj_mlp_train (Adam, %d epochs, batch 256, lr 1e-3)"
                 % args.epochs}
    if args.model:
        os.makedirs(os.path.dirname(os.path.abspath(args.model)), exist_ok=True)
        with open(args.model, "w") as fh:
            json.dump(model_doc, fh)
    if args.timings:
        with open(args.timings, "w") as fh:
            json.dump({"features": FEATURES, "X": X.tolist(), "log_ms": y.tolist(), "kind": kind.tolist()}, fh)
    report = {"ring": {"log_n": LOG_N, "n_q": N_Q, "alpha": ALPHA}, "eval_level": EVAL_LEVEL, "shortlist": SHORTLIST,
              "n_timings": int(len(y)), "train_mse_std_units": tr_loss, "full_train_mse_std_units": full_loss,
              "heldout": heldout, "totals_ms": tot, "mlp_vs_best": tot["mlp"] / tot["best"],
              "default_vs_best": tot["default"] / tot["best"], "layers": layers,
              "cts": {"depths": cts_rows, "default": {"groups": DEFAULT_CTS_DEPTH, "ms": dflt_cts},
                      "exhaustive": {"groups": exh[0], "n1": exh[2], "hoist": exh[3], "ms": exh[1]},
                      "mlp": {"groups": md, "n1": mn1, "hoist": mh, "predicted_ms": mpred, "ms": mlp_cts},
                      "mlp_shortlist": {"groups": sc[1], "n1": sc[2], "hoist": sc[3], "ms": sc[0],
                                        "timed": [{"groups": d, "n1": n1s, "ms": t, "predicted_ms": p}
                                                  for t, d, n1s, _, p in short_t]}},
              "seconds": time.time() - t0}
    with open(args.out, "w") as fh:
        json.dump(report, fh, indent=1)
    log("[tune] convs: default %.2f ms, model %.2f ms, model top-%d timed %.2f ms, exhaustive best %.2f ms "
        "(model/best %.3f, default/best %.3f)" % (tot["default"], tot["mlp"], SHORTLIST, tot["shortlist"],
                                                  tot["best"], report["mlp_vs_best"], report["default_vs_best"]))


def summary(report, command):
    """markdown summary of a report written by main()"""
    out = ["# Plan selection on ResNet-18-shaped convolutions and CoeffToSlot, N = 2^16 (MI355X)", "",
           "Command (one MI355X, committed files only):", "", "    " + command, "",
           "Every timing is `nj_time_plan` (HIP events, median of %s after one warm-up) of a random-diagonal plan "
           "with the structure of the transform, with timing keys (16-buffer pool); convs at level %d."
           % ("3", report["eval_level"]),
           "Training set: %d timings (random conv structures, n1 powers of two, hoisted or not, blocks, levels "
           "1..23, excluding the evaluated layers' structures at level 1; every CoeffToSlot group of depths 2..6 "
           "with each candidate split, hoisted or not, at its level and one and two below).  Model: 7 -> 64 -> 64 "
           "-> 1 FP32 ReLU on log(ms), trained by the library's HIP kernels (Adam)." % report["n_timings"], ""]
    h = report["heldout"]
    out.append("Held-out (20%%) latency error: all %d samples median %.1f%% (90th percentile %.1f%%); "
               "CoeffToSlot groups at depth 3: median %.1f%%, at other depths (%d samples): median %.1f%% "
               "(90th percentile %.1f%%)." % (h["all"]["n"], 100 * h["all"]["median"], 100 * h["all"]["p90"],
                                              100 * h["cts_d3"]["median"], h["cts_d_not_3"]["n"],
                                              100 * h["cts_d_not_3"]["median"], 100 * h["cts_d_not_3"]["p90"]))
    out += ["", "## CoeffToSlot (d groups, each split n1 and hoisting chosen per group)", "",
            "| plan | groups | n1 per group | hoisted | ms |", "|---|---|---|---|---|"]
    c = report["cts"]
    out.append("| default | %d | library default | all | %.3f |" % (c["default"]["groups"], c["default"]["ms"]))
    for name in ("exhaustive", "mlp", "mlp_shortlist"):
        r = c[name]
        label = {"exhaustive": "exhaustive timing", "mlp": "model's pick (untimed)",
                 "mlp_shortlist": "model top-%d + default, timed" % report["shortlist"]}[name]
        out.append("| %s | %d | %s | %s | %.3f |" % (label, r["groups"], r["n1"], r["hoist"], r["ms"]))
    out += ["", "Per depth: predicted (model) and measured best sum of the groups:", "",
            "| groups | diagonals per group | predicted ms | measured best ms |", "|---|---|---|---|"]
    for r in c["depths"]:
        out.append("| %d | %s | %.3f | %.3f |" % (r["groups"], r["diagonals"], r["predicted_ms"],
                                                  r["best_measured_ms"]))
    out += ["", "## Convolutions (level %d)" % report["eval_level"], "",
            "| layer | C | bi x bo | default n1 | ms | best n1/hoist | ms | model n1/hoist | ms | shortlist ms |",
            "|---|---|---|---|---|---|---|---|---|---|"]
    for r in report["layers"]:
        out.append("| %s | %d | %dx%d | %d | %.3f | %d/%s | %.3f | %d/%s | %.3f | %.3f |" % (
            r["layer"], r["C"], r["bi"], r["bo"], r["default_n1"], r["default_ms"], r["best_n1"],
            "h" if r["best_hoist"] else "-", r["best_ms"], r["mlp_n1"], "h" if r["mlp_hoist"] else "-",
            r["mlp_ms"], r["shortlist_ms"]))
    t = report["totals_ms"]
    out += ["", "Totals over the convolutions: default %.2f ms, exhaustive best %.2f ms, model's picks %.2f ms, "
            "model top-%d + default timed %.2f ms.  The default split is already the best on these layers; the "
            "gain is in CoeffToSlot, where the model picks a deeper decomposition (%d groups) that the default "
            "does not try." % (t["default"], t["best"], t["mlp"], report["shortlist"], t["shortlist"],
                               c["mlp"]["groups"]), ""]
    return "\n".join(out)


if __name__ == "__main__":
    import sys
    if len(sys.argv) >= 3 and sys.argv[1] == "--md":  # render a report: --md REPORT.json "command"
        with open(sys.argv[2]) as fh:
            print(summary(json.load(fh), sys.argv[3] if len(sys.argv) > 3 else "(not given)"))
    else:
        main()
