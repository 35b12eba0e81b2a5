"""Benchmark: fused CinS-conv + CoeffToSlot at N=2^16 and key switches per second.

One step = the whole hot path on one ciphertext of the full-size workload
(N = 2^16, 24 ciphertext primes + 8 special primes, 3x3 conv 16->16 on a 32x32
image packed as real CinS): BSGS conv with the fused K' = S'K diagonals at level 1,
rescale, ModRaise to level 23, CoeffToSlot in 3 stage groups, real/imaginary split.
Inputs (keys, plan diagonals, the encrypted image) are resident in HBM before the
timed region.  Prints one JSON line.

Order of GPU work: setup, key switches per second (plain and batched), the mixed
job list at uneven levels (plain vs batched HIP-graph replay), ModEval and StoC1
timings (reported separately), the batched pipeline,
warmup, timed steps, then the same number of steps again with the library's
per-kernel event timing (the last GPU work of the run, so a kernel trace's final
dispatches are those steps).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fused CinS-conv+CoeffToSlot ms and keyswitch/s at N=2^16; batched vs plain"
HBM_PEAK_GBS = 8000.0
# rocprofv3 counter summary of the step (FETCH_SIZE and WRITE_SIZE per launch, scaled by a
# copy of known size); its machine-readable line carries the digest of the kernel sources
# it was taken with, and `traffic` is reported only while the sources still match
PMC_SUMMARY = os.path.join(ROOT, "profiles", "pmc_fused_conv_cts_n65536.md")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="full")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--ks-iters", type=int, default=50)
    ap.add_argument("--batch", type=int, default=64, help="ciphertexts in the batched measurements")
    ap.add_argument("--batch-steps", type=int, default=2)
    ap.add_argument("--jobs", type=int, default=64, help="mixed jobs at uneven levels (0 skips them)")
    ap.add_argument("--no-boot", action="store_true", help="skip the ModEval / StoC1 timing")
    ap.add_argument("--no-lazy", action="store_true", help="one ModDown per giant step in CoeffToSlot")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-plan step")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run 10 device-to-device copies of 128 MiB (the counter calibration of the "
                         "rocprofv3 traffic figures) and exit")
    return ap.parse_args()


def copy_calibration():
    """device-to-device copies of a known size: the runtime's copy kernel reads and writes
    128 MiB per launch, the reference for scaling FETCH_SIZE / WRITE_SIZE to bytes"""
    import torch
    n = 128 * 2 ** 20 // 8
    src = torch.arange(n, dtype=torch.int64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(10):
        dst.copy_(src)
    torch.cuda.synchronize()
    assert torch.equal(dst, src)
    print(json.dumps({"copy_bytes": n * 8, "launches": 10}))


def group_rotations(g):
    """key-switched rotations of each CoeffToSlot group (baby steps except 0, giant steps except 0)"""
    out = []
    for t in range(g.cts_plan.count()):
        js = g.cts_plan.offsets(t)
        n1 = int(math.ceil(math.sqrt(len(js))))
        babies = {j - (j // n1) * n1 for j in js}
        giants = {j // n1 for j in js}
        out.append(len(babies - {0}) + len(giants - {0}))
    return out


def step_bytes(g):
    """Algorithmic HBM bytes of one step by kind: every switching key at the level it is
    used (active limbs and digits only), every plaintext diagonal, and the ciphertexts
    (the input, one read and one write per BSGS group, the ModRaise output, the two
    outputs).
      key(l) = 2 dnum_l (l+1+alpha) N 8,  pt(l) = (l+1) N 8,  ct(l) = 2 (l+1) N 8."""
    c = g.ctx
    N, a = c.N, c.alpha

    def key(l):
        return 2 * (-(-(l + 1) // a)) * (l + 1 + a) * N * 8

    def pt(l):
        return (l + 1) * N * 8

    def ct(l):
        return 2 * (l + 1) * N * 8

    keys = len(g.conv_plan.galois()) * key(1)
    pts = len(g.conv_plan.offsets(0)) * pt(1)
    cts = ct(1) + ct(0) + ct(c.L)  # input, conv output, ModRaise output
    level = c.L
    for t, r in enumerate(group_rotations(g)):
        pts += len(g.cts_plan.offsets(t)) * pt(level)
        cts += 2 * ct(level)
        keys += r * key(level)
        level -= 1
    keys += key(level)  # conjugation
    cts += 2 * ct(level)  # Re and Im
    return {"keys": float(keys), "plaintexts": float(pts), "ciphertexts": float(cts)}


def pipeline_bytes(g):
    return sum(step_bytes(g).values())


def source_digest():
    """SHA-256 (first 16 hex digits) of the library's kernel and host sources"""
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2312_04356_amd", "csrc", "*"))):
        h.update(os.path.basename(f).encode())
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def pmc_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary, if it was
    taken with the current sources (else None) -> (bytes or None, note)"""
    if not os.path.exists(PMC_SUMMARY):
        return None, "no counter summary"
    rec = None
    for line in open(PMC_SUMMARY):
        if line.startswith("traffic-record: "):
            rec = json.loads(line[len("traffic-record: "):])
    if rec is None:
        return None, "counter summary has no traffic record"
    if rec.get("source_sha16") != source_digest():
        return None, "kernel sources changed since the counters were taken"
    row = rec.get("kernels", {}).get(kernel)
    if row is None:
        return None, "kernel not in the counter summary"
    return row["hbm_bytes_per_launch"], "rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated"


def job_plans(g, specs, n1_of=None):
    """conv plans (encoded at the top level, used at every job level) for each (op, C)
    of the job mix; weights U(-1,1) scaled by 1/(f sqrt(C_in))"""
    import synth
    gctx, plans = g.ctx, {}
    for op, C in sorted({(o, c) for o, c, _ in specs}):
        k = 8 * synth.JOB_OPS.index(op) + sorted(synth.JOB_CHANNELS).index(C)  # weights per (op, C)
        w0 = synth.JOB_CHANNELS[C]
        n1 = 0 if n1_of is None else n1_of[(op, C)]
        if op == "dw3x3":
            K = synth.uniform_real((C, 3, 3), 1004, 100 + k) / 3.0
            plans[(op, C)] = gctx.nj_conv_plan_create_layer(w0, K, depthwise=True, n1=n1, level=gctx.L)
        else:
            f = 1 if op == "1x1" else 3
            K = synth.uniform_real((C, C, f, f), 1004, 100 + k) / (f * math.sqrt(C))
            plans[(op, C)] = gctx.nj_conv_plan_create_layer(w0, K, stride=2 if op == "3x3s2" else 1, n1=n1,
                                                            level=gctx.L)
    return plans


def tune_splits(g, plans, level=15, reps=3):
    """the library's autotuner (nj_tune_split, every candidate timed) per plan structure:
    baby-step count n1, hoisting and the giant steps' ModDown form (one per giant step,
    or one for all: lazy), on random-diagonal plans with timing keys; returns
    {key: (n1, hoist, lazy)}"""
    gctx, out = g.ctx, {}
    gctx.nj_timing_keys(16)
    try:
        for key, plan in plans.items():
            n1, hoist, lazy, _, _ = gctx.nj_tune_split(plan, level, model=None, reps=reps, lazy=True)
            out[key] = (n1, hoist, lazy)
    finally:
        gctx.nj_timing_keys(0)
    return out


def jobs_bench(g, n_jobs, steps=2):
    """64 jobs at uneven levels 7..23, each conv (3x3, 3x3 stride 2, 1x1 or depthwise 3x3
    on 16/64/256 channels per ciphertext) at its level -> level drop -> ModRaise ->
    CoeffToSlot -> split.  Plain: one job after another with default plans.  Batched:
    each conv on its fused path, then CoeffToSlot over all 64 outputs together, replayed
    as one HIP graph, with n1, hoisting and lazy giant steps tuned per shape by the
    library's autotuner; across
    levels: the same with each conv
    plan's jobs grouped across their levels.  Concurrent: the plain schedule spread over
    4 worker streams, as one HIP graph."""
    import torch
    import synth
    gctx = g.ctx
    specs = synth.job_mix(n_jobs, 1004)
    default = job_plans(g, specs)
    best = tune_splits(g, default)
    n1_of = {k: v[0] for k, v in best.items()}
    tuned = job_plans(g, [(o, c, 0) for (o, c) in best], n1_of)
    for k, (_, hoist, lazy) in best.items():
        tuned[k].set_hoist(hoist).set_lazy(lazy)
    gs = set(g.cts_plan.galois())
    for p in list(default.values()) + list(tuned.values()):
        gs |= set(p.galois())
    g.make_keys(sorted(gs))
    lvl = gctx.L - g.w["cts_groups"]
    xs = []
    for op, C, level in specs:
        x = gctx.empty_batch(1, level)
        x.data.random_(0, 2 ** 40)
        x.scale = g.scale
        xs.append(x)

    def jobs_with(plans):
        return [(plans[(op, C)], x, gctx.empty_batch(1, lvl), gctx.empty_batch(1, lvl))
                for (op, C, _), x in zip(specs, xs)]

    jp, jt = jobs_with(default), jobs_with(tuned)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    plain = timed(lambda: gctx.nj_batch_run(g.cts_plan, jp, 0))
    eager = timed(lambda: gctx.nj_batch_run(g.cts_plan, jp, 1))
    graph = gctx.nj_batch_create(g.cts_plan, jt)
    replay = timed(lambda: graph.launch())
    del graph
    # the same with the convs of one plan grouped across levels (keys shared, transforms
    # unfused)
    graph = gctx.nj_batch_create(g.cts_plan, jt, mode=3)
    across = timed(lambda: graph.launch())
    del graph
    # the plain schedule of every job on 4 worker streams, as one graph (default plans)
    graph = gctx.nj_batch_create(g.cts_plan, jp, mode=2)
    conc = timed(lambda: graph.launch())
    del graph
    return {"n_jobs": n_jobs, "levels": "7..23", "plain_ms": round(plain, 3),
            "batched_default_plans_ms": round(eager, 3), "batched_graph_tuned_ms": round(replay, 3),
            "speedup_vs_plain": round(plain / replay, 3), "across_levels_graph_ms": round(across, 3),
            "concurrent_graph_ms": round(conc, 3),
            "concurrent_speedup_vs_plain": round(plain / conc, 3),
            "tuned_n1_hoist_lazy": {"%s/C%d" % k: list(v) for k, v in sorted(best.items())}}


PLAN_MODEL = os.path.join(ROOT, "paper_2312_04356_amd", "data", "plan_model_n65536.json")


def bitrev_perm(n):
    b = n.bit_length() - 1
    return [int(format(j, "0%db" % b)[::-1], 2) for j in range(n)]


def crt2(res, q):
    """centred integers from residues [2][N] modulo q[0], q[1]"""
    Q = q[0] * q[1]
    h0, h1 = q[1] * pow(q[1], -1, q[0]), q[0] * pow(q[0], -1, q[1])
    out = []
    for a, b in zip(res[0].tolist(), res[1].tolist()):
        x = (a * h0 + b * h1) % Q
        out.append(x - Q if x > Q // 2 else x)
    return out


def slot_error(g, y, re, im, lvl):
    """max |CoeffToSlot slot - bit-reversed coefficient| of the step's outputs (the
    decryption accuracy the plans are compared at): the level-0 conv output is decrypted
    over the integers (c0 + c1 s, which ModRaise lifts), each CoeffToSlot output by the
    library and decoded by it"""
    import numpy as np
    import torch
    gctx, n = g.ctx, g.N // 2
    t = y.data.clone()
    gctx.nj_to_coeff(t, 0, 2)
    torch.cuda.synchronize()
    c = gctx.to_host(t)
    q0 = g.q[0]
    c0 = np.where(c[0][0] > q0 // 2, c[0][0].astype(np.int64) - np.int64(q0), c[0][0].astype(np.int64))
    c1 = np.where(c[1][0] > q0 // 2, c[1][0].astype(np.int64) - np.int64(q0), c[1][0].astype(np.int64))
    prod = np.zeros_like(c0)
    for i in np.nonzero(g.s)[0]:
        sh = np.roll(c1, i)
        sh[:i] = -sh[:i]
        prod += int(g.s[i]) * sh
    raw = (c0 + prod).astype(np.float64) / g.scale
    rev = np.array(bitrev_perm(n))
    err = 0.0
    for ct, want in ((re, raw[:n][rev]), (im, raw[n:][rev])):
        d = torch.empty((lvl + 1, g.N), dtype=torch.int64, device=gctx.device)
        gctx.nj_decrypt(ct, d)
        m = crt2(gctx.to_host(d)[:2], g.q[:2])
        z = gctx.nj_decode_slots(np.array(m, dtype=np.float64), g.scale)
        err = max(err, float(np.max(np.abs(z.real - want))), float(np.max(np.abs(z.imag))))
    return err


def encrypted_batch(g, n):
    """n distinct secret-key encryptions of the workload's image at level 1, as one batch"""
    import torch

    import synth
    from paper_2312_04356_amd import Ct
    gctx = g.ctx
    coeffs = gctx.nj_encode_cins(g.image_slices(), g.scale)
    mdev = torch.empty((2, g.N), dtype=torch.int64, device=gctx.device)
    gctx.nj_upload_plain(coeffs, 1, mdev)
    xb = gctx.empty_batch(n, 1)
    for z in range(n):
        a, e = synth.enc_randomness(g.q[:2], g.N, g.w["data_seed"], 100 + z)
        gctx.nj_encrypt_sk(mdev, 1, a, e, g.scale, Ct(xb.data[z], 1))
    return xb


def batched_ms(g, conv, cts, xb, n, lvl, steps):
    """ms per batch of n ciphertexts through conv + CoeffToSlot (batched calls), and the
    slot error of the first ciphertext's outputs"""
    import torch

    from paper_2312_04356_amd import Ct
    gctx = g.ctx
    yb = gctx.empty_batch(n, 0)
    reb, imb = gctx.empty_batch(n, lvl), gctx.empty_batch(n, lvl)

    def bstep():
        gctx.nj_conv2d_cins_batch(conv, xb, n, yb)
        gctx.nj_coeff_to_slot_batch(cts, yb, n, reb, imb)

    bstep()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        bstep()
    e1.record()
    torch.cuda.synchronize()
    err = slot_error(g, Ct(yb.data[0], 0), Ct(reb.data[0], lvl), Ct(imb.data[0], lvl), lvl)
    return e0.elapsed_time(e1) / steps, err


def learned_plan_bench(g, ct, default_ms, steps, reps=3, batch=0, batch_steps=2):
    """The step with the plan the learned latency model proposes (the model trained by
    paper_2312_04356_amd/tune.py from the library's own timings, run by nj_mlp_predict):
    the conv's BSGS split and hoisting, CoeffToSlot's depth (2..6, within Algorithm 1's
    level budget), each group's split and hoisting.  The model ranks every candidate; its
    best few are timed (nj_time_plan, timing keys for rotations without a key) and the
    fastest is built with real keys, timed like the default step, and its CoeffToSlot
    outputs checked against the bit-reversed coefficients as the default's are."""
    import torch

    from paper_2312_04356_amd import Mlp
    from paper_2312_04356_amd.tune import SHORTLIST, rank_conv, rank_cts
    if not os.path.exists(PLAN_MODEL):
        return None
    doc = json.load(open(PLAN_MODEL))
    model = Mlp.from_dict(doc)
    gctx = g.ctx
    convs = {(n1, h): gctx.nj_conv_plan_create(g.w["w0"], g.w["f"], g.K, n1).set_hoist(h)
             for n1 in (1, 2, 4, 8, 16) for h in (True, False)}
    gctx.nj_timing_keys(16)
    try:
        # the model's best candidates and the benchmark's own plan (n1 = 4, hoisted; depth 3
        # with the workload's splits) are timed; the fastest is used
        cr = rank_conv(gctx, model, convs, 1)
        pred_of = {k: p for p, k in cr}
        short = [k for _, k in cr[:SHORTLIST]] + ([(4, True)] if (4, True) not in [k for _, k in cr[:SHORTLIST]] else [])
        conv_t = [(gctx.nj_time_plan(convs[k], 1, reps=reps), k, pred_of[k]) for k in short]
        conv_ms, (cn1, ch), conv_pred = min(conv_t)
        ranked = rank_cts(gctx, model)
        dflt_n1 = list(g.w.get("cts_n1") or [int(math.ceil(math.sqrt(f[1]))) for f in gctx.nj_cts_plan_features(3)])
        cands = [(d, n1s, hs, pred) for pred, d, n1s, hs in ranked[:SHORTLIST]]
        if not any(d == 3 and n1s == dflt_n1 and all(hs) for d, n1s, hs, _ in cands):
            cands.append((3, dflt_n1, [True] * 3, None))
        cts_t = []
        for d, n1s, hs, pred in cands:
            plan = gctx.nj_cts_plan_create_split(d, n1s).set_lazy(True).set_hoist(hs)
            cts_t.append((sum(gctx.nj_time_plan(plan, gctx.L - t, t=t, reps=reps) for t in range(d)), d, n1s, hs, pred))
            del plan
    finally:
        gctx.nj_timing_keys(0)
    cts_ms, d, n1s, hs, cts_pred = min(cts_t, key=lambda r: r[0])
    conv = convs.pop((cn1, ch))
    del convs
    cts = gctx.nj_cts_plan_create_split(d, n1s).set_lazy(True).set_hoist(hs)
    g.make_keys(sorted(set(conv.galois()) | set(cts.galois())))
    lvl = gctx.L - d
    y = gctx.empty_ct(0)
    re, im = gctx.empty_ct(lvl), gctx.empty_ct(lvl)

    def step():
        gctx.nj_conv2d_cins(conv, ct, y)
        gctx.nj_coeff_to_slot(cts, y, re, im)

    step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    err = slot_error(g, y, re, im, lvl)
    both = None
    if batch > 0:
        # batched and learned together: the model's plans on the batched calls
        xb = encrypted_batch(g, batch)
        bms, berr = batched_ms(g, conv, cts, xb, batch, lvl, batch_steps)
        del xb
        both = {"n_ct": batch, "ms_per_ct": round(bms / batch, 4), "speedup_vs_plain": round(default_ms / (bms / batch), 3),
                "cts_slot_err_first_ct": berr}
    return {"conv": {"n1": cn1, "hoist": ch, "predicted_ms": round(conv_pred, 3), "timed_ms": round(conv_ms, 3)},
            "cts": {"groups": d, "n1": n1s, "hoist": hs, "predicted_ms": None if cts_pred is None else round(cts_pred, 3),
                    "timed_ms": round(cts_ms, 3)},
            "shortlist": SHORTLIST,
            "cts_shortlist": [{"groups": dd, "n1": nn, "hoist": hh, "timed_ms": round(t, 3),
                               "predicted_ms": None if p is None else round(p, 3)} for t, dd, nn, hh, p in cts_t],
            "ms": round(ms, 4), "default_ms": round(default_ms, 4), "speedup_vs_default": round(default_ms / ms, 3),
            "cts_slot_err": err, "output_level": lvl, "batched_with_learned_plan": both,
            "model": os.path.relpath(PLAN_MODEL, ROOT),
            "model_heldout_rel_err": doc.get("heldout_rel_err")}


def boot_bench(g, steps=3):
    """the bootstrapping steps after CoeffToSlot on the step's Re / Im outputs (level 20):
    ModEval of Re and of Im (11 levels each), Re + i Im, StoC1 for l = 2048 in 3 groups"""
    import torch
    import synth
    gctx = g.ctx
    lo = gctx.L - g.w["cts_groups"]
    stoc1 = gctx.nj_stoc1_plan_create(g.ell, 3, lo - 11)
    a, e = synth.key_randomness(g.q + g.p, g.N, gctx.dnum, g.w["key_seed"], synth.RELIN_KEY_ID)
    gctx.nj_gen_switch_key(0, a, e)
    g.make_keys(sorted(stoc1.galois()))
    ct = g.encrypt_input(1)
    y = gctx.empty_ct(0)
    gctx.nj_conv2d_cins(g.conv_plan, ct, y)
    re, im = gctx.empty_ct(lo), gctx.empty_ct(lo)
    gctx.nj_coeff_to_slot(g.cts_plan, y, re, im)
    er, ei, z = gctx.empty_ct(lo - 11), gctx.empty_ct(lo - 11), gctx.empty_ct(lo - 11)
    out = gctx.empty_ct(lo - 14)
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))

    def run():
        gctx.nj_eval_mod(re, 32, 3, None, er)
        gctx.nj_eval_mod(im, 32, 3, None, ei)
        e1.record()
        gctx.nj_combine(er, ei, z)
        gctx.nj_stoc1(stoc1, z, out)

    run()
    torch.cuda.synchronize()
    t_mod = t_all = 0.0
    for _ in range(steps):
        e0.record()
        run()
        e2.record()
        torch.cuda.synchronize()
        t_mod += e0.elapsed_time(e1)
        t_all += e0.elapsed_time(e2)
    res = {"eval_mod_re_im_ms": round(t_mod / steps, 3), "stoc1_ms": round((t_all - t_mod) / steps, 3),
           "levels": {"in": lo, "after_eval_mod": lo - 11, "after_stoc1": lo - 14}, "K": 32, "degree": 63,
           "double_angles": 3, "stoc1_groups": 3}
    # the same tail as one call: ModEval of Re and Im evaluated together (each HMult, constant
    # multiply, rescale and key switch of the chain on both ciphertexts per launch), Re + i Im, StoC1
    out2 = gctx.empty_ct(lo - 14)
    gctx.nj_slot_activation(32, 3, None, None, None, 0, stoc1, re, im, out2)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        gctx.nj_slot_activation(32, 3, None, None, None, 0, stoc1, re, im, out2)
    e2.record()
    torch.cuda.synchronize()
    res["eval_mod_packed_and_stoc1_ms"] = round(e0.elapsed_time(e2) / steps, 3)
    # one whole Algorithm 1 layer: conv (fused StoC2) -> ModRaise -> CoeffToSlot -> ModEval of
    # Re and Im -> zero-padding masks -> square activation -> Re + i Im -> StoC1
    from paper_2312_04356_amd import nj_layer_masks
    le = lo - 11
    st1 = gctx.nj_stoc1_plan_create(g.ell, 3, le - 2)
    g.make_keys(sorted(st1.galois()))
    masks = []
    for mk in nj_layer_masks(gctx.log_n, g.W, g.C, g.w["w0"]):
        t = torch.empty((le + 1, g.N), dtype=torch.int64, device=gctx.device)
        gctx.nj_upload_plain(gctx.nj_encode_slots(mk, float(g.q[le])), le, t)
        gctx.nj_to_eval(t, le, 1)
        masks.append(t)
    lout = gctx.empty_ct(le - 5)

    def layer():
        gctx.nj_conv_act_layer(g.conv_plan, g.cts_plan, 32, 3, None, masks[0], masks[1], 1, st1, ct, lout)

    layer()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        layer()
    e2.record()
    torch.cuda.synchronize()
    res["algorithm1_layer"] = {"ms": round(e0.elapsed_time(e2) / steps, 3), "activation": "square", "masks": True,
                               "levels": {"in": 1, "out": le - 5}}
    return res


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_step(name, threads_list):
    """the oracle's whole step on workload `name` timed once per thread count, and one
    top-level rotation timed per thread count -> ({threads: step s}, {threads: rotation s})"""
    import oracle as O
    from oracle.plans import galois_elt
    from tests.oracle_workload import OracleWorkload
    O.set_threads(0)
    o = OracleWorkload(name, with_cts=True)
    o.make_keys()
    ct = o.encrypt_input(1)
    step, rot = {}, {}
    y = None
    for n in threads_list:
        O.set_threads(n)
        t = time.perf_counter()
        y = o.ctx.conv2d_cins(ct, o.conv_bsgs, o.conv_pts)
        o.ctx.coeff_to_slot(y, [p for p, _ in o.cts], [pts for _, pts in o.cts], lazy=True)
        step[n] = time.perf_counter() - t
    x = o.ctx.ct_modraise(y)
    r = o.cts[0][0].rotations()[0]
    assert galois_elt(r, o.N) in o.ctx.keys
    for n in sorted(set(threads_list) | {1}):
        O.set_threads(n)
        t = time.perf_counter()
        o.ctx.rotate(o.ring.L, x, r)
        rot[n] = time.perf_counter() - t
    O.set_threads(0)
    return step, rot


def cpu_baseline(name):
    """The oracle on the host, the whole step once: the fused conv at level 1, rescale,
    ModRaise, CoeffToSlot in three groups with lazy giant steps and the real split, on
    one ciphertext with its limb loops on every host core (keys generated before the
    timed region, as they are resident on the GPU).  The single-thread figure scales
    that time by the one-core / all-core ratio of one top-level rotation; the same
    estimate is checked on the small workload (N = 2^12), whose whole step is also
    timed on one core."""
    import oracle as O
    t0 = time.time()
    O.set_threads(0)
    threads = O.get_threads()
    step, rot = _oracle_step(name, [threads])
    total = step[threads]
    s_small, r_small = _oracle_step("small", [threads, 1])
    est_small = s_small[threads] * r_small[1] / r_small[threads]
    return {"value": round(total * 1e3, 1), "unit": "ms", "cores": threads, "kind": "oracle",
            "sample": "the whole step once (conv at level 1, rescale, ModRaise, CoeffToSlot 3 groups with lazy "
                      "giant steps, real split) on one ciphertext, limb loops over %d OpenMP threads" % threads,
            "single_thread_ms_est": round(total * rot[1] / rot[threads] * 1e3, 1),
            "thread_speedup_one_rotation": round(rot[1] / rot[threads], 2),
            "estimate_check_n4096": {"single_thread_ms": round(s_small[1] * 1e3, 1),
                                     "all_threads_ms": round(s_small[threads] * 1e3, 1),
                                     "single_thread_ms_est": round(est_small * 1e3, 1),
                                     "rel_err": round(est_small / s_small[1] - 1.0, 3)},
            "nproc": os.cpu_count(), "cpu_model": cpu_model(), "wall_s": round(time.time() - t0, 1)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    import torch

    from paper_2312_04356_amd import PROF_KERNELS
    from paper_2312_04356_amd.workload import GpuWorkload

    g = GpuWorkload(args.workload, with_cts=True, lazy=not args.no_lazy)
    gctx = g.ctx
    g.make_keys()
    ct = g.encrypt_input(1)
    lvl = gctx.L - g.w["cts_groups"]
    y = gctx.empty_ct(0)
    re, im = gctx.empty_ct(lvl), gctx.empty_ct(lvl)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    # key switches per second, one ciphertext per call (plain)
    ks = {}
    gk = g.conv_plan.galois()[0]
    for level in (23, 15, 7):
        if level > gctx.L:
            continue
        x = gctx.empty_ct(level)
        x.data.random_(0, 2 ** 40)
        for _ in range(3):
            gctx.nj_apply_galois(x, gk, x)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.ks_iters):
            gctx.nj_apply_galois(x, gk, x)
        e1.record()
        torch.cuda.synchronize()
        ks[str(level)] = round(args.ks_iters / (e0.elapsed_time(e1) / 1e3), 1)

    # batched: the same key switch on 64 ciphertexts per call (each key word read once per 8)
    ks_batch = {}
    nbk = args.batch
    for level in (23, 15, 7):
        if level > gctx.L:
            continue
        xb, ob = gctx.empty_batch(nbk, level), gctx.empty_batch(nbk, level)
        xb.data.random_(0, 2 ** 40)
        gctx.nj_apply_galois_batch(xb, nbk, gk, ob)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(max(1, args.ks_iters // nbk * 4)):
            gctx.nj_apply_galois_batch(xb, nbk, gk, ob)
        e1.record()
        torch.cuda.synchronize()
        it = max(1, args.ks_iters // nbk * 4)
        ks_batch[str(level)] = round(it * nbk / (e0.elapsed_time(e1) / 1e3), 1)
        del xb, ob

    jobs = jobs_bench(g, args.jobs) if args.jobs > 0 else None
    boot = None if args.no_boot else boot_bench(g)
    torch.cuda.empty_cache()

    # batched fused conv + CoeffToSlot: 64 ciphertexts (distinct encryptions of the image)
    xb = encrypted_batch(g, args.batch)
    batch_ms, batch_err = batched_ms(g, g.conv_plan, g.cts_plan, xb, args.batch, lvl, args.batch_steps)
    del xb

    def step():
        gctx.nj_conv2d_cins(g.conv_plan, ct, y)
        gctx.nj_coeff_to_slot(g.cts_plan, y, re, im)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    e0.record()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / args.steps

    default_err = slot_error(g, y, re, im, lvl)
    learned = None if args.no_learned else learned_plan_bench(g, ct, ms, args.steps, batch=args.batch,
                                                                batch_steps=args.batch_steps)
    torch.cuda.empty_cache()

    # the same steps again with the library's live per-kernel event timing
    for k in PROF_KERNELS:
        gctx.nj_prof_read(k, reset=True)
    gctx.nj_prof_enable(1)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    gctx.nj_prof_enable(0)
    kern = {}
    for k, name in PROF_KERNELS.items():
        n, kms, kby = gctx.nj_prof_read(k, reset=True)
        if n:
            kern[name] = {"launches_per_step": n / args.steps, "ms_per_step": kms / args.steps,
                          "avg_launch_us": 1e3 * kms / n, "gbs": kby / kms / 1e6}
    dom = max((k for k in kern if k != "other"), key=lambda k: kern[k]["ms_per_step"])
    sb = step_bytes(g)
    alg = sum(sb.values())
    if dom == "k_key_ip":  # algorithmic bytes of the key inner products: the switching keys they read
        dom_alg = sb["keys"]
    elif dom == "k_pmac":  # of the plaintext multiply-accumulate: the plaintext diagonals
        dom_alg = sb["plaintexts"]
    else:
        dom_alg = None
    launches = kern[dom]["launches_per_step"]
    traffic, traffic_note = pmc_traffic(dom)
    roofline = {"bound": "hbm", "kernel": dom, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "avg_launch_us": round(kern[dom]["avg_launch_us"], 2), "launches_per_step": launches,
                "traffic": traffic, "traffic_source": traffic_note,
                "io_gbs": round(kern[dom]["gbs"], 1),
                "io_bytes_per_launch": round(kern[dom]["gbs"] * kern[dom]["avg_launch_us"] * 1e3)}
    if dom_alg is not None:
        per_launch = dom_alg / launches
        achieved = per_launch / (kern[dom]["avg_launch_us"] * 1e-6) / 1e9
        roofline.update({"achieved": round(achieved, 1), "frac": round(achieved / HBM_PEAK_GBS, 4),
                         "algorithmic_bytes_per_launch": round(per_launch)})
    else:
        roofline.update({"achieved": roofline["io_gbs"], "frac": round(roofline["io_gbs"] / HBM_PEAK_GBS, 4),
                         "algorithmic_bytes_per_launch": roofline["io_bytes_per_launch"]})

    out = {
        "metric": METRIC,
        "value": round(ms, 4),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "N=2^16 fused CinS conv 3x3 16->16 32x32 + CoeffToSlot (3 groups), 24+8 primes, dnum=3",
                   "log_n": gctx.log_n, "n_q": gctx.L + 1, "alpha": gctx.alpha,
                   "cts_groups": g.w["cts_groups"], "cts_n1": g.w.get("cts_n1"), "lazy_giant_steps": not args.no_lazy,
                   "host_wall_s": round(wall, 3)},
        "keyswitch_per_s": {"plain": ks, "batched": ks_batch, "batch": nbk, "galois": gk},
        "batched": {"n_ct": args.batch, "ms_per_batch": round(batch_ms, 3),
                    "ms_per_ct": round(batch_ms / args.batch, 4),
                    "speedup_vs_plain": round(ms / (batch_ms / args.batch), 3),
                    "cts_slot_err_first_ct": batch_err,
                    "hbm_frac_per_ct": round(pipeline_bytes(g) / (batch_ms / args.batch * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
        "jobs": jobs,
        "learned_plan": learned,
        "default_plan_cts_slot_err": default_err,
        "bootstrap_after_cts": boot,
        "roofline": roofline,
        "pipeline": {"algorithmic_GB": round(alg / 1e9, 3),
                     "algorithmic_GB_by_kind": {k: round(v / 1e9, 3) for k, v in sb.items()},
                     "hbm_frac": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "source_sha16": source_digest(),
                     "kernels": {k: {kk: round(vv, 3) for kk, vv in v.items()} for k, v in kern.items()}},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.workload)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
