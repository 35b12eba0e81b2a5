"""What the trained latency model gains over planning without it (needs an MI355X).

The model (3 layers, 64 hidden, FP32; trained by the library's own kernels on the
library's own timings and stored in paper_2312_04356_amd/data) ranks every
CoeffToSlot plan of the full-size workload (N = 2^16, 24 + 8 primes, three digits):
depth 2..6 within the level budget, each group's baby-step count and hoisting
(Sec. 2.6 BSGS and its decomposition-depth trade-off; Sec. 4.2 fusion).  Without the
model the step runs the workload's default plan (depth 3, baby-step counts 4, 8, 8,
every group hoisted).

Checked: the model's first choice, built with real keys and timed as one whole step
(conv + CoeffToSlot, the timed calls interleaved with the default's), is faster than
the default step; its CoeffToSlot outputs decode to the conv output's bit-reversed
coefficients as accurately as the default's (both within 2^-15); and the model's
predicted CoeffToSlot latency is within 50% of the time measured for that plan.
"""
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from bench import PLAN_MODEL, slot_error  # noqa: E402
from paper_2312_04356_amd import Mlp  # noqa: E402
from paper_2312_04356_amd.tune import rank_cts  # noqa: E402
from paper_2312_04356_amd.workload import GpuWorkload  # noqa: E402


def _step_ms(gctx, conv, cts, ct, y, re, im, steps):
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    gctx.nj_conv2d_cins(conv, ct, y)
    gctx.nj_coeff_to_slot(cts, y, re, im)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        gctx.nj_conv2d_cins(conv, ct, y)
        gctx.nj_coeff_to_slot(cts, y, re, im)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def test_learned_cts_plan_beats_default_at_equal_accuracy():
    assert os.path.exists(PLAN_MODEL), "trained plan model missing"
    doc = json.load(open(PLAN_MODEL))
    model = Mlp.from_dict(doc)

    g = GpuWorkload("full", with_cts=True, lazy=True)
    gctx = g.ctx
    pred_ms, d, n1s, hs = rank_cts(gctx, model)[0]
    print("model's plan: depth %d, n1 %s, hoist %s, predicted %.3f ms" % (d, n1s, hs, pred_ms), flush=True)
    learned = gctx.nj_cts_plan_create_split(d, n1s).set_lazy(True).set_hoist(hs)

    # the model's CoeffToSlot latency against the time measured for that plan
    gctx.nj_timing_keys(16)
    try:
        timed = sum(gctx.nj_time_plan(learned, gctx.L - t, t=t, reps=3) for t in range(d))
    finally:
        gctx.nj_timing_keys(0)
    print("measured %.3f ms" % timed, flush=True)
    assert abs(pred_ms - timed) / timed < 0.5

    g.make_keys(sorted(set(g.conv_plan.galois()) | set(g.cts_plan.galois()) | set(learned.galois())))
    ct = g.encrypt_input(1)
    y = gctx.empty_ct(0)
    l_def, l_new = gctx.L - g.w["cts_groups"], gctx.L - d
    re0, im0 = gctx.empty_ct(l_def), gctx.empty_ct(l_def)
    re1, im1 = gctx.empty_ct(l_new), gctx.empty_ct(l_new)

    t_def, t_new = [], []
    for _ in range(3):
        t_def.append(_step_ms(gctx, g.conv_plan, g.cts_plan, ct, y, re0, im0, 8))
        t_new.append(_step_ms(gctx, g.conv_plan, learned, ct, y, re1, im1, 8))
    ms_def, ms_new = float(np.median(t_def)), float(np.median(t_new))
    print("step: default %.3f ms, model's plan %.3f ms (%.3fx)" % (ms_def, ms_new, ms_def / ms_new), flush=True)
    assert ms_new < ms_def

    err_def = slot_error(g, y, re0, im0, l_def)
    err_new = slot_error(g, y, re1, im1, l_new)
    print("slot error: default %.3g, model's plan %.3g" % (err_def, err_new), flush=True)
    assert err_def < 2.0 ** -15 and err_new < 2.0 ** -15
