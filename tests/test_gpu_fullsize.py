"""Full-size parity (N = 2^16, 24 + 8 primes, three key-switching digits) through the
C ABI, word for word against the oracle (needs an MI355X):

* the benchmark step exactly as bench.py times it: fused conv at level 1 (hoisted baby
  steps, per-rotation giant steps) -> rescale -> ModRaise -> CoeffToSlot in three groups
  at levels 23/22/21 (lazy giant steps, partial last digits of 8/7/6 primes) -> the
  conjugate split fused into the conjugation's ModDown (Algorithm 1, conv through CoeffToSlot);
* ModEval as one call on a level-20 ciphertext (Sec. 2.4; the library's evaluation in
  both Chebyshev orders);
* a mixed-level job list run by the batched schedule (mode 1: two jobs of one conv plan
  at levels 9 and 13 sharing each key read across levels) and by its HIP-graph replay, against
  SHA-256 digests of the oracle's outputs written by tests/golden/full_batch_jobs.py.

The oracle's share of these tests runs its limb loops on every host core.
"""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle as O
import oracle.bootstrap as B
import oracle.plans as PL
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2312_04356_amd.workload import GpuWorkload  # noqa: E402
from tests.boot_rig import Rig  # noqa: E402
from tests.golden import full_batch_jobs as GJ  # noqa: E402
from tests.oracle_workload import OracleWorkload  # noqa: E402

RNG = np.random.default_rng(41)
SCALE = 2.0 ** 40


def host_coeff(gctx, ct, n_polys=2):
    t = ct.data.clone()
    gctx.nj_to_coeff(t, ct.level, n_polys)
    torch.cuda.synchronize()
    return gctx.to_host(t)


def load(gctx, plan, t, pts):
    for idx, j in enumerate(plan.offsets(t)):
        gctx.nj_plan_set_diagonal(plan, t, idx, pts[j])


def say(msg):
    print("[fullsize] " + msg, flush=True)


@pytest.mark.timeout(600)
def test_bench_step_parity_full():
    O.set_threads(0)
    say("bench step: setup")
    o = OracleWorkload("full", with_cts=True)
    g = GpuWorkload("full", with_cts=True, lazy=True)
    gctx = g.ctx
    assert g.q == o.ring.q and g.p == o.ring.p
    assert sorted(g.conv_plan.offsets(0)) == sorted(o.conv_bsgs.js)
    load(gctx, g.conv_plan, 0, o.conv_pts)
    assert g.cts_plan.count() == len(o.cts) == 3
    for t, (_, pts) in enumerate(o.cts):
        load(gctx, g.cts_plan, t, pts)
    gs = g.galois_elements()
    assert sorted(gs) == sorted(set(o.galois_elements()))
    g.make_keys(gs)
    o.make_keys(gs)
    m = o.ring.to_rns(o.input_plaintext(), 1)
    x_o = o.encrypt_input(1)
    x_g = g.encrypt_input(1, m_dev=gctx.to_device(m))
    say("bench step: library (conv + CoeffToSlot)")
    y = gctx.empty_ct(0)
    gctx.nj_conv2d_cins(g.conv_plan, x_g, y)
    lvl = gctx.L - 3
    re, im = gctx.empty_ct(lvl), gctx.empty_ct(lvl)
    gctx.nj_coeff_to_slot(g.cts_plan, y, re, im)
    torch.cuda.synchronize()
    say("bench step: oracle conv")
    y_o = o.ctx.conv2d_cins(x_o, o.conv_bsgs, o.conv_pts)
    assert np.array_equal(host_coeff(gctx, y), y_o), "conv output differs"
    say("bench step: oracle CoeffToSlot (three groups, lazy giant steps, split)")
    w_re, w_im = o.ctx.coeff_to_slot(y_o, [p for p, _ in o.cts], [pts for _, pts in o.cts], lazy=True)
    got_re, got_im = host_coeff(gctx, re), host_coeff(gctx, im)
    assert got_re.shape == w_re.shape == (2, lvl + 1, g.N)
    assert np.array_equal(got_re, w_re), "Re differs in %d words" % np.count_nonzero(got_re != w_re)
    assert np.array_equal(got_im, w_im), "Im differs in %d words" % np.count_nonzero(got_im != w_im)
    assert re.level == im.level == lvl


@pytest.mark.timeout(600)
def test_eval_mod_parity_full():
    """one ModEval call at N = 2^16 (level 20 -> 9) on slots t = m + P I, both
    Chebyshev orders, against the oracle's evaluation in the same order"""
    O.set_threads(0)
    say("ModEval: setup")
    full = Rig(16, 24, 8, 192)
    n = full.N // 2
    P = full.q[0] / SCALE
    m = RNG.uniform(-1, 1, n)
    t = m + P * RNG.integers(-12, 13, n)
    xo, ct = full.enc(t, 20, SCALE, 7)
    K, r = 32, 3
    coeffs = B.cheb_coeffs(K, r)
    for order in (0, 1):
        full.g.nj_eval_order(order)
        out = full.g.empty_ct(9)
        say("ModEval: library, order %d" % order)
        full.g.nj_eval_mod(ct, K, r, coeffs, out)
        torch.cuda.synchronize()
        say("ModEval: oracle, order %d" % order)
        want = full.boot.eval_mod((xo, 20, SCALE), K, r, coeffs, accumulate=bool(order))
        assert out.level == want[1] == 9 and out.scale == want[2]
        assert np.array_equal(full.coeff(out), want[0]), "order %d" % order
        z = full.dec_slots(out).real
        print("ModEval order %d at N=2^16: |z - m| %.2e" % (order, np.max(np.abs(z - m))))
    full.g.nj_eval_order(0)


def _digest(arr):
    return hashlib.sha256(np.ascontiguousarray(arr, dtype="<u8").tobytes()).hexdigest()


@pytest.mark.timeout(600)
def test_batched_mixed_levels_parity_full():
    """the batched schedule (mode 1) and its graph replay of three jobs at levels 9, 11
    and 13, the plain schedule and the batched schedule with the convs grouped across
    levels (mode 3) against the oracle's digests"""
    doc = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "full_batch_jobs.json")))
    O.set_threads(0)
    say("batched jobs: setup")
    o = OracleWorkload("full", with_cts=True, cts_split=False)  # the split the digests were made with
    g = GpuWorkload("full", with_cts=True, lazy=True, cts_split=False)
    gctx = g.ctx
    for t, (_, pts) in enumerate(o.cts):
        load(gctx, g.cts_plan, t, pts)
    plans = {}
    for name, (bs, pts) in GJ.oracle_plans(o).items():
        K = GJ.plan_weights(o)[name]
        p = gctx.nj_conv_plan_create_taps(o.w["w0"], o.C, o.C, PL.taps_same(K), fuse=1, level=GJ.TOP)
        assert sorted(p.offsets(0)) == sorted(bs.js)
        load(gctx, p, 0, pts)
        plans[name] = p
    gs = set(g.cts_plan.galois())
    for p in plans.values():
        gs |= set(p.galois())
    g.make_keys(sorted(gs))
    lo = gctx.L - 3
    jobs = []
    for (name, level, sub), row in zip(GJ.JOBS, doc["jobs"]):
        assert (row["plan"], row["level"], row["sub"]) == (name, level, sub)
        m = o.ring.to_rns(o.input_plaintext(), level)
        a, e = synth.enc_randomness(o.ring.q[:level + 1], o.N, o.w["data_seed"], sub)
        x = gctx.empty_batch(1, level)
        gctx.nj_encrypt_sk(gctx.to_device(m), level, a, e, SCALE, x)
        jobs.append((plans[name], x, gctx.empty_batch(1, lo), gctx.empty_batch(1, lo)))

    def check(what):
        for k, ((_, _, re, im), row) in enumerate(zip(jobs, doc["jobs"])):
            assert re.level == im.level == row["out_level"]
            assert _digest(host_coeff(gctx, re)[0]) == row["re_sha256"], "%s: job %d Re" % (what, k)
            assert _digest(host_coeff(gctx, im)[0]) == row["im_sha256"], "%s: job %d Im" % (what, k)

    say("batched jobs: mode 1")
    gctx.nj_batch_run(g.cts_plan, jobs, 1)
    torch.cuda.synchronize()
    check("batched")
    for j in jobs:
        j[2].data.zero_()
        j[3].data.zero_()
    say("batched jobs: graph replay")
    graph = gctx.nj_batch_create(g.cts_plan, jobs)
    for rep in range(2):
        graph.launch()
        torch.cuda.synchronize()
        check("graph replay %d" % rep)
        _ = torch.ones(1 << 20, device=gctx.device).sum().item()
    del graph
    say("batched jobs: mode 0")
    gctx.nj_batch_run(g.cts_plan, jobs, 0)
    torch.cuda.synchronize()
    check("plain")
    for j in jobs:
        j[2].data.zero_()
        j[3].data.zero_()
    say("batched jobs: mode 3 (convs grouped across levels)")
    gctx.nj_batch_run(g.cts_plan, jobs, 3)
    torch.cuda.synchronize()
    check("batched across levels")
