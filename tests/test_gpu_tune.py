"""Plan selection on the GPU (needs an MI355X): the cost-model kernels against the
float64 oracle (forward values and loss gradient), training reduces the loss, and the
timing helpers (random-diagonal plans, timing keys, features)."""
import json

import numpy as np
import pytest

import oracle.mlp as M

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2312_04356_amd import Mlp, NjError  # noqa: E402
from paper_2312_04356_amd.workload import GpuWorkload  # noqa: E402

RNG = np.random.default_rng(41)


@pytest.mark.parametrize("n", [1, 63, 64, 200])
def test_mlp_gradient_matches_oracle(n):
    m = Mlp(seed=5)
    p = RNG.normal(0, 0.3, M.N_PARAMS).astype(np.float32)
    m.set_params(p)
    X = RNG.normal(0, 1, (n, 7)).astype(np.float32)
    y = RNG.normal(0, 1, n).astype(np.float32)
    g, loss = m.grad(X, y)
    want = M.grad(p.astype(np.float64), X.astype(np.float64), y.astype(np.float64))
    scale = np.max(np.abs(want))
    assert np.max(np.abs(g - want)) <= 1e-4 * scale
    assert abs(loss - M.loss(p, X, y)) <= 1e-4 * max(1.0, M.loss(p, X, y))


def test_mlp_forward_matches_oracle():
    m = Mlp(seed=9)  # untrained: identity standardisation
    p = m.params()
    X = RNG.normal(0, 1, (130, 7)).astype(np.float32)
    out, _ = M.forward(p.astype(np.float64), X.astype(np.float64))
    assert np.allclose(m.predict(X), out, rtol=1e-4, atol=1e-4)


def test_mlp_training_fits_a_smooth_target():
    X = RNG.uniform(0, 1, (2000, 7)).astype(np.float32)
    y = (np.log1p(X[:, 0] * X[:, 2] * 8) + 0.5 * X[:, 3] + 0.2 * np.sin(4 * X[:, 4])).astype(np.float32)
    m = Mlp(seed=1)
    loss = m.train(X, y, epochs=150, batch=128, lr=2e-3, seed=2)
    pred = m.predict(X)
    r = np.corrcoef(pred, y)[0, 1]
    print("train MSE (standardised) %.4f, correlation %.4f" % (loss, r))
    assert loss < 0.05 and r > 0.97


def test_timing_plans_and_keys():
    g = GpuWorkload("full", with_cts=False)
    ctx = g.ctx
    n = g.N // 2
    plan = ctx.nj_plan_create_random(3, 2048, list(range(16)), n1=4)  # C = 16 conv structure
    f = plan.features(3)
    # limbs, diagonals, log2(n/u), baby steps, hoisted baby rotations, fusion depth, bo
    assert list(f) == [4, 16, 4, 4, 3, 4, 1]
    assert list(plan.set_hoist(False).features(3)) == [4, 16, 4, 4, 0, 4, 1]
    plan.set_hoist(True)
    with pytest.raises(NjError):  # no keys: the transform refuses to run
        ctx.nj_time_plan(plan, 3)
    ctx.nj_timing_keys(16)
    try:
        t1 = ctx.nj_time_plan(plan, 3, reps=3)
        t2 = ctx.nj_time_plan(plan, 1, reps=3)
        t_plain = ctx.nj_time_plan(plan.set_hoist(False), 3, reps=3)
        plan.set_hoist(True)
        print("C=16 n1=4 at level 3: hoisted %.3f ms, not hoisted %.3f ms" % (t1, t_plain))
        # either may be faster (the unhoisted path runs the fused key-switch kernels):
        # both modes run and are timed, which is what the plan search needs
        assert t1 > 0 and t_plain > 0
        blk = ctx.nj_plan_create_random(1, 2048, list(range(16)), n1=4, bi=2, bo=2)
        t3 = ctx.nj_time_plan(blk, 1, reps=3)
        print("C=16 n1=4: level 3 %.3f ms, level 1 %.3f ms, 2x2 blocks level 1 %.3f ms" % (t1, t2, t3))
        assert 0 < t2 < t1 and t3 > t2
    finally:
        ctx.nj_timing_keys(0)
    assert n == 32768


def test_mlp_save_and_restore():
    """a trained model's parameters and standardisation written out and read back into a
    new model predict the same values"""
    rng = np.random.default_rng(3)
    X = rng.uniform(0, 8, (300, 7)).astype(np.float32)
    y = (0.3 * X[:, 0] + np.sin(X[:, 1]) + 0.1 * X[:, 2] * X[:, 3]).astype(np.float32)
    m = Mlp(seed=9)
    m.train(X, y, epochs=20, batch=64, lr=1e-3, seed=1)
    doc = json.loads(json.dumps(m.to_dict()))
    m2 = Mlp.from_dict(doc)
    assert np.array_equal(m.predict(X), m2.predict(X))
    norm = m.norm()
    assert norm.shape == (16,) and np.all(norm[7:14] > 0) and abs(norm[14] - y.mean()) < 1e-4
    with pytest.raises(NjError):
        bad = norm.copy()
        bad[7] = 0.0
        m2.set_norm(bad)


def test_autotuner_behind_the_abi():
    """nj_tune_split at N = 2^16: exhaustive over the candidate splits, and the committed
    model's shortlist; either choice is at least as fast as the default split as timed"""
    import os
    g = GpuWorkload("full", with_cts=False)
    ctx = g.ctx
    here = os.path.join(os.path.dirname(__file__), "..", "paper_2312_04356_amd", "data", "plan_model_n65536.json")
    with open(here) as fh:
        model = Mlp.from_dict(json.load(fh))
    conv = ctx.nj_plan_create_random(1, 2048, list(range(-33, 34)), n1=0)  # a 3x3 conv's offset spread
    cts = ctx.nj_plan_create_random(23, 1, list(range(-15, 17)), n1=0)  # 32 diagonals at level 23
    with pytest.raises(NjError):  # no keys, no timing mode
        ctx.nj_tune_split(conv, 1, model=None)
    ctx.nj_timing_keys(16)
    try:
        for name, plan, level in (("conv", conv, 1), ("32 diagonals", cts, 23), ("conv at level 15", conv, 15)):
            if level > 1 and name.startswith("conv"):
                plan = ctx.nj_plan_create_random(level, 2048, list(range(-33, 34)), n1=0)
            n1, h, lz, ms, dms = ctx.nj_tune_split(plan, level, model=None, reps=3)
            n1m, hm, _, msm, dmsm = ctx.nj_tune_split(plan, level, model=model, shortlist=3, reps=3)
            n1z, hz, lzz, msz, dmsz = ctx.nj_tune_split(plan, level, model=None, reps=3, lazy=True)
            print("%s at level %d: exhaustive n1=%d hoist=%s %.3f ms, model n1=%d hoist=%s %.3f ms, default %.3f ms; "
                  "with the ModDown form: n1=%d hoist=%s lazy=%s %.3f ms" % (name, level, n1, h, ms, n1m, hm, msm, dms,
                                                                             n1z, hz, lzz, msz))
            assert lz is None and lzz in (False, True)
            assert 0 < ms <= dms and 0 < msm <= dmsm and 0 < msz <= dmsz
            assert n1 == 0 or (n1 & (n1 - 1)) == 0
    finally:
        ctx.nj_timing_keys(0)
