"""Batched execution (one key / diagonal read per sub-batch) equals separate calls, bit for bit."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2312_04356_amd.workload import GpuWorkload  # noqa: E402
from tests.midsize import mid_workload  # noqa: E402


def encrypt_many(g, n, level):
    """n distinct fresh ciphertexts: the same image under different encryption randomness"""
    import synth
    coeffs = g.ctx.nj_encode_cins(g.image_slices(), g.scale)
    m = torch.empty((level + 1, g.N), dtype=torch.int64, device=g.ctx.device)
    g.ctx.nj_upload_plain(coeffs, level, m)
    batch = g.ctx.empty_batch(n, level)
    from paper_2312_04356_amd import Ct
    for z in range(n):
        a, e = synth.enc_randomness(g.q[:level + 1], g.N, g.w["data_seed"], 100 + z)
        g.ctx.nj_encrypt_sk(m, level, a, e, g.scale, Ct(batch.data[z], level))
    return batch


@pytest.mark.parametrize("name,n,lazy", [("small", 10, False), ("full", 3, False), ((14, 4), 11, True),
                                         ((15, 3), 9, False)],
                         ids=["small-10", "full-3", "n14_a4-11-lazy", "n15_a3-9"])
def test_batched_conv_and_coeff_to_slot_equal_separate_calls(name, n, lazy):
    """(log_n, alpha) names a ring between the small ring and the benchmark's (12 + alpha
    primes); 9 and 11 ciphertexts run as sub-batches of 8 and the rest"""
    from paper_2312_04356_amd import Ct
    if isinstance(name, tuple):
        name = mid_workload(*name)
    g = GpuWorkload(name, with_cts=True, lazy=lazy)
    gctx = g.ctx
    g.make_keys()
    x = encrypt_many(g, n, 1)
    y = gctx.empty_batch(n, 0)
    gctx.nj_conv2d_cins_batch(g.conv_plan, x, n, y)
    lvl = gctx.L - g.w["cts_groups"]
    re, im = gctx.empty_batch(n, lvl), gctx.empty_batch(n, lvl)
    gctx.nj_coeff_to_slot_batch(g.cts_plan, y, n, re, im)
    torch.cuda.synchronize()
    for z in range(n):
        yz = gctx.empty_ct(0)
        gctx.nj_conv2d_cins(g.conv_plan, Ct(x.data[z], 1), yz)
        assert torch.equal(yz.data, y.data[z]), "conv %d" % z
        rz, iz = gctx.empty_ct(lvl), gctx.empty_ct(lvl)
        gctx.nj_coeff_to_slot(g.cts_plan, yz, rz, iz)
        assert torch.equal(rz.data, re.data[z]) and torch.equal(iz.data, im.data[z]), "cts %d" % z


def test_batched_with_the_cost_models_plan_equals_separate_calls():
    """the trained cost model's first-choice CoeffToSlot plan at full size (N = 2^16; its
    depth, splits and hoisting) with lazy giant steps on the batched calls, 3 ciphertexts,
    equals single calls word for word (single calls of split plans are checked against the
    oracle at this size in test_gpu_plans)"""
    import json

    from bench import PLAN_MODEL
    from paper_2312_04356_amd import Ct, Mlp
    from paper_2312_04356_amd.tune import rank_cts
    g = GpuWorkload("full", with_cts=False)
    gctx = g.ctx
    _, d, n1s, hs = rank_cts(gctx, Mlp.from_dict(json.load(open(PLAN_MODEL))))[0]
    cts = gctx.nj_cts_plan_create_split(d, n1s).set_lazy(True).set_hoist(hs)
    print("plan: depth %d, n1 %s, hoist %s" % (d, n1s, hs), flush=True)
    g.make_keys(sorted(set(g.conv_plan.galois()) | set(cts.galois())))
    n, lvl = 3, gctx.L - d
    x = encrypt_many(g, n, 1)
    y = gctx.empty_batch(n, 0)
    re, im = gctx.empty_batch(n, lvl), gctx.empty_batch(n, lvl)
    gctx.nj_conv2d_cins_batch(g.conv_plan, x, n, y)
    gctx.nj_coeff_to_slot_batch(cts, y, n, re, im)
    torch.cuda.synchronize()
    for z in range(n):
        rz, iz = gctx.empty_ct(lvl), gctx.empty_ct(lvl)
        gctx.nj_coeff_to_slot(cts, Ct(y.data[z], 0), rz, iz)
        assert torch.equal(rz.data, re.data[z]) and torch.equal(iz.data, im.data[z]), "cts %d" % z


def test_batched_galois_equals_separate_calls():
    from paper_2312_04356_amd import Ct
    g = GpuWorkload("small", with_cts=False)
    gctx = g.ctx
    gk = g.conv_plan.galois()[0]
    g.make_keys([gk])
    for level in (7, 3):
        n = 11
        x = gctx.empty_batch(n, level)
        x.data.random_(0, 2 ** 40)
        out = gctx.empty_batch(n, level)
        gctx.nj_apply_galois_batch(x, n, gk, out)
        for z in range(n):
            o = gctx.empty_ct(level)
            gctx.nj_apply_galois(Ct(x.data[z], level), gk, o)
            assert torch.equal(o.data, out.data[z])
