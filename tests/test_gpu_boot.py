"""Bootstrapping after CoeffToSlot through the C ABI (needs an MI355X): HMult with
relinearisation, constant multiplication, ModEval and StoC1 bit-exact against the
oracle at N = 2^12 (21 primes), and whole bootstraps with the library's own plans:
coefficients -> ModRaise -> CoeffToSlot -> ModEval (Re, Im) -> Re + i Im -> StoC1 ->
StoC2 (the fused conv plan of the identity kernel) at N = 2^12, and the full-size conv
of the benchmark workload bootstrapped at N = 2^16."""
import numpy as np
import pytest

import oracle as O
import oracle.bootstrap as B
import oracle.encoding as E
import oracle.plans as PL
from oracle.pipeline import Ctx as OCtx

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import synth  # noqa: E402
from paper_2312_04356_amd import Ct, Ctx, chain_primes, nj_cheb_interpolate  # noqa: E402
from paper_2312_04356_amd.workload import GpuWorkload  # noqa: E402
from tests.boot_rig import Rig  # noqa: E402
from tests.oracle_workload import OracleWorkload  # noqa: E402

RNG = np.random.default_rng(29)
SCALE = 2.0 ** 40


@pytest.fixture(scope="module")
def rig():
    return Rig()


def test_hmult_parity(rig):
    n = rig.N // 2
    xa, ca = rig.enc(RNG.uniform(-1, 1, n), 12, 2.0 ** 45, 1)
    xb, cb = rig.enc(RNG.uniform(-1, 1, n), 9, 2.0 ** 44, 2)
    for (A, a), (Bo, b) in [((xa, ca), (xb, cb)), ((xa, ca), (xa, ca))]:
        want = rig.boot.hmult((A, a.level, a.scale), (Bo, b.level, b.scale))
        out = rig.g.empty_ct(min(a.level, b.level) - 1)
        rig.g.nj_hmult(a, b, out)
        assert out.level == want[1] and out.scale == want[2]
        assert np.array_equal(rig.coeff(out), want[0])


def test_hmult_parity_full():
    """N = 2^16 (24 + 8 primes, three digits): HMult's relinearisation runs on the fused
    key-switch kernels (digits' tile pass inside the inner product, special-prime rows
    handed to ModDown), word for word against the oracle"""
    full = Rig(16, 24, 8, 192)
    n = full.N // 2
    xa, ca = full.enc(RNG.uniform(-1, 1, n), 14, 2.0 ** 45, 5)
    xb, cb = full.enc(RNG.uniform(-1, 1, n), 12, 2.0 ** 44, 6)
    want = full.boot.hmult((xa, ca.level, ca.scale), (xb, cb.level, cb.scale))
    out = full.g.empty_ct(11)
    full.g.nj_hmult(ca, cb, out)
    assert out.level == want[1] == 11 and out.scale == want[2]
    assert np.array_equal(full.coeff(out), want[0])


def test_const_mult_and_add_const_parity(rig):
    n = rig.N // 2
    xa, ca = rig.enc(RNG.uniform(-1, 1, n), 10, 2.0 ** 46, 3)
    want = rig.boot.const_mult((xa, 10, ca.scale), -0.3125, 6, 2.0 ** 47)
    out = rig.g.empty_ct(6)
    rig.g.nj_mul_const(ca, -0.3125, 6, 2.0 ** 47, out)
    assert np.array_equal(rig.coeff(out), want[0])
    w2 = rig.boot.add_const(want, 0.75)
    rig.g.nj_add_const(out, 0.75)
    assert np.array_equal(rig.coeff(out), w2[0])


def test_eval_mod_parity_and_accuracy(rig):
    n = rig.N // 2
    P = rig.q[0] / SCALE
    m = RNG.uniform(-1, 1, n)
    t = m + P * RNG.integers(-6, 7, n)
    xo, ct = rig.enc(t, 20, SCALE, 4)
    K, r = 16, 3
    coeffs = B.cheb_coeffs(K, r)
    want = rig.boot.eval_mod((xo, 20, SCALE), K, r, coeffs)
    out = rig.g.empty_ct(9)
    rig.g.nj_eval_mod(ct, K, r, coeffs, out)
    assert out.level == want[1] == 9 and out.scale == want[2]
    assert np.array_equal(rig.coeff(out), want[0])
    # the library's own interpolant
    own = nj_cheb_interpolate(63, K, r)
    assert np.max(np.abs(own - coeffs)) < 1e-13
    out2 = rig.g.empty_ct(9)
    rig.g.nj_eval_mod(ct, K, r, None, out2)
    z = rig.dec_slots(out2).real
    err_model = np.max(np.abs(z - B.model(t, P, K, r, own)))
    err_m = np.max(np.abs(z - m))
    print("ModEval (library interpolant): |z - model| %.2e, |z - m| %.2e" % (err_model, err_m))
    assert err_model < 2.0 ** -15 and err_m < 1e-4


def test_stoc1_parity(rig):
    n, ell, lvl = rig.N // 2, 512, 12
    plan = rig.g.nj_stoc1_plan_create(ell, 3, lvl)
    oplan = B.stoc1_plan(rig.N, ell, 3)
    pts = []
    for t, (bs, diags) in enumerate(oplan):
        assert sorted(plan.offsets(t)) == sorted(bs.js)
        pt = PL.encode_diagonals(diags, rig.N, float(rig.q[lvl - t]), rig.R, lvl - t)
        for idx, j in enumerate(plan.offsets(t)):
            rig.g.nj_plan_set_diagonal(plan, t, idx, pt[j])
        pts.append((bs, pt))
    for gl in plan.galois():
        rig.key(gl)
    for bs, _ in oplan:
        for rr in bs.rotations():
            rig.key(PL.galois_elt(rr, rig.N))
    z = RNG.normal(size=n) + 1j * RNG.normal(size=n)
    xo, ct = rig.enc(z * 0.25, lvl, SCALE, 5)
    want = rig.boot.stoc1((xo, lvl, SCALE), pts)
    out = rig.g.empty_ct(lvl - 3)
    rig.g.nj_stoc1(plan, ct, out)
    assert out.level == want[1]
    assert np.array_equal(rig.coeff(out), want[0])


def bootstrap(g, ct0, cts_plan, K, stoc1, s2_plan, s2_level):
    """ModRaise + CoeffToSlot, ModEval on Re and Im, Re + i Im, StoC1, StoC2 (conv plan)"""
    lo = g.L - cts_plan.count()
    re, im = g.empty_ct(lo), g.empty_ct(lo)
    g.nj_coeff_to_slot(cts_plan, ct0, re, im)
    er, ei = g.empty_ct(lo - 11), g.empty_ct(lo - 11)
    g.nj_eval_mod(re, K, 3, None, er)
    g.nj_eval_mod(im, K, 3, None, ei)
    z = g.empty_ct(lo - 11)
    g.nj_combine(er, ei, z)
    y = g.empty_ct(lo - 11 - stoc1.count())
    g.nj_stoc1(stoc1, z, y)
    if y.level > s2_level:
        y2 = g.empty_ct(s2_level)
        g.nj_drop_level(y, s2_level, y2)
        y = y2
    out = g.empty_ct(s2_level - 1)
    g.nj_conv2d_cins(s2_plan, y, out)
    return out


def test_bootstrap_round_trip_small(rig):
    """coefficients (|c| < 1, scale 2^40, level 0) bootstrapped with the library's own
    plans: CoeffToSlot in 2 groups, StoC1 for l = 512 in 3 groups, StoC2 as the fused
    conv plan of the identity kernel (C = 4, W = 32)"""
    g, N = rig.g, rig.N
    coeffs = RNG.uniform(-1, 1, N)
    m = rig.R.to_rns(np.rint(coeffs * SCALE).astype(np.int64), 0)
    a, e = synth.enc_randomness(rig.q[:1], N, 79, 6)
    ct0 = g.empty_ct(0)
    g.nj_encrypt_sk(g.to_device(m), 0, a, e, SCALE, ct0)
    cts = g.nj_cts_plan_create(2)
    lo = g.L - 2
    stoc1 = g.nj_stoc1_plan_create(512, 3, lo - 11)
    s2 = g.nj_conv_plan_create_taps(32, 4, 4, [(c, c, 0, 0, 1.0) for c in range(4)], fuse=1, level=lo - 14)
    for gl in sorted(set(cts.galois()) | set(stoc1.galois()) | set(s2.galois())):
        rig.key(gl)
    out = bootstrap(g, ct0, cts, 16, stoc1, s2, lo - 14)
    d = torch.empty((out.level + 1, N), dtype=torch.int64, device=g.device)
    g.nj_decrypt(out, d)
    got = np.array(O.centred_from_limbs(g.to_host(d)[:2], rig.q[:2]), dtype=np.float64) / out.scale
    err = np.max(np.abs(got - coeffs))
    print("bootstrap round trip N=2^12: output level %d, max coefficient error %.2e" % (out.level, err))
    assert err < 1e-4


def test_bootstrap_full_size_conv():
    """the benchmark's conv (3x3 16->16 on 32x32, N = 2^16) -> bootstrap -> the conv
    output back in coefficient layout at level 5, against the function ModEval
    evaluates, (P / 2 pi) sin(2 pi o / P) with P = q_0 / scale, of the FP64 conv2d o"""
    g = GpuWorkload("full", with_cts=True)
    gctx = g.ctx
    K = 32  # |I| (about 4.5 standard deviations of sqrt(h / 12) for h = 192) stays below K
    lo = gctx.L - g.w["cts_groups"]
    stoc1 = gctx.nj_stoc1_plan_create(g.ell, 3, lo - 11)
    s2l = lo - 14
    # the identity kernel has no reach: width W itself gives the workload's layout (W = 64)
    s2 = gctx.nj_conv_plan_create_taps(g.W, g.C, g.C, [(c, c, 0, 0, 1.0) for c in range(g.C)], fuse=1, level=s2l)
    assert s2.layout()[1:3] == (g.W, g.C)
    a, e = synth.key_randomness(g.q + g.p, g.N, gctx.dnum, g.w["key_seed"], synth.RELIN_KEY_ID)
    gctx.nj_gen_switch_key(0, a, e)
    g.make_keys(sorted(set(g.galois_elements()) | set(stoc1.galois()) | set(s2.galois())))
    ct = g.encrypt_input(1)
    y = gctx.empty_ct(0)
    gctx.nj_conv2d_cins(g.conv_plan, ct, y)
    out = bootstrap(gctx, y, g.cts_plan, K, stoc1, s2, s2l)
    d = torch.empty((out.level + 1, g.N), dtype=torch.int64, device=gctx.device)
    gctx.nj_decrypt(out, d)
    vals = np.array(O.centred_from_limbs(gctx.to_host(d)[:2], g.q[:2]), dtype=np.float64) / out.scale
    ow = OracleWorkload.__new__(OracleWorkload)  # layout helper only
    ow.w, ow.W, ow.C = g.w, g.W, g.C
    conv = PL.conv2d_same(g.img, g.K)
    P = g.q[0] / g.scale
    got = ow.read_conv_output(vals)
    err = np.max(np.abs(got - P / (2 * np.pi) * np.sin(2 * np.pi * conv / P)))
    print("full-size conv + bootstrap: output level %d, max |out - (P/2pi) sin(2pi o/P)| %.2e, max |out - o| %.2e"
          % (out.level, err, np.max(np.abs(got - conv))))
    assert err < 1e-3
