"""Algorithm 1 through the C ABI (needs an MI355X): the tail after CoeffToSlot (ModEval of
Re and Im, zero-padding masks, the square activation, Re + i Im, StoC1) bit-exact
against the oracle at N = 2^12; nj_bootstrap equal word for word to the chain of single
calls; and one whole layer at N = 2^16 (the benchmark conv, the library's masks, the
square) decrypting to the masked square of the conv output's ModEval image."""
import numpy as np
import pytest

import oracle as O
import oracle.bootstrap as B
import oracle.encoding as E
import oracle.plans as PL

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import synth  # noqa: E402
from paper_2312_04356_amd import Ct, nj_layer_masks  # noqa: E402
from paper_2312_04356_amd.workload import GpuWorkload  # noqa: E402
from tests.boot_rig import SCALE, Rig  # noqa: E402
from tests.oracle_workload import OracleWorkload  # noqa: E402

RNG = np.random.default_rng(31)


@pytest.fixture(scope="module")
def rig():
    return Rig()


def eval_form(g, coeffs_rns, level):
    """an oracle plaintext (coefficient form, level+1 limbs) on the device in evaluation form"""
    t = g.to_device(coeffs_rns)
    g.nj_to_eval(t, level, 1)
    return t


def stoc1_plan_from_oracle(rig, ell, groups, level):
    plan = rig.g.nj_stoc1_plan_create(ell, groups, level)
    pts = []
    for t, (bs, diags) in enumerate(B.stoc1_plan(rig.N, ell, groups)):
        pt = PL.encode_diagonals(diags, rig.N, float(rig.q[level - t]), rig.R, level - t)
        for idx, j in enumerate(plan.offsets(t)):
            rig.g.nj_plan_set_diagonal(plan, t, idx, pt[j])
        pts.append((bs, pt))
        for rr in bs.rotations():
            rig.key(PL.galois_elt(rr, rig.N))
    for gl in plan.galois():
        rig.key(gl)
    return plan, pts


@pytest.mark.parametrize("masked,act", [(True, 1), (False, 0), (True, 0)])
def test_slot_activation_parity(rig, masked, act):
    n, N = rig.N // 2, rig.N
    W, C, w0, ell = 32, 4, 16, 512
    lo = 18
    le = lo - 11
    lp = le - (1 if masked else 0) - (1 if act else 0)
    P = rig.q[0] / SCALE
    vals = []
    for sub in (11, 12):
        t = RNG.uniform(-1, 1, n) + P * RNG.integers(-6, 7, n)
        vals.append(rig.enc(t, lo, SCALE, sub))
    (xr, cr), (xi, ci) = vals
    K, r = 16, 3
    coeffs = B.cheb_coeffs(K, r)
    masks_o = masks_d = (None, None)
    if masked:
        mre, mim = B.layer_masks(N, W, C, w0)
        masks_o = tuple(rig.R.to_rns(E.encode(m, N, float(rig.q[le])), le) for m in (mre, mim))
        masks_d = tuple(eval_form(rig.g, m, le) for m in masks_o)
    plan, pts = stoc1_plan_from_oracle(rig, ell, 3, lp)
    want = rig.boot.slot_activation((xr, lo, SCALE), (xi, lo, SCALE), K, r, coeffs,
                                    masks_o if masked else None, act, pts, lp)
    out = rig.g.empty_ct(lp - 3)
    rig.g.nj_slot_activation(K, r, coeffs, masks_d[0], masks_d[1], act, plan, cr, ci, out)
    assert out.level == want[1] == lp - 3 and out.scale == want[2]
    assert np.array_equal(rig.coeff(out), want[0])


def test_bootstrap_call_equals_chain(rig):
    """nj_bootstrap = ModRaise + CoeffToSlot, ModEval of Re and Im, Re + i Im, StoC1"""
    g, N = rig.g, rig.N
    coeffs = RNG.uniform(-1, 1, N)
    m = rig.R.to_rns(np.rint(coeffs * SCALE).astype(np.int64), 0)
    a, e = synth.enc_randomness(rig.q[:1], N, 79, 13)
    ct0 = g.empty_ct(0)
    g.nj_encrypt_sk(g.to_device(m), 0, a, e, SCALE, ct0)
    cts = g.nj_cts_plan_create(2)
    lo = g.L - 2
    stoc1 = g.nj_stoc1_plan_create(512, 3, lo - 11)
    for gl in sorted(set(cts.galois()) | set(stoc1.galois())):
        rig.key(gl)
    out = g.empty_ct(lo - 14)
    g.nj_bootstrap(cts, 16, 3, None, stoc1, ct0, out)
    re, im = g.empty_ct(lo), g.empty_ct(lo)
    g.nj_coeff_to_slot(cts, ct0, re, im)
    er, ei = g.empty_ct(lo - 11), g.empty_ct(lo - 11)
    g.nj_eval_mod(re, 16, 3, None, er)
    g.nj_eval_mod(im, 16, 3, None, ei)
    z = g.empty_ct(lo - 11)
    g.nj_combine(er, ei, z)
    y = g.empty_ct(lo - 14)
    g.nj_stoc1(stoc1, z, y)
    assert out.level == y.level and out.scale == y.scale
    assert torch.equal(out.data, y.data)


def test_conv_act_layer_full_size():
    """the benchmark's conv (3x3 16->16, 32x32 in 64x64, N = 2^16, U(-1, 1) weights and
    inputs, outputs up to ~15) through one Algorithm 1 layer, then the identity kernel's
    fused StoC2 plan back to coefficient layout.  The bound B = 16 of the conv output is
    folded into the conv diagonals (weights / B) and back into the masks (value B), so
    ModEval sees |m / B| <= 1, where its sine departs from the identity by at most
    (2 pi)^2 / (6 P^2) ~ 6e-6 (P = q_0 / scale = 2^10; Sec. 2.4).  The larger term is
    ModEval's own rounding: each rescale at its working scale (~2^48) leaves noise near
    2^-38 in the slots, which the squarings up to T_32, the three double angles (up to 4x
    each) and the factor P / 2 pi amplify about 10^6-fold, to ~3e-5 of B (measured 4.6e-4
    absolute).  That noise has an imaginary part too, and recombining Re + i Im carries
    it onto the other half's coefficients, so padding sees the same magnitude although
    its slots are masked.  Bounds: 1e-3 without activation; 2e-2 with
    the square (Sec. 2.5.2), the same error times 2 |m| <= 30 (measured 5.8e-3)."""
    g = GpuWorkload("full", with_cts=True, lazy=True)
    gctx = g.ctx
    K, B = 32, 16.0
    lo = gctx.L - g.w["cts_groups"]
    le = lo - 11
    lp = le - 2
    stoc1 = gctx.nj_stoc1_plan_create(g.ell, 3, lp)
    s2l = lp - 3
    s2 = gctx.nj_conv_plan_create_taps(g.W, g.C, g.C, [(c, c, 0, 0, 1.0) for c in range(g.C)], fuse=1, level=s2l)
    conv = gctx.nj_conv_plan_create(g.w["w0"], g.w["f"], g.K / B)
    a, e = synth.key_randomness(g.q + g.p, g.N, gctx.dnum, g.w["key_seed"], synth.RELIN_KEY_ID)
    gctx.nj_gen_switch_key(0, a, e)
    g.make_keys(sorted(set(g.galois_elements()) | set(stoc1.galois()) | set(s2.galois())))
    masks = []
    for mk in nj_layer_masks(gctx.log_n, g.W, g.C, g.w["w0"]):
        cf = gctx.nj_encode_slots(B * mk, float(g.q[le]))
        t = torch.empty((le + 1, g.N), dtype=torch.int64, device=gctx.device)
        gctx.nj_upload_plain(cf, le, t)
        gctx.nj_to_eval(t, le, 1)
        masks.append(t)
    ct = g.encrypt_input(1)
    ow = OracleWorkload.__new__(OracleWorkload)  # layout helper only
    ow.w, ow.W, ow.C = g.w, g.W, g.C
    conv_fp64 = PL.conv2d_same(g.img, g.K)
    p = np.arange(g.N) // g.C
    pad = ~((p // g.W < g.w["w0"]) & (p % g.W < g.w["w0"]))
    errs = {}
    for act, want in ((0, conv_fp64), (1, conv_fp64 ** 2)):
        out = gctx.empty_ct(lp - 3)
        gctx.nj_conv_act_layer(conv, g.cts_plan, K, 3, None, masks[0], masks[1], act, stoc1, ct, out)
        assert out.level == lp - 3
        y = gctx.empty_ct(s2l - 1)
        gctx.nj_conv2d_cins(s2, out, y)
        d = torch.empty((y.level + 1, g.N), dtype=torch.int64, device=gctx.device)
        gctx.nj_decrypt(y, d)
        vals = np.array(O.centred_from_limbs(gctx.to_host(d)[:2], g.q[:2]), dtype=np.float64) / y.scale
        got = ow.read_conv_output(vals)
        errs[act] = (np.max(np.abs(got - want)), np.max(np.abs(vals[pad])), np.max(np.abs(want)))
        print("full-size layer, act %d: max |out - exact| %.2e on pixels (max |exact| %.1f), max |out| %.2e on "
              "padding" % (act, errs[act][0], errs[act][2], errs[act][1]))
    assert errs[0][0] < 1e-3 and errs[0][1] < 1e-3
    assert errs[1][0] < 2e-2 and errs[1][1] < 2e-2


def test_slot_activation_full_size_equals_single_calls():
    """at N = 2^16 ModEval of Re and Im runs as one packed evaluation: the tail equals,
    word for word, single-ciphertext ModEval calls followed by Re + i Im and StoC1"""
    g = GpuWorkload("full", with_cts=True, lazy=True)
    gctx = g.ctx
    lo = gctx.L - g.w["cts_groups"]
    stoc1 = gctx.nj_stoc1_plan_create(g.ell, 3, lo - 11)
    a, e = synth.key_randomness(g.q + g.p, g.N, gctx.dnum, g.w["key_seed"], synth.RELIN_KEY_ID)
    gctx.nj_gen_switch_key(0, a, e)
    g.make_keys(sorted(set(g.galois_elements()) | set(stoc1.galois())))
    ct = g.encrypt_input(1)
    y = gctx.empty_ct(0)
    gctx.nj_conv2d_cins(g.conv_plan, ct, y)
    re, im = gctx.empty_ct(lo), gctx.empty_ct(lo)
    gctx.nj_coeff_to_slot(g.cts_plan, y, re, im)
    out = gctx.empty_ct(lo - 14)
    gctx.nj_slot_activation(32, 3, None, None, None, 0, stoc1, re, im, out)
    er, ei, z = gctx.empty_ct(lo - 11), gctx.empty_ct(lo - 11), gctx.empty_ct(lo - 11)
    gctx.nj_eval_mod(re, 32, 3, None, er)
    gctx.nj_eval_mod(im, 32, 3, None, ei)
    gctx.nj_combine(er, ei, z)
    want = gctx.empty_ct(lo - 14)
    gctx.nj_stoc1(stoc1, z, want)
    assert out.level == want.level and out.scale == want.scale
    assert torch.equal(out.data, want.data)


def test_slot_activation_decompose_equals_chain(rig):
    """Algorithm 2's slot-domain part as one call (N = 2^12, W = 32, C = 4): ModEval of Re
    and Im, masks, square, the decomposition of each half into phase images, Re + i Im,
    StoC1 at l/4, word for word equal to the chain of single calls"""
    g, n = rig.g, rig.N // 2
    W, C, w0, lo, K, r = 32, 4, 16, 18, 16, 3
    le = lo - 11
    xs = []
    for sub in (21, 22):
        _, ct = rig.enc(RNG.uniform(-0.5, 0.5, n), lo, SCALE, sub)
        xs.append(ct)
    masks = []
    for mk in nj_layer_masks(rig.R.n.bit_length() - 1, W, C, w0):
        t = torch.empty((le + 1, rig.N), dtype=torch.int64, device=g.device)
        g.nj_upload_plain(g.nj_encode_slots(mk, float(rig.q[le])), le, t)
        g.nj_to_eval(t, le, 1)
        masks.append(t)
    dec = [g.nj_downsample_plan_create(0, W, C, h, le - 2) for h in (0, 1)]
    stoc1 = g.nj_stoc1_plan_create((W // 2) ** 2 // 2, 3, le - 3)
    for gl in sorted(set(dec[0].galois()) | set(dec[1].galois()) | set(stoc1.galois())):
        rig.key(gl)
    out = g.empty_ct(le - 6)
    g.nj_slot_activation_decompose(K, r, None, masks[0], masks[1], 1, dec[0], dec[1], stoc1, xs[0], xs[1], out)
    halves = []
    for h, ct in enumerate(xs):
        e = g.empty_ct(le)
        g.nj_eval_mod(ct, K, r, None, e)
        t, m = g.empty_ct(le), g.empty_ct(le - 1)
        g.nj_pmult(e, masks[h], t)
        g.nj_rescale(t, m)
        m.scale = e.scale
        sq = g.empty_ct(le - 2)
        g.nj_hmult(m, m, sq)
        d = g.empty_ct(le - 3)
        g.nj_conv2d_cins(dec[h], sq, d)
        halves.append(d)
    z = g.empty_ct(le - 3)
    g.nj_combine(halves[0], halves[1], z)
    y = g.empty_ct(le - 6)
    g.nj_stoc1(stoc1, z, y)
    assert out.level == y.level == le - 6 and out.scale == y.scale
    assert torch.equal(out.data, y.data)


def test_block_conv_then_bootstrap_each_full_size():
    """the larger layer's conv (3x3 64 -> 64 at 56 x 56 in 4 ciphertexts of 16 channels,
    W = 64, U(-1, 1) weights and inputs) followed by full bootstrapping of every output
    ciphertext (ModRaise, CoeffToSlot, ModEval of Re and Im, Re + i Im, StoC1), then the
    fused StoC2 identity plan back to coefficient layout.  The outputs reach ~40, so the
    bound B = 64 is folded into the conv (weights / B) and multiplied back after
    decryption: bootstrapping's noise floor (~3e-5 of B) gives ~2e-3 absolute."""
    g = GpuWorkload("full", with_cts=True, lazy=True)
    gctx, N, Bf = g.ctx, g.N, 64.0
    img = RNG.uniform(-1, 1, (64, 56, 56))
    K = RNG.uniform(-1, 1, (64, 64, 3, 3))
    want = PL.conv2d_same(img, K)
    plan = gctx.nj_conv_plan_create_taps(56, 64, 64, PL.taps_same(K / Bf), fuse=True, level=1)
    lvl, W, C, ell, bi, bo = plan.layout()
    assert (W, C, bi, bo) == (64, 16, 4, 4) and ell == g.ell
    le = gctx.L - g.w["cts_groups"] - 11  # ModEval output level
    stoc1 = gctx.nj_stoc1_plan_create(g.ell, 3, le)
    s2 = gctx.nj_conv_plan_create_taps(W, C, C, [(c, c, 0, 0, 1.0) for c in range(C)], fuse=1, level=le - 3)
    a, e = synth.key_randomness(g.q + g.p, N, gctx.dnum, g.w["key_seed"], synth.RELIN_KEY_ID)
    gctx.nj_gen_switch_key(0, a, e)
    g.make_keys(sorted(set(g.galois_elements()) | set(plan.galois()) | set(stoc1.galois()) | set(s2.galois())))
    batch = gctx.empty_batch(bi, 1)
    for ib in range(bi):
        ch = img[ib * C:(ib + 1) * C]
        coeffs = gctx.nj_encode_cins(PL.image_to_slices(ch, W), g.scale)
        m = torch.empty((2, N), dtype=torch.int64, device=gctx.device)
        gctx.nj_upload_plain(coeffs, 1, m)
        ra, re = synth.enc_randomness(g.q[:2], N, 78, 200 + ib)
        gctx.nj_encrypt_sk(m, 1, ra, re, g.scale, Ct(batch.data[ib], 1))
    batch.scale = g.scale
    out = gctx.empty_batch(bo, 0)
    gctx.nj_conv2d_block(plan, batch, out)
    worst = 0.0
    for ob in range(bo):
        z = gctx.empty_ct(le - 3)
        gctx.nj_bootstrap(g.cts_plan, 32, 3, None, stoc1, Ct(out.data[ob], 0, scale=out.scale), z)
        assert z.level == le - 3
        y = gctx.empty_ct(le - 4)
        gctx.nj_conv2d_cins(s2, z, y)
        d = torch.empty((y.level + 1, N), dtype=torch.int64, device=gctx.device)
        gctx.nj_decrypt(y, d)
        vals = np.array(O.centred_from_limbs(gctx.to_host(d)[:2], g.q[:2]), dtype=np.float64) / y.scale
        got = np.zeros((C, 56, 56))
        for c in range(C):
            rc = E.bitrev(c, C)
            for yy in range(56):
                got[c, yy] = vals[(yy * W + np.arange(56)) * C + rc]
        err = np.max(np.abs(Bf * got - want[ob * C:(ob + 1) * C]))
        worst = max(worst, err)
        print("block conv output %d after bootstrapping: max |B out - conv| %.2e (max |conv| %.1f)"
              % (ob, err, np.max(np.abs(want[ob * C:(ob + 1) * C]))))
    assert worst < 1e-2
