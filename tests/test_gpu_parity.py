"""HIP path vs oracle, bit for bit, through the C ABI (needs an MI355X).

Every comparison is made in coefficient form on identical integer inputs
(primes, secret, key randomness, plaintext residues, plan diagonals): the HIP
library's output must equal the oracle's word for word.  Accuracy checks of the
library's own encoder and plan builder compare decrypted results with plain
FP64 conv2d (bound 2^-15 at scale 2^40) and with the bit-reversed coefficients
CoeffToSlot must produce (Sec. 2.4).
"""
import numpy as np
import pytest

import oracle as O
import oracle.encoding as E

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import synth  # noqa: E402
from paper_2312_04356_amd.workload import GpuWorkload  # noqa: E402
from tests.oracle_workload import OracleWorkload  # noqa: E402

RNG = np.random.default_rng(11)


class Pair:
    def __init__(self, name, with_cts):
        print("\n[setup] workload %s (cts=%s)" % (name, with_cts), flush=True)
        self.o = OracleWorkload(name, with_cts=with_cts)
        self.g = GpuWorkload(name, with_cts=with_cts)
        assert self.g.q == self.o.ring.q and self.g.p == self.o.ring.p
        self.N = self.g.N
        self.oracle_keys = set()

    def oracle_key(self, g):
        if g not in self.oracle_keys:
            self.o.make_keys([g])
            self.oracle_keys.add(g)
        return self.o.ctx.keys[g]


@pytest.fixture(scope="module")
def small():
    return Pair("small", True)


@pytest.fixture(scope="module")
def full():
    return Pair("full", False)


def host_coeff(gctx, ct):
    t = ct.data.clone()
    gctx.nj_to_coeff(t, ct.level, 2)
    torch.cuda.synchronize()
    return gctx.to_host(t)


def dev_eval(gctx, arr, level, n_polys):
    t = gctx.to_device(np.ascontiguousarray(arr, dtype=np.uint64))
    gctx.nj_to_eval(t, level, n_polys)
    return t


def rand_res(primes, n):
    return np.stack([RNG.integers(0, q, n, dtype=np.uint64) for q in primes])


# ------------------------------------------------------------------ transforms

@pytest.mark.parametrize("which", ["small", "full"])
def test_ntt_roundtrip(which, request):
    P = request.getfixturevalue(which)
    gctx = P.g.ctx
    primes = P.g.q + P.g.p
    idx = list(range(len(primes)))
    a = rand_res(primes, P.N)
    t = gctx.to_device(a)
    gctx.nj_ntt_limbs(t, idx, 0)
    fwd = gctx.to_host(t)
    assert not np.array_equal(fwd, a)
    assert all(int(fwd[i].max()) < primes[i] for i in idx)
    gctx.nj_ntt_limbs(t, idx, 1)
    assert np.array_equal(gctx.to_host(t), a)


@pytest.mark.parametrize("which,level", [("small", 7), ("full", 2)])
def test_pmult_equals_negacyclic_product(which, level, request):
    P = request.getfixturevalue(which)
    gctx, R = P.g.ctx, P.o.ring
    q = P.g.q[:level + 1]
    ct = np.stack([rand_res(q, P.N), rand_res(q, P.N)])
    pt = rand_res(q, P.N)
    d_ct = dev_eval(gctx, ct, level, 2)
    d_pt = dev_eval(gctx, pt, level, 1)
    from paper_2312_04356_amd import Ct
    x = Ct(d_ct, level)
    out = gctx.empty_ct(level)
    gctx.nj_pmult(x, d_pt, out)
    got = host_coeff(gctx, out)
    for k in range(2):
        assert np.array_equal(got[k], R.pmult(level, ct[k], pt))


# ------------------------------------------------------------ encryption

@pytest.mark.parametrize("which", ["small", "full"])
def test_encrypt_decrypt_parity(which, request):
    P = request.getfixturevalue(which)
    gctx, R = P.g.ctx, P.o.ring
    level = 1
    m = R.to_rns(P.o.input_plaintext(), level)
    ct_o = P.o.encrypt_input(level)
    ct_g = P.g.encrypt_input(level, m_dev=gctx.to_device(m))
    assert np.array_equal(host_coeff(gctx, ct_g), ct_o)
    dec = torch.empty((level + 1, P.N), dtype=torch.int64, device=gctx.device)
    gctx.nj_decrypt(ct_g, dec)
    assert np.array_equal(gctx.to_host(dec), R.decrypt(level, P.o.s, ct_o))


@pytest.mark.parametrize("which,level", [("small", 3), ("full", 1), ("full", 23)])
def test_public_key_encryption_parity(which, level, request):
    """Sec. 2.1: the public key and Enc(m; pk) word for word against the oracle, and the
    decryption polynomial too"""
    import synth
    P = request.getfixturevalue(which)
    gctx, R = P.g.ctx, P.o.ring
    a, e = synth.pk_randomness(R.q, P.N, 31)
    gctx.nj_gen_public_key(a, e)
    pk = R.gen_public_key(P.o.s, a, e)
    m = R.to_rns(P.o.input_plaintext(), level)
    v, e0, e1 = synth.pk_enc_randomness(P.N, 32, level)
    ct_g = gctx.nj_encrypt_pk(gctx.to_device(m), level, v, e0, e1, 2.0 ** 40, gctx.empty_ct(level))
    ct_o = R.encrypt_pk(level, pk, m, v, e0, e1)
    assert ct_g.level == level and ct_g.scale == 2.0 ** 40
    assert np.array_equal(host_coeff(gctx, ct_g), ct_o)
    dec = torch.empty((level + 1, P.N), dtype=torch.int64, device=gctx.device)
    gctx.nj_decrypt(ct_g, dec)
    assert np.array_equal(gctx.to_host(dec), R.decrypt(level, P.o.s, ct_o))


# ----------------------------------------------------------- key switching

@pytest.mark.parametrize("which,level", [("small", 0), ("small", 4), ("small", 7), ("full", 1), ("full", 23)])
def test_keyswitch_parity(which, level, request):
    P = request.getfixturevalue(which)
    gctx, R = P.g.ctx, P.o.ring
    g = P.g.conv_plan.galois()[0]
    P.g.make_keys([g])
    key = P.oracle_key(g)
    d = rand_res(P.g.q[:level + 1], P.N)
    d_dev = dev_eval(gctx, d, level, 1)
    o0 = torch.empty((level + 1, P.N), dtype=torch.int64, device=gctx.device)
    o1 = torch.empty_like(o0)
    gctx.nj_keyswitch(d_dev, level, g, o0, o1)
    gctx.nj_to_coeff(o0, level, 1)
    gctx.nj_to_coeff(o1, level, 1)
    w0, w1 = R.keyswitch(level, d, key)
    assert np.array_equal(gctx.to_host(o0), w0)
    assert np.array_equal(gctx.to_host(o1), w1)


@pytest.mark.parametrize("which", ["small", "full"])
def test_rotation_parity(which, request):
    """rotations and an in-place conjugation (one key switch each) at level 1"""
    P = request.getfixturevalue(which)
    gctx = P.g.ctx
    level = 1
    m = P.o.ring.to_rns(P.o.input_plaintext(), level)
    ct_o = P.o.encrypt_input(level)
    ct_g = P.g.encrypt_input(level, m_dev=gctx.to_device(m))
    for r in (P.o.ell, 3 * P.o.ell):
        g = gctx.nj_galois_elt(r)
        P.g.make_keys([g])
        P.oracle_key(g)
        out = gctx.empty_ct(level)
        gctx.nj_rotate(ct_g, r, out)
        assert np.array_equal(host_coeff(gctx, out), P.o.ctx.rotate(level, ct_o, r))
    # conjugation through apply_galois, in place
    g = 2 * P.N - 1
    P.g.make_keys([g])
    P.oracle_key(g)
    gctx.nj_apply_galois(ct_g, g, ct_g)
    assert np.array_equal(host_coeff(gctx, ct_g), P.o.ctx.apply_galois(level, ct_o, g))


@pytest.mark.parametrize("which,level", [("small", 7), ("small", 1), ("full", 23), ("full", 1)])
def test_rescale_and_modraise_parity(which, level, request):
    P = request.getfixturevalue(which)
    gctx, R = P.g.ctx, P.o.ring
    q = P.g.q[:level + 1]
    ct = np.stack([rand_res(q, P.N), rand_res(q, P.N)])
    from paper_2312_04356_amd import Ct
    x = Ct(dev_eval(gctx, ct, level, 2), level)
    out = gctx.empty_ct(level - 1)
    gctx.nj_rescale(x, out)
    want = np.stack([R.rescale(level, ct[0]), R.rescale(level, ct[1])])
    assert np.array_equal(host_coeff(gctx, out), want)
    ct0 = np.stack([rand_res(P.g.q[:1], P.N), rand_res(P.g.q[:1], P.N)])
    y = Ct(dev_eval(gctx, ct0, 0, 2), 0)
    up = gctx.empty_ct(R.L)
    gctx.nj_modraise(y, R.L, up)
    want = np.stack([R.modraise(ct0[0][0]), R.modraise(ct0[1][0])])
    assert np.array_equal(host_coeff(gctx, up), want)


# ---------------------------------------------------- BSGS, conv, CoeffToSlot

def load_oracle_diagonals(gctx, plan, t, pts):
    for idx, j in enumerate(plan.offsets(t)):
        gctx.nj_plan_set_diagonal(plan, t, idx, pts[j])


@pytest.mark.parametrize("which", ["small", "full"])
def test_fused_conv_parity(which, request):
    P = request.getfixturevalue(which)
    gctx = P.g.ctx
    gs = P.g.conv_plan.galois()
    P.g.make_keys(gs)
    for g in gs:
        P.oracle_key(g)
    assert sorted(P.o.conv_bsgs.js) == sorted(P.g.conv_plan.offsets(0))
    load_oracle_diagonals(gctx, P.g.conv_plan, 0, P.o.conv_pts)
    m = P.o.ring.to_rns(P.o.input_plaintext(), 1)
    ct_o = P.o.encrypt_input(1)
    ct_g = P.g.encrypt_input(1, m_dev=gctx.to_device(m))
    for hoist in (1, 0):
        y = gctx.empty_ct(1)
        gctx.nj_plan_apply(P.g.conv_plan, 0, ct_g, y, hoist)
        want = P.o.ctx.bsgs(1, ct_o, P.o.conv_bsgs, P.o.conv_pts, hoist=bool(hoist))
        assert np.array_equal(host_coeff(gctx, y), want), "hoist=%d" % hoist
    # lazy giant steps (one ModDown for their sum), as the benchmark runs the conv
    P.g.conv_plan.set_lazy(True)
    y = gctx.empty_ct(1)
    gctx.nj_plan_apply(P.g.conv_plan, 0, ct_g, y, 1)
    assert np.array_equal(host_coeff(gctx, y), P.o.ctx.bsgs(1, ct_o, P.o.conv_bsgs, P.o.conv_pts, lazy=True))
    out = gctx.empty_ct(0)
    gctx.nj_conv2d_cins(P.g.conv_plan, ct_g, out)
    want = P.o.ctx.conv2d_cins(ct_o, P.o.conv_bsgs, P.o.conv_pts, level=1, hoist=True, lazy=True)
    assert np.array_equal(host_coeff(gctx, out), want)
    P.g.conv_plan.set_lazy(False)
    out = gctx.empty_ct(0)
    gctx.nj_conv2d_cins(P.g.conv_plan, ct_g, out)
    want = P.o.ctx.conv2d_cins(ct_o, P.o.conv_bsgs, P.o.conv_pts, level=1, hoist=True)
    assert np.array_equal(host_coeff(gctx, out), want)
    P.conv_out = (out, want)


def test_coeff_to_slot_parity(small):
    P = small
    gctx = P.g.ctx
    if not hasattr(P, "conv_out"):
        pytest.skip("needs test_fused_conv_parity[small] first")
    gs = P.g.cts_plan.galois()
    P.g.make_keys(gs)
    for g in gs:
        P.oracle_key(g)
    for t, (plan, pts) in enumerate(P.o.cts):
        assert sorted(plan.js) == sorted(P.g.cts_plan.offsets(t))
        load_oracle_diagonals(gctx, P.g.cts_plan, t, pts)
    ct_g, ct_o = P.conv_out
    lvl = P.o.ring.L - len(P.o.cts)
    re, im = gctx.empty_ct(lvl), gctx.empty_ct(lvl)
    gctx.nj_coeff_to_slot(P.g.cts_plan, ct_g, re, im)
    w_re, w_im = P.o.ctx.coeff_to_slot(ct_o, [p for p, _ in P.o.cts], [pts for _, pts in P.o.cts])
    assert np.array_equal(host_coeff(gctx, re), w_re)
    assert np.array_equal(host_coeff(gctx, im), w_im)


# --------------------------------------- the library's own encoder and plans

def centred(vals, q):
    v = vals.astype(np.int64)
    return np.where(vals > q // 2, v - np.int64(q), v)


def raw_modraised(ct0_coeff, s, q0):
    """c0 + c1 s over the integers for a level-0 ciphertext (coefficient form): m + q0 I"""
    c0, c1 = centred(ct0_coeff[0][0], q0), centred(ct0_coeff[1][0], q0)
    prod = np.zeros_like(c0)
    for i in np.nonzero(s)[0]:
        sh = np.roll(c1, i)
        sh[:i] = -sh[:i]
        prod += int(s[i]) * sh
    return c0 + prod


@pytest.mark.parametrize("which", ["small", "full"])
def test_own_plans_conv_and_coeff_to_slot_accuracy(which):
    g = GpuWorkload(which, with_cts=True)
    gctx = g.ctx
    g.make_keys()
    ct = g.encrypt_input(1)
    out = gctx.empty_ct(0)
    gctx.nj_conv2d_cins(g.conv_plan, ct, out)
    dec = torch.empty((1, g.N), dtype=torch.int64, device=gctx.device)
    gctx.nj_decrypt(out, dec)
    vals = centred(gctx.to_host(dec)[0], g.q[0]).astype(np.float64) / g.scale
    ow = OracleWorkload.__new__(OracleWorkload)  # only the layout helpers
    ow.w, ow.W, ow.C = g.w, g.W, g.C
    got = ow.read_conv_output(vals)
    from oracle.plans import conv2d_same
    err = np.max(np.abs(got - conv2d_same(g.img, g.K)))
    print("conv max abs error %.3e" % err)
    assert err <= 2.0 ** -15
    # CoeffToSlot: slots hold the bit-reversed coefficient halves of m + q0 I
    lvl = g.ctx.L - g.w["cts_groups"]
    re, im = gctx.empty_ct(lvl), gctx.empty_ct(lvl)
    gctx.nj_coeff_to_slot(g.cts_plan, out, re, im)
    raw = raw_modraised(host_coeff(gctx, out), g.s, g.q[0]).astype(np.float64) / g.scale
    n = g.N // 2
    rev = np.array([E.bitrev(j, n) for j in range(n)])
    for ctx_ct, want in ((re, raw[:n][rev]), (im, raw[n:][rev])):
        d = torch.empty((lvl + 1, g.N), dtype=torch.int64, device=gctx.device)
        gctx.nj_decrypt(ctx_ct, d)
        m = O.centred_from_limbs(gctx.to_host(d)[:2], g.q[:2])
        z = gctx.nj_decode_slots(np.array(m, dtype=np.float64), g.scale)
        err = max(np.max(np.abs(z.real - want)), np.max(np.abs(z.imag)))
        print("CoeffToSlot max abs slot error %.3e" % err)
        assert err < 1e-3
