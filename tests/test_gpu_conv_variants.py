"""Conv variants through the C ABI (needs an MI355X): block convs over several
ciphertexts (Sec. 3.3.4), pointwise, stride 2 by polyphase decomposition, and
depthwise (one PMult) followed by a separate StoC2 transform.

Bit-exact: the library's block BSGS evaluated with the oracle's diagonals on the
oracle's ciphertexts equals `oracle.pipeline.block_conv` word for word.
Accuracy: the library's own plans (its own encoder and plan builder) decrypt to the
plain FP64 convolution within 2^-15 at scale 2^40, at N = 2^12 and at N = 2^16
(64 -> 64 channels at 56 x 56 in 4 ciphertexts; 64 -> 128 stride 2 to 28 x 28).
"""
import numpy as np
import pytest

import oracle as O
import oracle.encoding as E
import oracle.plans as PL
from oracle.pipeline import block_conv

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import synth  # noqa: E402
from paper_2312_04356_amd import Ct  # noqa: E402
from paper_2312_04356_amd.workload import GpuWorkload  # noqa: E402
from tests.oracle_workload import OracleWorkload  # noqa: E402

RNG = np.random.default_rng(23)
BOUND = 2.0 ** -15


class Rig:
    def __init__(self, name, with_oracle):
        print("\n[setup] conv variants on workload %s" % name, flush=True)
        self.g = GpuWorkload(name, with_cts=False)
        self.o = OracleWorkload(name, with_cts=False) if with_oracle else None
        self.N, self.scale, self.q = self.g.N, self.g.scale, self.g.q
        self.okeys = set()

    def keys(self, gs):
        self.g.make_keys(gs)
        if self.o is not None:
            new = [g for g in gs if g not in self.okeys]
            self.o.make_keys(new)
            self.okeys |= set(new)


@pytest.fixture(scope="module")
def small():
    return Rig("small", True)


@pytest.fixture(scope="module")
def full():
    return Rig("full", False)


def cins_plaintext(chans, W, N, scale):
    ell = W * W // 2
    return E.encode(E.real_cins_slots(PL.image_to_slices(chans, W), ell), N, scale)


def encrypt_blocks(rig, img, W, level, with_oracle):
    """channel blocks of img (C per ciphertext) -> device batch [bi][2][level+1][N]
    (and the oracle's ciphertexts from the same residues and randomness)"""
    N, gctx = rig.N, rig.g.ctx
    C = N // (W * W)
    bi = -(-img.shape[0] // C)
    batch = gctx.empty_batch(bi, level)
    xs = []
    for ib in range(bi):
        ch = np.zeros((C,) + img.shape[1:])
        part = img[ib * C:(ib + 1) * C]
        ch[:part.shape[0]] = part
        a, e = synth.enc_randomness(rig.q[:level + 1], N, 77, 100 + ib)
        if with_oracle:
            m = rig.o.ring.to_rns(cins_plaintext(ch, W, N, rig.scale), level)
            xs.append(rig.o.ring.encrypt_sk(level, rig.o.s, m, a, e))
            m_dev = gctx.to_device(m)
        else:
            coeffs = gctx.nj_encode_cins(PL.image_to_slices(ch, W), rig.scale)  # the library's encoder
            m_dev = torch.empty((level + 1, N), dtype=torch.int64, device=gctx.device)
            gctx.nj_upload_plain(coeffs, level, m_dev)
        gctx.nj_encrypt_sk(m_dev, level, a, e, rig.scale, Ct(batch.data[ib], level))
    batch.scale = rig.scale
    return xs, batch


def host_coeff_batch(gctx, batch, n):
    t = batch.data.clone()
    gctx.nj_to_coeff(t, batch.level, 2 * n)
    torch.cuda.synchronize()
    return gctx.to_host(t)


def read_layout(vals, W, C, w0):
    out = np.zeros((C, w0, w0))
    for c in range(C):
        rc = E.bitrev(c, C)
        for y in range(w0):
            out[c, y] = vals[(y * W + np.arange(w0)) * C + rc]
    return out


def decrypt_outputs(rig, batch, n, W, w0):
    gctx = rig.g.ctx
    C = rig.N // (W * W)
    res = []
    for z in range(n):
        d = torch.empty((1, rig.N), dtype=torch.int64, device=gctx.device)
        gctx.nj_decrypt(Ct(batch.data[z], batch.level), d)
        vals = np.array(O.centred_from_limbs(gctx.to_host(d), rig.q[:1]), dtype=np.float64) / rig.scale
        res.append(read_layout(vals, W, C, w0))
    return np.concatenate(res)


def load_oracle_blocks(rig, plan, ob_plan, bi, bo, pts, level):
    """the oracle's residues replace the library's diagonals; where the oracle has
    none (a zero diagonal) the library's own zero diagonal, skipped, stays"""
    gctx = rig.g.ctx
    js = plan.offsets(0)
    assert sorted(js) == sorted(ob_plan.js)
    for ob in range(bo):
        for ib in range(bi):
            for d, j in enumerate(js):
                if j in pts[(ob, ib)]:
                    gctx.nj_plan_set_diagonal(plan, 0, (ob * bi + ib) * len(js) + d, pts[(ob, ib)][j])


def run_parity(rig, img, taps, c_in, c_out, w0, fuse=True, level=1):
    """library block conv with the oracle's diagonals == oracle block_conv, bit for bit"""
    N, gctx, R = rig.N, rig.g.ctx, rig.o.ring
    plan = gctx.nj_conv_plan_create_taps(w0, c_in, c_out, taps, fuse=fuse, level=level)
    lvl, W, C, ell, bi, bo = plan.layout()
    assert lvl == level and W == PL.padded_width_taps(w0, taps)
    rig.keys(plan.galois())
    oplan, obi, obo, diags = PL.block_conv_plan(taps, c_in, c_out, W, N, fuse)
    assert (obi, obo) == (bi, bo)
    pts = {k: PL.encode_diagonals(v, N, float(rig.q[level]), R, level) for k, v in diags.items()}
    load_oracle_blocks(rig, plan, oplan, bi, bo, pts, level)
    xs, batch = encrypt_blocks(rig, img, W, level, True)
    assert np.array_equal(host_coeff_batch(gctx, batch, bi), np.stack(xs))
    out = gctx.empty_batch(bo, level - 1)
    gctx.nj_conv2d_block(plan, batch, out)
    want = block_conv(rig.o.ctx, level, xs, oplan, pts, bo)
    got = host_coeff_batch(gctx, out, bo)
    for ob in range(bo):
        assert np.array_equal(got[ob], want[ob]), "output block %d" % ob
    return plan, W, out, want


# ------------------------------------------------------------- bit-exact, N = 2^12

@pytest.mark.parametrize("c_in,c_out", [(8, 8), (12, 6)])
def test_block_conv_parity(small, c_in, c_out):
    """3x3 conv over 2 or 3 input and 2 output ciphertexts (C = 4 channels each)"""
    w0 = 24
    img = RNG.uniform(-1, 1, (c_in, w0, w0))
    K = RNG.uniform(-1, 1, (c_out, c_in, 3, 3))
    _, W, out, _ = run_parity(small, img, PL.taps_same(K), c_in, c_out, w0)
    got = decrypt_outputs(small, out, out.data.shape[0], W, w0)[:c_out]
    assert np.max(np.abs(got - PL.conv2d_same(img, K))) <= BOUND


def test_pointwise_conv_parity(small):
    w0, c = 24, 4
    img = RNG.uniform(-1, 1, (c, w0, w0))
    K = RNG.uniform(-1, 1, (c, c, 1, 1))
    _, W, out, _ = run_parity(small, img, PL.taps_same(K), c, c, w0)
    assert W == 32
    got = decrypt_outputs(small, out, 1, W, w0)
    assert np.max(np.abs(got - PL.conv2d_same(img, K))) <= BOUND


def test_stride2_conv_parity(small):
    """stride-2 3x3 conv 2 -> 4 channels, 48 x 48 -> 24 x 24, as a unit-stride conv
    over the 8 polyphase channels (two input ciphertexts)"""
    img = RNG.uniform(-1, 1, (2, 48, 48))
    K = RNG.uniform(-1, 1, (4, 2, 3, 3))
    taps = PL.taps_stride2(K)
    _, W, out, _ = run_parity(small, PL.polyphase(img), taps, 8, 4, 24)
    got = decrypt_outputs(small, out, 1, W, 24)[:4]
    assert np.max(np.abs(got - PL.conv2d_strided(img, K, 2))) <= BOUND


def test_depthwise_then_stoc2_parity(small):
    """depthwise 3x3 (one diagonal per block, one PMult, no rotation) at level 2,
    then StoC2 as its own transform at level 1; 8 channels in 2 ciphertexts"""
    w0, c = 24, 8
    img = RNG.uniform(-1, 1, (c, w0, w0))
    Kd = RNG.uniform(-1, 1, (c, 3, 3))
    taps = PL.taps_depthwise(Kd)
    plan, W, mid, mid_o = run_parity(small, img, taps, c, c, w0, fuse=False, level=2)
    assert plan.galois() == [] and len(plan.offsets(0)) == 1
    # StoC2: the fused plan of the identity kernel, applied to the depthwise output
    gctx, R = small.g.ctx, small.o.ring
    ident = [(ch, ch, 0, 0, 1.0) for ch in range(c)]
    s2 = gctx.nj_conv_plan_create_taps(W, c, c, ident, fuse=True, level=1)
    small.keys(s2.galois())
    oplan, bi, bo, diags = PL.block_conv_plan(ident, c, c, W, small.N, True)
    pts = {k: PL.encode_diagonals(v, small.N, float(small.q[1]), R, 1) for k, v in diags.items()}
    load_oracle_blocks(small, s2, oplan, bi, bo, pts, 1)
    out = gctx.empty_batch(bo, 0)
    gctx.nj_conv2d_block(s2, mid, out)
    want = block_conv(small.o.ctx, 1, mid_o, oplan, pts, bo)
    got = host_coeff_batch(gctx, out, bo)
    for ob in range(bo):
        assert np.array_equal(got[ob], want[ob])
    dec = decrypt_outputs(small, out, bo, W, w0)
    assert np.max(np.abs(dec - PL.conv2d_taps(img, taps, c))) <= BOUND


def test_block_conv_rejects_bad_calls(small):
    gctx = small.g.ctx
    with pytest.raises(Exception):
        gctx.nj_conv_plan_create_taps(24, 4, 4, [(4, 0, 0, 0, 1.0)])  # out channel out of range
    with pytest.raises(Exception):
        gctx.nj_conv_plan_create_taps(100, 4, 4, [(0, 0, 1, 0, 1.0)])  # W^2 > N
    plan = gctx.nj_conv_plan_create_taps(24, 4, 4, [(0, 0, 0, 0, 1.0)], fuse=False, level=1)
    x = gctx.empty_batch(1, 2)
    with pytest.raises(Exception):
        gctx.nj_conv2d_block(plan, x, gctx.empty_batch(1, 1))  # wrong level


# --------------------------------------------------------- accuracy, N = 2^16

def own_plan_accuracy(rig, img, taps, c_in, c_out, w0, want):
    gctx = rig.g.ctx
    plan = gctx.nj_conv_plan_create_taps(w0, c_in, c_out, taps, fuse=True, level=1)
    lvl, W, C, ell, bi, bo = plan.layout()
    rig.keys(plan.galois())
    _, batch = encrypt_blocks(rig, img, W, 1, False)
    out = gctx.empty_batch(bo, 0)
    gctx.nj_conv2d_block(plan, batch, out)
    got = decrypt_outputs(rig, out, bo, W, w0)[:c_out]
    err = np.max(np.abs(got - want))
    print("W %d C %d blocks %dx%d max abs error %.3e" % (W, C, bi, bo, err), flush=True)
    assert err <= BOUND
    return bi, bo


def test_full_block_conv_64_channels_56x56(full):
    """64 -> 64 channels at 56 x 56: W = 64, C = 16, 4 x 4 blocks"""
    img = RNG.uniform(-1, 1, (64, 56, 56))
    K = RNG.uniform(-1, 1, (64, 64, 3, 3))
    assert own_plan_accuracy(full, img, PL.taps_same(K), 64, 64, 56, PL.conv2d_same(img, K)) == (4, 4)


def test_full_stride2_64_to_128(full):
    """64 -> 128 stride 2, 56 x 56 -> 28 x 28: polyphase inputs 256 channels at W = 32
    (C = 64, 4 input ciphertexts), 2 output ciphertexts"""
    img = RNG.uniform(-1, 1, (64, 56, 56))
    K = RNG.uniform(-1, 1, (128, 64, 3, 3))
    taps = PL.taps_stride2(K)
    want = PL.conv2d_strided(img, K, 2)
    assert own_plan_accuracy(full, PL.polyphase(img), taps, 256, 128, 28, want) == (4, 2)


@pytest.mark.parametrize("n1", [32, 2])
def test_large_bsgs_split_parity(small, n1):
    """64 channels per ciphertext (W = 8) with 31 baby steps (n1 = 32) or 31 giant steps
    (n1 = 2): the multiply-accumulate runs in passes of 16 x 16 steps"""
    w0, c = 6, 64
    img = RNG.uniform(-1, 1, (c, w0, w0))
    K = RNG.uniform(-1, 1, (c, c, 3, 3))
    taps = PL.taps_same(K)
    N, gctx, R = small.N, small.g.ctx, small.o.ring
    plan = gctx.nj_conv_plan_create_taps(w0, c, c, taps, fuse=1, n1=n1, level=1)
    lvl, W, C, ell, bi, bo = plan.layout()
    assert (W, C, bi, bo) == (8, 64, 1, 1)
    small.keys(plan.galois())
    oplan, _, _, diags = PL.block_conv_plan(taps, c, c, W, N, True, n1=n1)
    assert max(len(oplan.babies), len(oplan.giants)) > 16
    pts = {k: PL.encode_diagonals(v, N, float(small.q[1]), R, 1) for k, v in diags.items()}
    load_oracle_blocks(small, plan, oplan, 1, 1, pts, 1)
    xs, batch = encrypt_blocks(small, img, W, 1, True)
    out = gctx.empty_batch(1, 0)
    gctx.nj_conv2d_block(plan, batch, out)
    want = block_conv(small.o.ctx, 1, xs, oplan, pts, 1)
    assert np.array_equal(host_coeff_batch(gctx, out, 1)[0], want[0])
    got = decrypt_outputs(small, out, 1, W, w0)
    assert np.max(np.abs(got - PL.conv2d_same(img, K))) <= BOUND


def test_full_stride2_256_channels_14x14(full):
    """256 -> 256 stride 2, 14 x 14 -> 7 x 7: polyphase inputs 1024 channels at W = 8
    (C = 1024, one ciphertext), 1024 diagonals with 31 baby and 31 giant steps"""
    img = RNG.uniform(-1, 1, (256, 14, 14))
    K = RNG.uniform(-1, 1, (256, 256, 3, 3)) / 48.0
    taps = PL.taps_stride2(K)
    want = PL.conv2d_strided(img, K, 2)
    assert own_plan_accuracy(full, PL.polyphase(img), taps, 1024, 256, 7, want) == (1, 1)
