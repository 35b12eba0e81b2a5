"""Degenerate and boundary cases through the C ABI (needs an MI355X): rotations that are
the identity, invalid Galois elements, a single-channel conv on a ragged image, the
largest image a ciphertext holds, an all-zero kernel, and an empty job list."""
import numpy as np
import pytest

import oracle.plans as PL

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2312_04356_amd import NjError  # noqa: E402
from tests.test_gpu_conv_variants import Rig, decrypt_outputs, encrypt_blocks, own_plan_accuracy  # noqa: E402

RNG = np.random.default_rng(59)
NJ_EINVAL = -1


@pytest.fixture(scope="module")
def rig():
    return Rig("small", False)


def test_identity_rotations_need_no_key(rig):
    """HRot by 0 or by a multiple of N/2 slots is X -> X^1: the input, word for word,
    without a switching key (none is made here); an even or too large Galois element
    is an argument error"""
    g = rig.g
    ctx = g.ctx
    ct = g.encrypt_input(3)
    for r in (0, g.N // 2, -g.N):
        out = ctx.empty_ct(3)
        ctx.nj_rotate(ct, r, out)
        assert torch.equal(out.data, ct.data) and out.level == 3 and out.scale == ct.scale
    same = g.encrypt_input(3)
    ctx.nj_apply_galois(same, 1, same)  # in place
    assert torch.equal(same.data, ct.data)
    out = ctx.empty_ct(3)
    ctx.nj_apply_galois_noalloc(ct, 1, out)
    assert torch.equal(out.data, ct.data)
    for bad in (2, 2 * g.N + 1, 4 * g.N - 1):
        with pytest.raises(NjError) as e:
            ctx.nj_apply_galois(ct, bad, ctx.empty_ct(3))
        assert e.value.code == NJ_EINVAL


def test_single_channel_conv_on_a_ragged_image(rig):
    """1 -> 1 channel, 13 x 13 (W = 16, so 16 channel slots of which one is used)"""
    img = RNG.uniform(-1, 1, (1, 13, 13))
    K = RNG.uniform(-1, 1, (1, 1, 3, 3))
    assert own_plan_accuracy(rig, img, PL.taps_same(K), 1, 1, 13, PL.conv2d_same(img, K)) == (1, 1)


def test_largest_image_in_one_ciphertext(rig):
    """31 x 31 with a 3 x 3 kernel fills W = 32 (the 'same' conv's reach lands on the
    last padding column); 4 channels fill N = 2^12"""
    img = RNG.uniform(-1, 1, (4, 31, 31))
    K = RNG.uniform(-1, 1, (4, 4, 3, 3))
    assert own_plan_accuracy(rig, img, PL.taps_same(K), 4, 4, 31, PL.conv2d_same(img, K)) == (1, 1)


def test_all_zero_kernel_decrypts_to_zero(rig):
    gctx = rig.g.ctx
    plan = gctx.nj_conv_plan_create_taps(16, 1, 1, [(0, 0, 0, 0, 0.0)], fuse=True, level=1)
    lvl, W, C, ell, bi, bo = plan.layout()
    rig.keys(plan.galois())
    _, batch = encrypt_blocks(rig, RNG.uniform(-1, 1, (1, 16, 16)), W, 1, False)
    out = gctx.empty_batch(bo, 0)
    gctx.nj_conv2d_block(plan, batch, out)
    got = decrypt_outputs(rig, out, bo, W, 16)
    print("zero kernel: max |out| %.2e" % np.max(np.abs(got)))
    assert np.max(np.abs(got)) < 2.0 ** -20


def test_empty_job_list_is_refused(rig):
    g = rig.g
    cts = g.ctx.nj_cts_plan_create(2)
    with pytest.raises(NjError) as e:
        g.ctx.nj_batch_run(cts, [], 0)
    assert e.value.code == NJ_EINVAL
