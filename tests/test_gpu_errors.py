"""Error statuses through the C ABI (needs an MI355X): each call refuses what it cannot
compute with the documented status code and leaves its output untouched; a refused
call does not disturb the next valid one."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2312_04356_amd import Ct, NjError  # noqa: E402
from paper_2312_04356_amd.workload import GpuWorkload  # noqa: E402

NJ_EINVAL, NJ_ELEVEL, NJ_ESCALE, NJ_ENOKEY = -1, -2, -3, -4


@pytest.fixture(scope="module")
def g():
    return GpuWorkload("small", with_cts=False)


def status(fn):
    with pytest.raises(NjError) as e:
        fn()
    return e.value.code


def test_missing_rotation_key_is_enokey(g):
    ctx = g.ctx
    ct = g.encrypt_input(3)
    out = ctx.empty_ct(3)
    before = out.data.clone()
    assert status(lambda: ctx.nj_rotate(ct, 5, out)) == NJ_ENOKEY
    assert torch.equal(out.data, before)  # nothing written
    g.make_keys([ctx.nj_galois_elt(5)])
    ctx.nj_rotate(ct, 5, out)  # with its key the same call succeeds
    assert out.level == 3


def test_sums_refuse_mismatched_levels_and_scales(g):
    ctx = g.ctx
    a, b = g.encrypt_input(3), g.encrypt_input(3)
    out = ctx.empty_ct(3)
    c2 = g.encrypt_input(2)
    assert status(lambda: ctx.nj_add(a, c2, out)) == NJ_ELEVEL
    b_off = Ct(b.data, b.level, scale=b.scale * 2.0)
    assert status(lambda: ctx.nj_add(a, b_off, out)) == NJ_ESCALE
    assert status(lambda: ctx.nj_sub(a, b_off, out)) == NJ_ESCALE
    assert status(lambda: ctx.nj_combine(a, b_off, ctx.empty_ct(3))) == NJ_ESCALE
    b_near = Ct(b.data, b.level, scale=b.scale * (1 + 1e-12))  # rounding-level difference is a sum
    ctx.nj_add(a, b_near, out)
    ctx.nj_add(a, b, out)
    assert out.level == 3 and out.scale == a.scale


def test_rescale_and_level_errors(g):
    ctx = g.ctx
    c0 = g.encrypt_input(0)
    assert status(lambda: ctx.nj_rescale(c0, ctx.empty_ct(0))) == NJ_ELEVEL
    c3 = g.encrypt_input(3)
    assert status(lambda: ctx.nj_rescale(c3, c3)) == NJ_EINVAL  # output aliasing input
    assert status(lambda: ctx.nj_drop_level(c3, 5, ctx.empty_ct(5))) == NJ_ELEVEL
    y = ctx.empty_ct(2)
    ctx.nj_rescale(c3, y)
    assert y.level == 2


def test_plan_level_and_key_errors(g):
    ctx = g.ctx
    plan = g.conv_plan  # encoded for level 1
    ct = g.encrypt_input(2)
    out = ctx.empty_ct(1)
    code = status(lambda: ctx.nj_conv2d_cins(plan, ct, out))
    assert code == NJ_ELEVEL
    ct1 = g.encrypt_input(1)
    fresh = GpuWorkload("small", with_cts=False)  # a context without the conv's keys
    fplan = fresh.ctx.nj_conv_plan_create(fresh.w["w0"], fresh.w["f"], fresh.K)
    assert status(lambda: fresh.ctx.nj_conv2d_cins(fplan, fresh.encrypt_input(1), fresh.ctx.empty_ct(0))) == NJ_ENOKEY
    g.make_keys(plan.galois())
    ctx.nj_conv2d_cins(plan, ct1, ctx.empty_ct(0))
    assert np.isfinite(ct1.scale)


def test_keys_saved_and_restored(g, tmp_path):
    """switching keys written to a file and read into a fresh context of the same
    parameters and secret rotate word for word as the originals; another secret is refused"""
    ctx = g.ctx
    gs = [ctx.nj_galois_elt(r) for r in (1, 3)]
    g.make_keys(gs)
    path = str(tmp_path / "keys.npz")
    saved = ctx.save_keys(path, gs)
    assert saved == gs and ctx.nj_key_words() == ctx.dnum * 2 * (ctx.L + 1 + ctx.alpha) * ctx.N
    assert status(lambda: ctx.nj_key_export(ctx.nj_galois_elt(7))) == NJ_ENOKEY
    fresh = GpuWorkload("small", with_cts=False)
    assert fresh.ctx.load_keys(path) == sorted(gs)
    assert sorted(fresh.ctx.nj_key_list()) == sorted(gs)
    ct = g.encrypt_input(4)
    ct2 = fresh.encrypt_input(4)
    assert torch.equal(ct.data, ct2.data)
    for r in (1, 3):
        a, b = ctx.empty_ct(4), fresh.ctx.empty_ct(4)
        ctx.nj_rotate(ct, r, a)
        fresh.ctx.nj_rotate(ct2, r, b)
        assert torch.equal(a.data, b.data)
    other = GpuWorkload("small", with_cts=False)
    other.ctx.nj_set_secret(-np.asarray(other.ctx.secret))
    with pytest.raises(ValueError):
        other.ctx.load_keys(path)


def test_decryption_bound_check_flags_wrap_around(g):
    """constant messages m at level 0 (coefficient 0 = m scale): a bound below
    q_0 / (2 scale) with m inside it passes; m beyond its bound is flagged; a bound
    reaching q_0 / (2 scale) is flagged even where m decrypts, since a message that
    large wraps around (0.75 P comes back as -0.25 P)"""
    import synth
    ctx = g.ctx
    P = g.q[0] / g.scale  # 2^10
    cases = ((0.25 * P, 0.3 * P, True), (0.4 * P, 0.3 * P, False), (0.75 * P, 0.8 * P, False))
    for k, (m, bound, ok) in enumerate(cases):
        coeffs = ctx.nj_encode_slots(np.full(g.N // 2, m), g.scale)
        dev = torch.empty((1, g.N), dtype=torch.int64, device=ctx.device)
        ctx.nj_upload_plain(coeffs, 0, dev)
        a, e = synth.enc_randomness(g.q[:1], g.N, 91, k)
        ct = ctx.nj_encrypt_sk(dev, 0, a, e, g.scale, ctx.empty_ct(0))
        vals, valid = ctx.decrypt_checked(ct, bound)
        assert valid == ok, (m, bound, vals[0])
        want = m if m < P / 2 else m - P
        assert abs(vals[0] - want) < 1e-6 and np.max(np.abs(vals[1:])) < 1e-6


def test_plan_from_spec_rebuilds_the_plan(g):
    ctx = g.ctx
    spec = {"groups": 2, "n1": [4, 8], "hoist": [False, True], "lazy": True}
    p = ctx.cts_plan_from_spec(spec)
    q = ctx.nj_cts_plan_create_split(2, [4, 8]).set_hoist([False, True]).set_lazy(True)
    for t in range(2):
        assert np.array_equal(p.features(ctx.L - t, t), q.features(ctx.L - t, t))
        assert sorted(p.offsets(t)) == sorted(q.offsets(t))
    assert list(p.features(ctx.L, 0))[4] == 0  # group 0 not hoisted
