"""The no-allocation key switch (nj_apply_galois_noalloc) through the C ABI (needs an
MI355X): word for word equal to nj_apply_galois on two calls in a row at N = 2^16, the
second on a smaller ciphertext (lower level), in place and out of place; equal to the
oracle's rotation; and refused with NJ_EUNSUPPORTED when a key switch needs more scratch
than its static buffer holds."""
import numpy as np
import pytest

import oracle.plans as PL

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2312_04356_amd import Ct, Ctx, NjError, chain_primes  # noqa: E402
from paper_2312_04356_amd.workload import GpuWorkload  # noqa: E402
from tests.oracle_workload import OracleWorkload  # noqa: E402


def host_coeff(gctx, ct):
    t = ct.data.clone()
    gctx.nj_to_coeff(t, ct.level, 2)
    torch.cuda.synchronize()
    return gctx.to_host(t)


def test_noalloc_key_switch_equals_allocating_one():
    print("\n[noalloc] full workload", flush=True)
    g = GpuWorkload("full", with_cts=False)
    gctx = g.ctx
    ge = PL.galois_elt(2048, g.N)
    g.make_keys([ge])
    gen = torch.Generator(device=gctx.device).manual_seed(5)
    for level in (23, 9):  # the second call on a smaller input
        print("[noalloc] level %d" % level, flush=True)
        x = gctx.empty_ct(level)
        x.data.random_(0, 2 ** 40, generator=gen)
        want, got = gctx.empty_ct(level), gctx.empty_ct(level)
        gctx.nj_apply_galois(x, ge, want)
        gctx.nj_apply_galois_noalloc(x, ge, got)
        torch.cuda.synchronize()
        assert torch.equal(got.data, want.data), "level %d" % level
        assert got.level == level
        # in place, as nj_apply_galois allows
        y = Ct(x.data.clone(), level)
        gctx.nj_apply_galois_noalloc(y, ge, y)
        torch.cuda.synchronize()
        assert torch.equal(y.data, want.data), "in place, level %d" % level


def test_noalloc_rotation_matches_oracle():
    print("\n[noalloc] oracle rotation at level 5", flush=True)
    o = OracleWorkload("full", with_cts=False)
    g = GpuWorkload("full", with_cts=False)
    gctx, lvl = g.ctx, 5
    ge = PL.galois_elt(3 * 2048, g.N)
    g.make_keys([ge])
    o.make_keys([ge])
    m = o.ring.to_rns(o.input_plaintext(), lvl)
    x_o = o.encrypt_input(lvl)
    x_g = g.encrypt_input(lvl, m_dev=gctx.to_device(m))
    out = gctx.empty_ct(lvl)
    gctx.nj_apply_galois_noalloc(x_g, ge, out)
    assert np.array_equal(host_coeff(gctx, out), o.ctx.apply_galois(lvl, x_o, ge))


def test_noalloc_refuses_oversized_key_switch():
    """N = 2^16 with 32 ciphertext primes and 16 special primes: a key switch at level 31
    needs more words than the static buffer; at level 20 it fits"""
    print("\n[noalloc] oversized ring", flush=True)
    q, p = chain_primes(16, 32, 16, 50, 48, 50)
    gctx = Ctx(16, q, p, 2.0 ** 40)
    x = gctx.empty_ct(31)
    x.data.zero_()
    with pytest.raises(NjError) as ei:
        gctx.nj_apply_galois_noalloc(x, 5, gctx.empty_ct(31))
    assert ei.value.code == -7 and "static buffer" in str(ei.value)
    x20 = gctx.empty_ct(20)
    x20.data.zero_()
    with pytest.raises(NjError) as ei:  # fits, but no key was generated
        gctx.nj_apply_galois_noalloc(x20, 5, gctx.empty_ct(20))
    assert ei.value.code == -4
