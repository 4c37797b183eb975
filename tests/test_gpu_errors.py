"""Failure handling of the HIP path, each failure forced from the host so
that every kernel still runs to its normal end: non-finite singular values,
a QR panel barrier that gives up (its poll bound set to zero), the Jacobi
sweep cap, a truncated unswap log, and device allocations refused by the
caller's allocator hooks.  A failed absorption must leave the MPO unchanged."""
import ctypes
import os

import numpy as np
import pytest

from oracle import mpo_oracle as mo
from paper_2604_21908_amd import circuitgen as cg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    from paper_2604_21908_amd import mpo as mpolib
    mpolib.load_library()
    return mpolib


def random_state(n, seed, layers, chi_max=64):
    rng = np.random.default_rng(seed)
    m = mo.OracleMPO(n)
    for l in range(layers):
        for i in range(l % 2, n - 1, 2):
            mo.commit(m, mo.bond_update(m, i, cg.haar_su4(rng), cg.haar_su4(rng), chi_max, 1e-13, "rel_sv"))
    return m


def snapshot(g):
    return g.bond_dims(), [g.read_site(i) for i in range(g.n)], [g.singular_values(b) for b in range(g.n - 1)]


def assert_same(a, b):
    assert a[0] == b[0]
    for x, y in zip(a[1], b[1]):
        assert np.array_equal(x, y)
    for x, y in zip(a[2], b[2]):
        assert np.array_equal(x, y)


def test_non_finite_singular_values_raise_and_leave_state(lib):
    """A site scaled to 1e200 (finite) makes theta's Gram entries overflow to
    inf in FP64; the truncation kernel flags the non-finite values before it
    sorts them, and the call fails with MPO_ENUMERIC."""
    n = 6
    m = random_state(n, 3, 4, chi_max=16)
    sites = [b.copy() for b in m.B]
    sites[2] = sites[2] * 1e200
    g = lib.MPO(n, 16, 1e-12, 0, 0, max_sweeps=4)
    g.load_state(sites, m.lam)
    before = snapshot(g)
    with pytest.raises(lib.MpoError) as e:
        g.absorb(2, cg.haar_su4(np.random.default_rng(1)), None)
    assert e.value.status == -4
    assert_same(before, snapshot(g))
    g.close()


def test_qr_barrier_give_up_is_an_error(lib, monkeypatch):
    """theta 512 x 512: every QR panel spans two or more workgroups.  With the
    barrier's poll bound at zero every workgroup gives up at its first barrier
    (no wave waits), the panel sets the problem's status word, and the call
    fails with MPO_EHIP before anything of the MPO is written."""
    n = 10
    m = random_state(n, 5, 9, chi_max=128)
    b = 4
    assert m.chi(b - 1) == 128 and m.chi(b + 1) == 128
    monkeypatch.setenv("MPO_QR_SPIN", "0")
    g = lib.MPO(n, 128, 1e-8, 1, 1)
    monkeypatch.delenv("MPO_QR_SPIN")
    g.load_state(m.B, m.lam)
    before = snapshot(g)
    rng = np.random.default_rng(12)
    with pytest.raises(lib.MpoError) as e:
        g.absorb(b, cg.haar_su4(rng), cg.haar_su4(rng))
    assert e.value.status == -3
    assert "barrier" in str(e.value)
    assert_same(before, snapshot(g))
    g.close()
    # a handle with the normal bound does the same update
    h = lib.MPO(n, 128, 1e-8, 1, 1)
    h.load_state(m.B, m.lam)
    rng = np.random.default_rng(12)
    info = h.absorb(b, cg.haar_su4(rng), cg.haar_su4(rng))
    assert info["k"] >= 1
    h.close()


def test_sweep_cap_warns_and_writes(lib):
    """max_sweeps = 1: the Jacobi SVD stops at its cap, the result is still
    written and the call returns MPO_WARN_NOCONV (noconv in the binding)."""
    n = 8
    m = random_state(n, 9, 6, chi_max=64)
    g = lib.MPO(n, 64, 1e-12, 0, 0, max_sweeps=1)
    g.load_state(m.B, m.lam)
    rng = np.random.default_rng(3)
    info = g.absorb(3, cg.haar_su4(rng), cg.haar_su4(rng))
    assert info["noconv"] and info["sweeps"] == 1
    assert g.bond_dims()[3] == info["k"]
    g.close()


def _swap_layer_state(n):
    m = mo.OracleMPO(n)
    for b in range(0, n - 1, 2):
        mo.commit(m, mo.bond_update(m, b, mo.SWAP4, None, 64, 1e-12, "rel_sv"))
    return m


def test_unswap_log_overflow(lib):
    """log_cap = 0: the sweep completes, n_accepted counts every swap and the
    status is MPO_EOVERFLOW; the MPO equals that of a sweep with a full log."""
    n = 7
    m = _swap_layer_state(n)
    a = lib.MPO(n, 64, 1e-12, 0, 0)
    b = lib.MPO(n, 64, 1e-12, 0, 0)
    a.load_state(m.B, m.lam)
    b.load_state(m.B, m.lam)
    opts = lib.UnswapOpts(1, 0, 20)
    nacc = ctypes.c_int32(-1)
    s = a.lib.mpo_unswap_sweep(a.h, ctypes.byref(opts), None, 0, ctypes.byref(nacc))
    assert s == -5
    log = b.unswap("parallel")
    assert nacc.value == len(log) > 0
    assert a.bond_dims() == b.bond_dims() == [1] * (n - 1)
    a.close()
    b.close()


def test_allocator_hooks_serve_every_device_buffer(lib):
    """Every device buffer of a handle comes through the alloc hook (PyTorch's
    caching allocator here) and goes back through the free hook."""
    import torch
    n = 8
    m = random_state(n, 11, 5, chi_max=64)
    al = lib.TorchAllocator()
    g = lib.MPO(n, 64, 1e-10, 1, 1, allocator=al)
    g.load_state(m.B, m.lam)
    rng = np.random.default_rng(4)
    for b in (1, 3, 5, 3):
        g.absorb(b, cg.haar_su4(rng), cg.haar_su4(rng))
    g.unswap("parallel")
    g.extract_peak()
    c = g.counters()
    assert c["hook_allocs"] == al.calls > 0
    assert al.bytes_live > 0
    g.close()
    assert al.bytes_live == 0 and not al.live
    torch.cuda.synchronize()


def test_allocation_refused_leaves_state_unchanged(lib):
    """The hook refuses every allocation beyond what init took: the first
    update that needs workspace fails with MPO_ENOMEM and the MPO is
    unchanged; with the limit lifted the same update succeeds."""
    n = 8
    m = random_state(n, 12, 5, chi_max=64)
    al = lib.TorchAllocator()
    g = lib.MPO(n, 64, 1e-10, 1, 1, allocator=al)
    g.load_state(m.B, m.lam)
    before = snapshot(g)            # (reading FP32 sites takes a temporary)
    al.limit = al.bytes_live
    rng = np.random.default_rng(5)
    go, gi = cg.haar_su4(rng), cg.haar_su4(rng)
    with pytest.raises(lib.MpoError) as e:
        g.absorb(3, go, gi)
    assert e.value.status == -2
    al.limit = None
    assert_same(before, snapshot(g))
    info = g.absorb(3, go, gi)
    r = mo.bond_update(m, 3, go, gi, 64, 1e-10, "weight")
    assert info["k"] == r.k
    g.close()
