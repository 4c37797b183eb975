"""The allocation-free absorption (mpo_absorb_gate_pair_noalloc) against the
ordinary one (mpo_absorb_gate_pair), through the C ABI: the same kept rank,
singular values within the precision's normwise tolerance (1e-10 FP64,
1e-4 FP32 and mixed) and the same contracted two-site operator, on two calls
in a row (the second on a smaller theta, so that the first call's contents
of the shared scratch array must not leak into it), with no call of the
device-allocation hook.  An update too large for the static scratch array
is refused and leaves the MPO unchanged."""
import numpy as np
import pytest

from oracle import mpo_oracle as mo
from paper_2604_21908_amd import circuitgen as cg

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-4, "mixed": 1e-4}
PREC = {"fp64": 0, "fp32": 1, "mixed": 2}


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


def two_site(g, bond):
    a, b = g.read_site(bond), g.read_site(bond + 1)
    return np.einsum("asc,ctb->astb", a, b)


def sv_err(a, b):
    k = min(len(a), len(b))
    return np.max(np.abs(np.asarray(a[:k]) - np.asarray(b[:k]))) / np.linalg.norm(b)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "mixed"])
def test_noalloc_equals_allocating_absorb(lib, prec):
    n = 8
    m = random_state(n, 21, 6)
    al_a, al_b = lib.TorchAllocator(), lib.TorchAllocator()
    a = lib.MPO(n, 64, 1e-10, 1, PREC[prec], allocator=al_a)
    b = lib.MPO(n, 64, 1e-10, 1, PREC[prec], allocator=al_b)
    a.load_state(m.B, m.lam)
    b.load_state(m.B, m.lam)
    dims = a.bond_dims()
    assert dims[3] == 64 and dims[2] == 64 and dims[4] == 64
    rng = np.random.default_rng(8)
    # first call: theta 256 x 256 at the middle bond; second: theta 16 x 256
    # at bond 1 (chi_0 = 4), a smaller shape on the same scratch array
    for bond in (3, 1):
        go, gi = cg.haar_su4(rng), cg.haar_su4(rng)
        calls = al_b.calls
        ra = a.absorb(bond, go, gi)
        rb = b.absorb_noalloc(bond, go, gi)
        assert al_b.calls == calls, "the allocation-free call used the allocation hook"
        assert rb["k"] == ra["k"]
        assert a.bond_dims() == b.bond_dims()
        sa, sb = a.singular_values(bond), b.singular_values(bond)
        assert sv_err(sb, sa) <= TOL[prec]
        ta, tb = two_site(a, bond), two_site(b, bond)
        assert np.linalg.norm(tb - ta) <= 10 * TOL[prec] * np.linalg.norm(ta)
        # and both agree with the oracle's update of the same state
        r = mo.bond_update(m, bond, go, gi, 64, 1e-10, "weight")
        assert r.k == rb["k"]
        assert sv_err(sb, r.s[:r.k]) <= TOL[prec]
        mo.commit(m, r)
    a.close()
    b.close()


def test_noalloc_refuses_what_does_not_fit(lib):
    """theta 1024 x 1024 in FP64 needs far more than 64 MiB of workspace: the
    call fails with MPO_EINVAL before any kernel runs and the MPO is
    unchanged; the ordinary call on the same state still works."""
    n = 10
    rng = np.random.default_rng(3)
    dims = [4, 16, 64, 256, 256, 256, 64, 16, 4]
    sites, lams = [], []
    for i in range(n):
        cl = 1 if i == 0 else dims[i - 1]
        cr = 1 if i == n - 1 else dims[i]
        x = rng.standard_normal((cl, 4 * cr)) + 1j * rng.standard_normal((cl, 4 * cr))
        q, _ = np.linalg.qr(x.conj().T)          # right-canonical rows
        sites.append(q.conj().T.reshape(cl, 4, cr))
    for d in dims:
        lam = np.sort(rng.random(d))[::-1]
        lams.append(lam / np.linalg.norm(lam))
    g = lib.MPO(n, 256, 1e-10, 1, 0)
    g.load_state(sites, lams)
    before = (g.bond_dims(), [g.read_site(i) for i in (3, 4, 5)], g.singular_values(4))
    go, gi = cg.haar_su4(rng), cg.haar_su4(rng)
    with pytest.raises(lib.MpoError) as e:
        g.absorb_noalloc(4, go, gi)
    assert e.value.status == -1
    after = (g.bond_dims(), [g.read_site(i) for i in (3, 4, 5)], g.singular_values(4))
    assert before[0] == after[0]
    for x, y in zip(before[1], after[1]):
        assert np.array_equal(x, y)
    assert np.array_equal(before[2], after[2])
    g.close()
