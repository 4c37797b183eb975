"""GPU parity of the HIP path (through the C ABI) against the CPU oracle.

Tolerances: singular values are compared normwise over the kept range,
max_j |s_j - s_j^ref| / |s^ref|_2 <= 1e-10 for FP64 and 1e-4 for FP32 and
mixed; kept ranks, peak bits and accepted-swap logs must be identical; the
peak probability must agree to 1e-3 relative (FP64 paths agree far tighter).
SVD factors are gauge-dependent, so tensors are compared through contracted
operators, never factor by factor."""
import numpy as np
import pytest

from oracle import brute as bf
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


def random_state(n, seed, layers, chi_max=256):
    rng = np.random.default_rng(seed)
    m = mo.OracleMPO(n)
    for l in range(layers):
        for i in range(l % 2, n - 1, 2):
            mo.commit(m, mo.bond_update(m, i, cg.haar_su4(rng), cg.haar_su4(rng), chi_max, 1e-13, "rel_sv"))
    return m


def sv_err(a, b):
    k = min(len(a), len(b))
    return np.max(np.abs(np.asarray(a[:k]) - np.asarray(b[:k]))) / np.linalg.norm(b)


def gpu_mpo(lib, m, prec, chi_max=256, cutoff=1e-12, mode=0):
    g = lib.MPO(m.n, chi_max, cutoff, mode, PREC[prec])
    g.load_state(m.B, m.lam)
    return g


def gpu_dense(g, n):
    o = mo.OracleMPO(n)
    o.B = [g.read_site(i) for i in range(n)]
    return o.dense_operator()


# ---------------------------------------------------------------- single updates
@pytest.mark.parametrize("prec", ["fp64", "fp32", "mixed"])
@pytest.mark.parametrize("bond", [0, 2, 4])
def test_single_update_matches_oracle(lib, prec, bond):
    n = 6
    m = random_state(n, 7 + bond, 4)
    rng = np.random.default_rng(bond)
    go, gi = cg.haar_su4(rng), cg.haar_su4(rng)
    g = gpu_mpo(lib, m, prec)
    info = g.absorb(bond, go, gi)
    r = mo.bond_update(m, bond, go, gi, 256, 1e-12, "rel_sv")
    mo.commit(m, r)
    assert info["k"] == r.k
    assert sv_err(g.singular_values(bond), r.s[:r.k]) <= TOL[prec]
    assert np.max(np.abs(gpu_dense(g, n) - m.dense_operator())) <= TOL[prec] * 10
    assert g.bond_dims() == m.bond_dims()
    g.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "mixed"])
def test_large_theta_update(lib, prec):
    """A 256 x 256 theta (chi 64 on both sides) spans many 16-column blocks."""
    n = 8
    m = random_state(n, 3, 7, chi_max=64)
    assert m.chi(2) == 64 and m.chi(4) == 64
    rng = np.random.default_rng(9)
    go, gi = cg.haar_su4(rng), cg.haar_su4(rng)
    g = gpu_mpo(lib, m, prec, chi_max=64, cutoff=1e-8, mode=1)
    info = g.absorb(3, go, gi)
    r = mo.bond_update(m, 3, go, gi, 64, 1e-8, "weight")
    assert info["k"] == r.k == 64
    assert sv_err(g.singular_values(3), r.s[:r.k]) <= TOL[prec]
    assert abs(info["discarded"] - r.discarded) <= TOL[prec] * r.total
    g.close()


@pytest.mark.parametrize("abc", [(0.3, 0.2, 0.1), (np.pi / 4, np.pi / 4, np.pi / 4), (np.pi / 4, 0, 0)])
def test_kak_closed_form_on_gpu(lib, abc):
    rng = np.random.default_rng(5)
    u = np.kron(cg.haar_unitary(rng, 2), cg.haar_unitary(rng, 2)) @ bf.kak_gate(*abc)
    g = lib.MPO(4, 16, 1e-12, 0, 0)
    info = g.absorb(1, u, None)
    want = bf.kak_schmidt_values(*abc)
    k = int(np.count_nonzero(want > 1e-12 * want[0]))
    assert info["k"] == k
    assert np.allclose(g.singular_values(1), want[:k], atol=1e-12)
    g.close()


def test_mirrored_pair_collapses(lib):
    rng = np.random.default_rng(1)
    u = cg.haar_su4(rng)
    g = lib.MPO(5, 16, 1e-12, 0, 0)
    info = g.absorb(2, u.conj().T, u)
    assert info["k"] == 1 and abs(g.singular_values(2)[0] - 1) < 1e-13
    g.close()


def test_batch_equals_one_by_one(lib):
    n = 9
    m = random_state(n, 21, 4)
    rng = np.random.default_rng(2)
    bonds = [0, 3, 5, 7]
    gs = [(cg.haar_su4(rng), cg.haar_su4(rng)) for _ in bonds]
    a = gpu_mpo(lib, m, "fp64")
    b = gpu_mpo(lib, m, "fp64")
    a.absorb_batch(bonds, [x[0] for x in gs], [x[1] for x in gs])
    for bd, (go, gi) in zip(bonds, gs):
        b.absorb(bd, go, gi)
    for i in range(n):
        assert np.array_equal(a.read_site(i), b.read_site(i))
    a.close()
    b.close()


@pytest.mark.parametrize("prec", ["fp32", "mixed"])
def test_group_of_mixed_widths_equals_lone_updates(lib, prec):
    """A grouped launch holding a wide update (theta 1024 x 1024, whose Jacobi
    operand is put in order of decreasing column norms before its first
    sweeps) and a narrow one (never ordered) gives each MPO the bits of its
    lone update: per-problem choices must not depend on the rest of the batch."""
    import bench
    nb, sites, lams, bb = bench.micro_state(256, seed=3)
    small = random_state(9, 21, 4)
    rng = np.random.default_rng(31)
    gates = [(cg.haar_su4(rng), cg.haar_su4(rng)) for _ in range(2)]
    bs = 3

    def fresh():
        big = lib.MPO(nb, 256, 1e-8, 1, PREC[prec])
        big.load_state(sites, lams)
        return big, gpu_mpo(lib, small, prec, chi_max=256, cutoff=1e-8, mode=1)

    lone_big, lone_small = fresh()
    ib = lone_big.absorb(bb, *gates[0])
    i_s = lone_small.absorb(bs, *gates[1])
    assert ib["k"] == 256
    grp = lib.Group(PREC[prec])
    g_big, g_small = fresh()
    infos = grp.absorb([g_big, g_small], [bb, bs], [gates[0][0], gates[1][0]], [gates[0][1], gates[1][1]])
    assert [x["k"] for x in infos] == [ib["k"], i_s["k"]]
    for a, b, n in ((lone_big, g_big, nb), (lone_small, g_small, small.n)):
        for i in range(n):
            assert np.array_equal(a.read_site(i), b.read_site(i))
        for i in range(n - 1):
            assert np.array_equal(a.singular_values(i), b.singular_values(i))
    for x in (lone_big, lone_small, g_big, g_small):
        x.close()
    grp.close()


def test_error_codes_leave_state_unchanged(lib):
    m = random_state(5, 4, 3)
    g = gpu_mpo(lib, m, "fp64")
    before = [g.read_site(i) for i in range(5)]
    with pytest.raises(lib.MpoError) as e:
        g.absorb(4, None, None)
    assert e.value.status == -1
    bad = np.eye(4, dtype=complex)
    bad[0, 0] = np.nan
    with pytest.raises(lib.MpoError) as e:
        g.absorb(1, bad, None)
    assert e.value.status == -4
    with pytest.raises(lib.MpoError):
        g.absorb_batch([1, 2], [None, None], [None, None])      # adjacent bonds
    for i in range(5):
        assert np.array_equal(g.read_site(i), before[i])
    g.close()


def test_two_sites_and_identity_gates(lib):
    g = lib.MPO(2, 4, 1e-12, 0, 0)
    info = g.absorb(0, None, None)
    assert info["k"] == 1
    bits, p, n2 = g.extract_peak()
    assert list(bits) == [0, 0] and abs(p - 1) < 1e-12 and abs(n2 - 0.25) < 1e-14
    g.close()


# ---------------------------------------------------------------- whole contractions
def run_both(circ, prec, chi_max, cutoff, mode, tau, unswap, relaxed=False):
    from paper_2604_21908_amd import driver as dr
    ocfg = mo.OracleConfig(chi_max=chi_max, cutoff=cutoff, mode=mode, tau=tau, unswap=unswap, relaxed=relaxed)
    ref = mo.contract(circ.n, circ.gates, ocfg)
    cfg = dr.RunConfig(chi_max=chi_max, cutoff=cutoff, cutoff_mode=mode, precision=prec, tau=tau,
                       unswap=unswap, relaxed=relaxed)
    c = dr.Contractor(circ, cfg)
    res = c.run()
    lams = [c.m.singular_values(b) for b in range(circ.n - 1)]
    c.close()
    return ref, res, lams


def compare_runs(ref, res, lams, prec):
    rk = [t for t in ref.trace if "k" in t]
    gk = [t for t in res.trace if "k" in t]
    assert [t["k"] for t in gk] == [t["k"] for t in rk]
    assert [t["bond"] for t in gk] == [t["bond"] for t in rk]
    ru = [t["log"] for t in ref.trace if t["stage"] == "unswap"]
    gu = [t["log"] for t in res.trace if t["stage"] == "unswap"]
    assert ru == gu
    for b in range(len(lams)):
        assert sv_err(lams[b], ref.mpo.lam[b]) <= TOL[prec]
    assert np.array_equal(res.bits, ref.bits)
    assert abs(res.prob - ref.prob) <= 1e-3 * ref.prob


@pytest.mark.parametrize("prec", ["fp64", "fp32", "mixed"])
def test_config0_contraction_matches_oracle(lib, prec):
    circ = cg.config_circuit(0)
    ref, res, lams = run_both(circ, prec, 64, 1e-12 if prec == "fp64" else 1e-8,
                              "rel_sv" if prec == "fp64" else "weight", 2000, "parallel")
    compare_runs(ref, res, lams, prec)
    assert (res.bits == circ.peak).all()
    assert abs(res.prob - bf.peak_probability_closed_form(circ.n, circ.k_gates)) < 1e-3 * res.prob


def test_sequential_unswap_matches_oracle(lib):
    circ = cg.mirrored_peaked_circuit(8, 3, 31, reading="B")
    ref, res, lams = run_both(circ, "fp64", 256, 1e-12, "rel_sv", 300, "sequential")
    compare_runs(ref, res, lams, "fp64")


def test_relaxed_parallel_unswap_matches_oracle(lib):
    circ = cg.mirrored_peaked_circuit(8, 3, 32, reading="B")
    ref, res, lams = run_both(circ, "fp64", 256, 1e-12, "rel_sv", 300, "parallel", relaxed=True)
    compare_runs(ref, res, lams, "fp64")


def test_mirror_collapse_on_gpu(lib):
    from paper_2604_21908_amd import driver as dr
    circ = cg.mirror_only_circuit(12, 6, 3)
    res = dr.contract(circ, dr.RunConfig(chi_max=64, unswap="none"))
    ks = [t["k"] for t in res.trace if "k" in t]
    assert ks and max(ks) == 1
    assert abs(res.prob - 1.0) < 1e-10 and not res.bits.any()


# ---------------------------------------------------------------- edge cases
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_chi_cap_of_one(lib, prec):
    """chi_max = 1 binds on every update: k = 1 and the leading value agrees."""
    n = 5
    rng = np.random.default_rng(4)
    g = lib.MPO(n, 1, 1e-12, 0, PREC[prec])
    o = mo.OracleMPO(n)
    for b in (0, 2, 3, 1):
        go, gi = cg.haar_su4(rng), cg.haar_su4(rng)
        info = g.absorb(b, go, gi)
        r = mo.bond_update(o, b, go, gi, 1, 1e-12, "rel_sv")
        mo.commit(o, r)
        assert info["k"] == r.k == 1
        assert abs(g.singular_values(b)[0] - r.s[0]) <= TOL[prec] * np.linalg.norm(r.s)
        assert abs(info["discarded"] - r.discarded) <= TOL[prec] * r.total
    assert g.bond_dims() == [1] * (n - 1)
    g.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "mixed"])
def test_odd_chain_end_bonds(lib, prec):
    """Odd n; updates on both end bonds (chi_l = 1 or chi_r = 1) and a
    one-sided gate."""
    n = 7
    m = random_state(n, 31, 5)
    rng = np.random.default_rng(6)
    g = gpu_mpo(lib, m, prec)
    for b, one_sided in ((0, False), (n - 2, False), (3, True)):
        go, gi = cg.haar_su4(rng), (None if one_sided else cg.haar_su4(rng))
        info = g.absorb(b, go, gi)
        r = mo.bond_update(m, b, go, gi, 256, 1e-12, "rel_sv")
        mo.commit(m, r)
        assert info["k"] == r.k
        assert sv_err(g.singular_values(b), r.s[:r.k]) <= TOL[prec]
    assert np.max(np.abs(gpu_dense(g, n) - m.dense_operator())) <= TOL[prec] * 10
    g.close()


@pytest.mark.parametrize("schedule", ["sequential", "parallel"])
def test_gpu_unswap_removes_bare_swap_layer(lib, schedule):
    """A layer of output SWAPs on even bonds and input SWAPs on odd bonds is
    undone exactly by the greedy trials, back to bond dimension 1."""
    n = 7
    g = lib.MPO(n, 64, 1e-12, 0, 0)
    o = mo.OracleMPO(n)
    for b in range(0, n - 1, 2):
        g.absorb(b, mo.SWAP4, None)
        mo.commit(o, mo.bond_update(o, b, mo.SWAP4, None, 64, 1e-12, "rel_sv"))
    for b in range(1, n - 1, 2):
        g.absorb(b, None, mo.SWAP4)
        mo.commit(o, mo.bond_update(o, b, None, mo.SWAP4, 64, 1e-12, "rel_sv"))
    assert g.bond_dims() == o.bond_dims() == [4] * (n - 1)
    log = g.unswap(schedule)
    run = mo.unswap_parallel if schedule == "parallel" else mo.unswap_sequential
    ref = run(o, mo.OracleConfig(chi_max=64, cutoff=1e-12, mode="rel_sv", unswap=schedule))
    assert g.bond_dims() == o.bond_dims() == [1] * (n - 1)
    assert sorted(log) == sorted(ref)
    g.close()


def test_peak_readout_of_generic_state(lib):
    n = 7
    m = random_state(n, 44, 5)
    g = gpu_mpo(lib, m, "fp64")
    bits, p, n2 = g.extract_peak()
    rb, rp, rn2 = mo.extract_peak(m)
    assert np.array_equal(bits, rb)
    assert abs(p - rp) <= 1e-10 * rp and abs(n2 - rn2) <= 1e-12 * rn2
    g.close()


@pytest.mark.parametrize("prec", ["fp32", "mixed"])
def test_chi128_update(lib, prec):
    """theta 512 x 512: 32 column blocks, 16 pairs per round-robin step."""
    n = 10
    m = random_state(n, 5, 9, chi_max=128)
    b = 4
    assert m.chi(b - 1) == 128 and m.chi(b + 1) == 128
    rng = np.random.default_rng(12)
    go, gi = cg.haar_su4(rng), cg.haar_su4(rng)
    g = gpu_mpo(lib, m, prec, chi_max=128, cutoff=1e-8, mode=1)
    info = g.absorb(b, go, gi)
    r = mo.bond_update(m, b, go, gi, 128, 1e-8, "weight")
    assert info["k"] == r.k
    assert sv_err(g.singular_values(b), r.s[:r.k]) <= TOL[prec]
    right = g.read_site(b + 1).reshape(info["k"], -1)            # V_k^dag: orthonormal rows
    assert np.max(np.abs(right @ right.conj().T - np.eye(info["k"]))) <= 1e-4
    assert abs(info["total"] - r.total) <= 1e-4 * r.total
    g.close()


_FULL = {}


def _full_size_oracle():
    """The chi = 1024 update (theta 4096 x 4096) in the oracle, once: its
    singular values, discarded weight, the untruncated theta (with the left
    bond values) and the truncated operator U_k S_k V_k^dag."""
    if not _FULL:
        import bench
        n, sites, lams, bond = bench.micro_state(1024)
        rng = np.random.default_rng(77)
        go, gi = bench.haar_su4(rng), bench.haar_su4(rng)
        m = mo.OracleMPO(n)
        m.B = [s.copy() for s in sites]
        m.lam = [l.copy() for l in lams]
        r = mo.bond_update(m, bond, go, gi, 1024, 1e-8, "weight", vectors=True)
        chil, chir = sites[bond].shape[0], sites[bond + 1].shape[2]
        th = mo.apply_gates_to_theta(np.tensordot(sites[bond], sites[bond + 1], axes=([2], [0])), go, gi)
        theta = (th * lams[bond - 1][:, None, None, None]).reshape(4 * chil, 4 * chir)
        _FULL.update(n=n, sites=sites, lams=lams, bond=bond, go=go, gi=gi, r=r, theta=theta)
    return _FULL


@pytest.mark.parametrize("prec,route", [("mixed", "qr2"), ("fp32", "qr2"), ("fp64", "accumulate"),
                                        ("mixed", "accumulate"), ("fp32", "accumulate")])
def test_full_size_chi1024_update(lib, prec, route, monkeypatch):
    """The benchmarked update itself (theta 4096 x 4096, chi_max = 1024 binds),
    on both SVD routes of the FP32 and mixed forms (second QR with vectors from
    the converged columns, the default; or accumulated rotations, as FP64),
    against the oracle: kept rank, singular values (normwise), discarded weight,
    orthonormal rows of the new right tensor, and the written two-site operator.
    With the left bond values applied, lambda B_i' B_i+1' is a rank-k
    approximation of theta; it must be a best one (Eckart-Young): its squared
    distance to the oracle's theta equals the oracle's discarded weight up to the
    tolerance times the total weight, and it lies within 2 sqrt(w) + tol of the
    oracle's U_k S_k V_k^dag.  A wrong row chunk of V_k, a wrong left tensor or a
    lost conjugate would show an O(1) excess."""
    f = _full_size_oracle()
    r = f["r"]
    tol = TOL[prec]
    monkeypatch.setenv("MPO_SVD", route)
    g = lib.MPO(f["n"], 1024, 1e-8, 1, PREC[prec])
    g.load_state(f["sites"], f["lams"])
    info = g.absorb(f["bond"], f["go"], f["gi"])
    b = f["bond"]
    s_gpu = g.singular_values(b)
    left = g.read_site(b)
    right = g.read_site(b + 1)
    g.close()
    k = info["k"]
    assert k == r.k == 1024
    assert sv_err(s_gpu, r.s[:r.k]) <= tol
    assert abs(info["discarded"] - r.discarded) <= max(tol, 1e-12) * r.total
    rr = right.reshape(k, -1)
    assert np.max(np.abs(rr @ rr.conj().T - np.eye(k))) <= (1e-4 if prec != "fp64" else 1e-10)
    lam = f["lams"][b - 1]
    op = (left * lam[:, None, None]).reshape(-1, k) @ rr
    theta = f["theta"]
    w_eff = np.linalg.norm(theta - op) ** 2
    assert w_eff >= r.discarded * (1 - 1e-9)
    assert w_eff - r.discarded <= max(tol, 1e-12) * r.total
    ref_op = (r.new_left * lam[:, None, None]).reshape(-1, k) @ r.new_right.reshape(k, -1)
    assert np.linalg.norm(op - ref_op) <= 2 * np.sqrt(r.discarded) + tol * np.sqrt(r.total)


def test_fp64_update_on_tall_panels(lib):
    """chi = 384 on both sides (theta 1536 x 1536): the QR preconditioner's
    panels of 1024 rows or more run on several workgroups (4 to 6) that meet
    at counter barriers; FP64 against the oracle."""
    import bench
    n, sites, lams, bond = bench.micro_state(384)
    rng = np.random.default_rng(91)
    go, gi = bench.haar_su4(rng), bench.haar_su4(rng)
    m = mo.OracleMPO(n)
    m.B = [s.copy() for s in sites]
    m.lam = [l.copy() for l in lams]
    r = mo.bond_update(m, bond, go, gi, 384, 1e-8, "weight", vectors=False)
    g = lib.MPO(n, 384, 1e-8, 1, PREC["fp64"])
    g.load_state(sites, lams)
    info = g.absorb(bond, go, gi)
    s_gpu = g.singular_values(bond)
    right = g.read_site(bond + 1).reshape(info["k"], -1)
    g.close()
    assert info["k"] == r.k
    assert sv_err(s_gpu, r.s[:r.k]) <= TOL["fp64"]
    assert abs(info["discarded"] - r.discarded) <= 1e-10 * r.total
    assert np.max(np.abs(right @ right.conj().T - np.eye(info["k"]))) <= 1e-10


def test_fp64_rank_deficient_tall_panels(lib):
    """theta of rank 8 (all bonds chi = 256, the left tensor a rank-8 product,
    no gate): in the first panel of 1024 rows the later columns are
    combinations of the first eight, so the carried tail norms cancel and the
    multi-workgroup panel falls back to exact sums; FP64 against the oracle."""
    import bench
    n, sites, lams, bond = bench.micro_state(256)
    rng = np.random.default_rng(93)
    cl, cm = sites[bond].shape[0], sites[bond].shape[2]
    u = rng.standard_normal((cl * 4, 8)) + 1j * rng.standard_normal((cl * 4, 8))
    v = rng.standard_normal((8, cm)) + 1j * rng.standard_normal((8, cm))
    b = u @ v
    sites[bond] = (b / np.linalg.norm(b)).reshape(cl, 4, cm)
    m = mo.OracleMPO(n)
    m.B = [x.copy() for x in sites]
    m.lam = [x.copy() for x in lams]
    r = mo.bond_update(m, bond, None, None, 256, 1e-12, "rel_sv", vectors=False)
    g = lib.MPO(n, 256, 1e-12, 0, PREC["fp64"])
    g.load_state(sites, lams)
    info = g.absorb(bond, None, None)
    s_gpu = g.singular_values(bond)
    right = g.read_site(bond + 1).reshape(info["k"], -1)
    g.close()
    assert info["k"] == r.k <= 8
    assert sv_err(s_gpu, r.s[:r.k]) <= TOL["fp64"]
    assert np.max(np.abs(right @ right.conj().T - np.eye(info["k"]))) <= 1e-10

