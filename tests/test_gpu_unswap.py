"""Unswapping (Sec. II.B.2, App. A.1, A.2) on the GPU: values-only SWAP
trials against the oracle, the exactness of reusing a trial whose inputs are
unchanged, and the acceptance rule as committed."""
import numpy as np
import pytest

from oracle import mpo_oracle as mo
from paper_2604_21908_amd import circuitgen as cg

pytestmark = pytest.mark.gpu
PREC = {"fp64": 0, "fp32": 1, "mixed": 2}
SIDES = ("L", "R", "B")


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    from paper_2604_21908_amd import mpo as mpolib
    mpolib.load_library()
    return mpolib


def swap_mixed_state(n, seed, chi_max):
    """Random gates, then a layer of SWAPs on one side: many trials reduce."""
    rng = np.random.default_rng(seed)
    m = mo.OracleMPO(n)
    for l in range(4):
        for i in range(l % 2, n - 1, 2):
            mo.commit(m, mo.bond_update(m, i, cg.haar_su4(rng), cg.haar_su4(rng), chi_max, 1e-13, "rel_sv"))
    for i in range(0, n - 1, 2):
        side = mo.swap_gates("L" if (i // 2) % 2 == 0 else "R")
        mo.commit(m, mo.bond_update(m, i, side[0], side[1], chi_max, 1e-13, "rel_sv"))
    return m


def layered_swap_state(n, seed, chi_max=64):
    """Haar gate pairs on every third bond, then four SWAP layers (left on
    even bonds, right on odd, left on odd, right on even): the SWAPs raise
    the bond dimensions to 16 and unswapping takes most of them back out over
    several cycles."""
    rng = np.random.default_rng(seed)
    m = mo.OracleMPO(n)
    for b in range(0, n - 1, 3):
        mo.commit(m, mo.bond_update(m, b, cg.haar_su4(rng), cg.haar_su4(rng), chi_max, 1e-13, "rel_sv"))
    for side, par in (("L", 0), ("R", 1), ("L", 1), ("R", 0)):
        go, gi = mo.swap_gates(side)
        for i in range(par, n - 1, 2):
            mo.commit(m, mo.bond_update(m, i, go, gi, chi_max, 1e-13, "rel_sv"))
    return m


def gray(s, k, chi_max, cutoff, rel):
    """True when the discarded-weight decision k sits within relative `rel` of
    its threshold (the tail at k or at k - 1 is that close to cutoff * total);
    a decision bound by chi_max is gray when the uncapped rank is that close."""
    sq = s * s
    total = sq.sum()
    thr = cutoff * total
    tail = np.cumsum(sq[::-1])[::-1]            # tail[j] = sum_{i >= j} s_i^2
    kc = mo.truncation_rank(s, s.size, cutoff, "weight")
    near = abs(tail[kc] - thr) <= rel * thr if kc < s.size else False
    near |= abs(tail[kc - 1] - thr) <= rel * thr if kc >= 1 else False
    if k == chi_max and kc > chi_max:
        return False
    return bool(near)


@pytest.mark.parametrize("prec", ["mixed", "fp32", "fp64"])
def test_trial_rank_matches_oracle_outside_gray_zone(lib, prec):
    """Every bond and side of two states: the GPU trial's k equals the
    oracle's (full SVD of the same SWAP-gated theta) wherever the oracle's
    decision is not within the gray zone of the cutoff (1e-3 relative for
    FP32 and mixed, 1e-6 for FP64); kept weights agree to the tolerance."""
    cutoff, chi_max = 1e-6, 64
    rel = 1e-6 if prec == "fp64" else 1e-3
    tol = 1e-10 if prec == "fp64" else 1e-4
    checked = 0
    for seed in (1, 2):
        m = swap_mixed_state(8, seed, 64)
        g = lib.MPO(m.n, chi_max, cutoff, 1, PREC[prec])
        g.load_state(m.B, m.lam)
        for b in range(m.n - 1):
            for sd in range(3):
                go, gi = mo.swap_gates(SIDES[sd])
                r = mo.bond_update(m, b, go, gi, chi_max, cutoff, "weight", vectors=False)
                t = g.trial_swap(b, sd)
                assert abs(t["total"] - r.total) <= tol * r.total
                if gray(r.s, r.k, chi_max, cutoff, rel):
                    continue
                assert t["k"] == r.k, (seed, b, SIDES[sd])
                assert abs(t["discarded"] - r.discarded) <= tol * r.total
                checked += 1
        assert g.bond_dims() == m.bond_dims()           # trials change nothing
        g.close()
    assert checked >= 30


@pytest.mark.parametrize("prec", ["mixed", "fp32"])
@pytest.mark.parametrize("schedule", ["parallel", "sequential"])
def test_accepted_swaps_lower_their_bonds(lib, prec, schedule):
    """Strict acceptance as committed: every accepted swap lowers its own bond
    and touches no other, so the sum of bond dimensions falls by at least the
    number of accepted swaps; the accepted swaps reproduce the oracle's log on
    this state (its decisions are far from the cutoff's gray zone)."""
    m = layered_swap_state(9, 7)
    g = lib.MPO(m.n, 64, 1e-8, 1, PREC[prec])
    g.load_state(m.B, m.lam)
    before = sum(g.bond_dims())
    log = g.unswap(schedule)
    after = sum(g.bond_dims())
    assert len(log) > 0
    assert before - after >= len(log)
    run = mo.unswap_parallel if schedule == "parallel" else mo.unswap_sequential
    o = m.copy()
    ref = run(o, mo.OracleConfig(chi_max=64, cutoff=1e-8, mode="weight", unswap=schedule))
    assert log == ref
    assert g.bond_dims() == o.bond_dims()
    g.close()


@pytest.mark.parametrize("prec", ["mixed", "fp32", "fp64"])
def test_trial_reuse_is_exact(lib, prec, monkeypatch):
    """Reusing the result of a trial whose B_b, B_b+1 and lambda_b-1 are
    unchanged is bit-identical to running it again: logs, bond values and
    tensors equal bit for bit with the memo on and off; the memo is used."""
    m = layered_swap_state(10, 4)

    def run(reuse):
        monkeypatch.setenv("MPO_TRIAL_REUSE", "1" if reuse else "0")
        g = lib.MPO(m.n, 64, 1e-8, 1, PREC[prec])
        monkeypatch.delenv("MPO_TRIAL_REUSE")
        g.load_state(m.B, m.lam)
        log = g.unswap("parallel")
        out = (log, g.bond_dims(), [g.read_site(i) for i in range(m.n)],
               [g.singular_values(b) for b in range(m.n - 1)], g.counters())
        g.close()
        return out

    a, b = run(True), run(False)
    assert a[0] == b[0] and len(a[0]) > 0
    assert a[1] == b[1]
    for x, y in zip(a[2], b[2]):
        assert np.array_equal(x, y)
    for x, y in zip(a[3], b[3]):
        assert np.array_equal(x, y)
    assert a[4]["trials_reused"] > 0 and b[4]["trials_reused"] == 0
    assert a[4]["trials"] + a[4]["trials_reused"] == b[4]["trials"]
