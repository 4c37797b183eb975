"""Side selection of the absorption stage (App. A.3) on the GPU, through the
C ABI (mpo_copy_state for the second copy of the adaptive mode), against the
oracle's run of the same circuit and settings: the same side taken at every
step, the same peak bits, every bond's values normwise within the
precision's tolerance and the peak probability within 1e-3 relative."""
import numpy as np
import pytest

from oracle import mpo_oracle as mo
from paper_2604_21908_amd import circuitgen as cg

pytestmark = pytest.mark.gpu
TOL = {"fp64": 1e-10, "fp32": 1e-4, "mixed": 1e-4}


@pytest.fixture(scope="module")
def dr():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    from paper_2604_21908_amd import driver
    return driver


def sides_of(trace):
    return [(t["stage"], t.get("side", t.get("taken"))) for t in trace if t.get("stage") in ("side", "layer")]


def run_both(dr, circ, **kw):
    cfg = dr.RunConfig(**kw)
    c = dr.Contractor(circ, cfg)
    res = c.run()
    lams = [c.m.singular_values(b) for b in range(circ.n - 1)]
    c.close()
    ocfg = mo.OracleConfig(chi_max=cfg.chi_max, cutoff=cfg.cutoff, mode=cfg.cutoff_mode, tau=cfg.tau,
                           unswap=cfg.unswap, side=cfg.side, fixed_freq=cfg.fixed_freq)
    ref = mo.contract(circ.n, circ.gates, ocfg)
    return res, lams, ref


@pytest.mark.parametrize("side,freq", [("adaptive", (1, 1)), ("fixed", (2, 1))])
def test_side_selection_matches_oracle_fp64(dr, side, freq):
    circ = cg.mirrored_peaked_circuit(8, 3, 41, reading="B")
    res, lams, ref = run_both(dr, circ, chi_max=256, cutoff=1e-12, cutoff_mode="rel_sv", precision="fp64",
                              tau=300, side=side, fixed_freq=freq)
    assert sides_of(res.trace) == sides_of(ref.trace) and sides_of(ref.trace)
    assert np.array_equal(res.bits, ref.bits) and np.array_equal(res.bits, circ.peak)
    assert abs(res.prob - ref.prob) <= 1e-9 * ref.prob
    for a, r in zip(lams, ref.mpo.lam):
        assert len(a) == len(r) and np.max(np.abs(a - r)) <= TOL["fp64"] * np.linalg.norm(r)


@pytest.mark.parametrize("prec", ["fp32", "mixed"])
def test_adaptive_matches_oracle_single_precision(dr, prec):
    circ = cg.mirrored_peaked_circuit(10, 4, 60, reading="A")
    res, lams, ref = run_both(dr, circ, chi_max=64, cutoff=1e-10, cutoff_mode="weight", precision=prec,
                              tau=200, side="adaptive")
    assert sides_of(res.trace) == sides_of(ref.trace)
    assert any(t["side"] == "R" for t in ref.trace if t.get("stage") == "side")
    assert np.array_equal(res.bits, ref.bits) and np.array_equal(res.bits, circ.peak)
    assert abs(res.prob - ref.prob) <= 1e-3 * ref.prob
    for a, r in zip(lams, ref.mpo.lam):
        assert len(a) == len(r) and np.max(np.abs(a - r)) <= TOL[prec] * np.linalg.norm(r)
