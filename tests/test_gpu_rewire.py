"""All-to-all input with the transpiler and eager rewiring of Alg. 1
(Sec. II.B.3: strip the transpilation SWAPs after unswapping, reindex by
the accepted swaps, transpile again) on the GPU, against the oracle's run of
the same circuit and settings: the same update sequence (stage, bond, kept
rank), the same peak bits, every bond's values within the precision's
tolerance; and eager and lazy rewiring both recover the planted peak, with
either routing rule (the lower qubit climbs, or the two meet halfway)."""
import numpy as np
import pytest

from oracle import mpo_oracle as mo
from paper_2604_21908_amd import circuitgen as cg

pytestmark = pytest.mark.gpu
TOL = {"fp64": 1e-10, "fp32": 1e-4}


@pytest.fixture(scope="module")
def dr():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    from paper_2604_21908_amd import driver
    return driver


@pytest.mark.parametrize("router", ["up", "middle"])
@pytest.mark.parametrize("rewire", ["eager", "lazy"])
@pytest.mark.parametrize("reading", ["A", "B"])
def test_all_to_all_rewiring_matches_oracle(dr, rewire, reading, router):
    circ = cg.mirrored_peaked_circuit(8, 3, 5, reading=reading, connectivity="all")
    kw = dict(chi_max=256, cutoff=1e-12, tau=400, unswap="parallel", rewire=rewire, router=router)
    c = dr.Contractor(circ, dr.RunConfig(cutoff_mode="rel_sv", precision="fp64", **kw))
    res = c.run()
    lams = [c.m.singular_values(b) for b in range(circ.n - 1)]
    c.close()
    ref = mo.contract(circ.n, circ.gates, mo.OracleConfig(mode="rel_sv", **kw))
    seq = [(t["stage"], t["bond"], t["k"]) for t in res.trace if "k" in t]
    rseq = [(t["stage"], t["bond"], t["k"]) for t in ref.trace if "k" in t]
    assert seq == rseq
    assert sum(1 for t in res.trace if t.get("stage") == "route") > 0
    assert np.array_equal(res.bits, ref.bits) and np.array_equal(res.bits, circ.peak)
    assert abs(res.prob - ref.prob) <= 1e-9 * ref.prob
    for a, r in zip(lams, ref.mpo.lam):
        assert len(a) == len(r) and np.max(np.abs(a - r)) <= TOL["fp64"] * np.linalg.norm(r)
