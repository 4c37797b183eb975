"""The sawtooth of Sec. III.A on the GPU: size(M) after every absorption
step and every unswapping stage, against the number of circuit gates
absorbed, equals the oracle's sequence exactly (integers) under both
unswapping schedules (Alg. 1 sequential, App. A.1 parallel) and both
acceptance rules (strict, App. A.2 relaxed), on a circuit whose ranks are
exact (no truncation, FP64)."""
import numpy as np
import pytest

from oracle import mpo_oracle as mo
from paper_2604_21908_amd import circuitgen as cg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dr():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    from paper_2604_21908_amd import driver
    return driver


@pytest.mark.parametrize("schedule", ["sequential", "parallel"])
@pytest.mark.parametrize("relaxed", [False, True])
def test_sawtooth_equals_oracle(dr, schedule, relaxed):
    circ = cg.mirrored_peaked_circuit(10, 4, 42, reading="B")
    kw = dict(chi_max=1024, cutoff=1e-12, tau=1000, unswap=schedule, relaxed=relaxed)
    c = dr.Contractor(circ, dr.RunConfig(cutoff_mode="rel_sv", precision="fp64", **kw))
    res = c.run()
    sizes = list(c.sizes)
    c.close()
    ref = mo.contract(circ.n, circ.gates, mo.OracleConfig(mode="rel_sv", **kw))
    assert sizes == ref.sizes
    assert sum(1 for s in sizes if s[0] == "unswap") >= 5
    assert sizes[-1][1] == len(circ.gates)
    assert np.array_equal(res.bits, ref.bits)
