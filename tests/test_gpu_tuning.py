"""Launch choices of the Jacobi sweeps (row chunk of the panel rotation,
sweep captured as a HIP graph and replayed) and their autotuner: every choice
gives bit-identical contractions (same bits, probability and bond values),
the graph choices really replay captured sweeps, and the autotuner settles
on one choice per bucket after measuring all of them."""
import numpy as np
import pytest

from paper_2604_21908_amd import circuitgen as cg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    from paper_2604_21908_amd import driver, mpo
    mpo.load_library()
    yield driver, mpo
    mpo.tuning_set(-1)


def contract(dr, prec):
    circ = cg.mirrored_peaked_circuit(10, 4, 42, reading="B")
    c = dr.Contractor(circ, dr.RunConfig(chi_max=64, cutoff=1e-10, cutoff_mode="weight", precision=prec,
                                         tau=1000))
    res = c.run()
    lams = [c.m.singular_values(b) for b in range(circ.n - 1)]
    cnt = c.m.counters()
    c.close()
    return res, lams, cnt


@pytest.mark.parametrize("prec", ["fp32", "mixed"])
def test_every_sweep_choice_is_bit_identical(mods, prec):
    dr, mpo = mods
    mpo.tuning_set(-2)
    ref, ref_lams, _ = contract(dr, prec)
    for choice in range(6):
        mpo.tuning_set(choice)
        res, lams, cnt = contract(dr, prec)
        assert np.array_equal(res.bits, ref.bits) and res.prob == ref.prob, choice
        for a, b in zip(lams, ref_lams):
            assert np.array_equal(a, b), choice
        if choice >= 3:
            assert cnt["graph_replays"] > 0 and cnt["graph_captures"] > 0
        else:
            assert cnt["graph_replays"] == 0
    mpo.tuning_set(-1)


def test_autotuner_decides_a_bucket(mods):
    dr, mpo = mods
    mpo.tuning_set(-1)
    n = 8
    rng = np.random.default_rng(3)
    m = mpo.MPO(n, 64, 1e-10, 1, 1)
    for layer in range(6):                       # bond dimensions up to 64 at the centre
        for b in range(layer % 2, n - 1, 2):
            m.absorb(b, cg.haar_su4(rng), cg.haar_su4(rng))
    for _ in range(16):                          # one bucket (fp32, r 256, single updates)
        m.absorb(3, cg.haar_su4(rng), cg.haar_su4(rng))
    m.close()
    rep = mpo.tuning_report()
    line = [x for x in rep.splitlines() if x.startswith("gfx950 fp32 r256 b1")]
    assert line and "rrc=" in line[0] and "graph=" in line[0], rep
