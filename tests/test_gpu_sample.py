"""Sampling of the output state (Sec. II.C) on the GPU (mpo_sample, through
the C ABI) against the oracle's sampler on the same MPO and the same
uniforms: every decision whose threshold P(0 | prefix) lies farther than the
precision's gray zone from its uniform (1e-9 in FP64, 1e-4 in FP32) is the
same, so the strings agree up to the first gray decision (none is expected
at these sizes), and each string's probability agrees to the precision's
tolerance.  Edge cases: no samples, uniforms outside [0, 1), a two-site
chain, and a chain with chi = 1024 bonds."""
import numpy as np
import pytest

from oracle import mpo_oracle as mo
from paper_2604_21908_amd import circuitgen as cg

pytestmark = pytest.mark.gpu
PREC = {"fp64": 0, "fp32": 1, "mixed": 2}
GRAY = {"fp64": 1e-9, "fp32": 1e-4, "mixed": 1e-4}
TOL = {"fp64": 1e-10, "fp32": 1e-4, "mixed": 1e-4}


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    from paper_2604_21908_amd import mpo as mpolib
    mpolib.load_library()
    return mpolib


def compare(bits, probs, rb, rp, q, u, prec):
    """Samples agree up to their first gray decision; returns how many rows
    were compared in full."""
    full = 0
    for s in range(u.shape[0]):
        gray = np.nonzero(np.abs(u[s] - q[s]) <= GRAY[prec])[0]
        stop = gray[0] if gray.size else u.shape[1]
        assert np.array_equal(bits[s, :stop], rb[s, :stop]), s
        if stop == u.shape[1]:
            full += 1
            assert abs(probs[s] - rp[s]) <= TOL[prec] * max(rp[s], 1e-300) * 10
    return full


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_samples_of_a_contracted_circuit_match_oracle(lib, prec):
    c = cg.mirrored_peaked_circuit(10, 4, 60, reading="A")
    res = mo.contract(c.n, c.gates, mo.OracleConfig(chi_max=64, cutoff=1e-10, mode="weight", tau=200))
    m = res.mpo
    g = lib.MPO(c.n, 64, 1e-10, 1, PREC[prec])
    g.load_state(m.B, m.lam)
    u = np.random.default_rng(5).random((400, c.n))
    bits, probs = g.sample(u)
    rb, rp, q = mo.sample(m, u, with_q=True)
    assert compare(bits, probs, rb, rp, q, u, prec) >= 395
    # the planted peak is the most frequent logical string
    logical = bits[:, res.layout_left]
    keys, counts = np.unique(logical, axis=0, return_counts=True)
    assert np.array_equal(keys[np.argmax(counts)], c.peak)
    g.close()


def test_sampling_edge_cases(lib):
    m = mo.OracleMPO(2)
    rng = np.random.default_rng(2)
    mo.commit(m, mo.bond_update(m, 0, cg.haar_su4(rng), cg.haar_su4(rng), 4, 1e-12, "rel_sv"))
    g = lib.MPO(2, 4, 1e-12, 0, 0)
    g.load_state(m.B, m.lam)
    b0, p0 = g.sample(np.zeros((0, 2)))
    assert b0.shape == (0, 2) and p0.shape == (0,)
    with pytest.raises(lib.MpoError) as e:
        g.sample(np.full((3, 2), 1.0))
    assert e.value.status == -1
    u = rng.random((64, 2))
    bits, probs = g.sample(u)
    rb, rp, q = mo.sample(m, u, with_q=True)
    assert compare(bits, probs, rb, rp, q, u, "fp64") == 64
    g.close()


def test_sampling_at_chi_1024(lib):
    """A right-canonical chain with bonds (4, 16, 64, 256, 1024, 1024, 256,
    64, 16, 4) in FP32: 32 samples agree with the oracle's."""
    n = 11
    dims = [4, 16, 64, 256, 1024, 1024, 256, 64, 16, 4]
    rng = np.random.default_rng(9)
    m = mo.OracleMPO(n)
    chis = [1] + dims + [1]
    m.B = []
    for i in range(n):
        cl, cr = chis[i], chis[i + 1]
        z = rng.standard_normal((4 * cr, cl)) + 1j * rng.standard_normal((4 * cr, cl))
        qm, _ = np.linalg.qr(z)
        m.B.append(qm.conj().T.reshape(cl, 4, cr))
    m.lam = []
    for d in dims:
        lam = np.logspace(0, -3, d)
        m.lam.append(lam / np.linalg.norm(lam))
    g = lib.MPO(n, 1024, 1e-8, 1, 1)
    g.load_state(m.B, m.lam)
    u = rng.random((32, n))
    bits, probs = g.sample(u)
    rb, rp, q = mo.sample(m, u, with_q=True)
    assert compare(bits, probs, rb, rp, q, u, "fp32") >= 31
    g.close()
