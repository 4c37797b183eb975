"""Stored expected values (tests/golden/config0_fp64.json, written by
tests/golden/make_golden.py from the CPU oracle and the dense brute force).

CPU: the oracle still reproduces them and the stored peak is the statevector
argmax.  GPU: the FP64 path reproduces the stored contraction."""
import json
import os

import numpy as np
import pytest

from oracle import brute as bf
from oracle import mpo_oracle as mo
from paper_2604_21908_amd import circuitgen as cg

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "config0_fp64.json")))


def _circuit():
    c = GOLD["circuit"]
    circ = cg.config_circuit(c["workload"], c["index"], reading=c["reading"])
    assert circ.n == c["n"] and [int(b) for b in circ.peak] == c["planted_peak"]
    return circ


def test_oracle_reproduces_golden():
    circ = _circuit()
    res = mo.contract(circ.n, circ.gates, mo.OracleConfig(**GOLD["config"]))
    g = GOLD["oracle"]
    assert [int(b) for b in res.bits] == g["bits"]
    assert abs(res.prob - g["prob"]) <= 1e-12 * g["prob"]
    assert res.mpo.bond_dims() == g["bond_dims"]
    for lam, ref in zip(res.mpo.lam, g["lambdas"]):
        assert np.max(np.abs(np.asarray(lam) - np.asarray(ref))) <= 1e-12


def test_golden_peak_is_the_statevector_argmax():
    """The stored readout is the true maximum of |<x|C|0>|^2 (brute force over
    all 2^10 strings) and equals the planted peak."""
    circ = _circuit()
    g, b = GOLD["oracle"], GOLD["brute"]
    assert g["bits"] == b["bits"] == GOLD["circuit"]["planted_peak"]
    assert abs(g["prob"] - b["prob"]) <= 1e-10 * b["prob"]
    psi = bf.circuit_state(circ.n, circ.gates)
    x = int("".join(map(str, b["bits"])), 2)
    assert abs(abs(psi[x]) ** 2 - b["prob"]) <= 1e-12


@pytest.mark.gpu
def test_gpu_fp64_reproduces_golden():
    import torch
    assert torch.cuda.is_available()
    from paper_2604_21908_amd import driver as dr
    circ = _circuit()
    cfg = GOLD["config"]
    c = dr.Contractor(circ, dr.RunConfig(chi_max=cfg["chi_max"], cutoff=cfg["cutoff"], cutoff_mode=cfg["mode"],
                                         precision="fp64", tau=cfg["tau"], unswap=cfg["unswap"]))
    res = c.run()
    lams = [c.m.singular_values(b) for b in range(circ.n - 1)]
    dims = c.m.bond_dims()
    c.close()
    g = GOLD["oracle"]
    assert [int(x) for x in res.bits] == g["bits"]
    assert abs(res.prob - g["prob"]) <= 1e-10 * g["prob"]
    assert dims == g["bond_dims"]
    for lam, ref in zip(lams, g["lambdas"]):
        assert np.max(np.abs(np.asarray(lam) - np.asarray(ref))) <= 1e-10 * np.linalg.norm(ref)
