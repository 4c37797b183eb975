"""Writes the stored expected values of tests/golden/ from the CPU oracle and
the dense brute force only (nothing from the HIP path):

    python tests/golden/make_golden.py

config0_fp64.json: the seeded n = 10 circuit of the CPU-sized workload
(literal reading, R depth 4, chi_max 64, relative cutoff 1e-12, tau 2000,
parallel unswapping), contracted by the oracle (Alg. 1 with App. A.1): the
peak bits and probability of the readout, the final bond dimensions and
singular values; and the argmax of |<x|C|0>|^2 over all 2^10 bitstrings from
the dense statevector, with its probability.

config2_middle.json: the n = 56 circuit of the precision workload (literal
reading, R depth 12, chi_max 1024, discarded-weight cutoff 1e-8, tau 2e4,
parallel unswapping, Alg. 1 alternation, routing rule "middle"), contracted
by the oracle (about a minute): the kept rank of every update in order, the
peak bits and probability, the final bond dimensions and singular values,
the summed discarded weight, and the closed form |<0|K|0>|^2.
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import brute as bf  # noqa: E402
from oracle import mpo_oracle as mo  # noqa: E402
from paper_2604_21908_amd import circuitgen as cg  # noqa: E402

CFG = dict(chi_max=64, cutoff=1e-12, mode="rel_sv", tau=2000.0, unswap="parallel")


def main():
    circ = cg.config_circuit(0, reading="A")
    res = mo.contract(circ.n, circ.gates, mo.OracleConfig(**CFG))
    psi = bf.circuit_state(circ.n, circ.gates)
    prob = np.abs(psi) ** 2
    x = int(np.argmax(prob))
    out = {
        "circuit": {"workload": 0, "index": 0, "reading": "A", "n": circ.n, "depth": circ.meta["depth"],
                    "seed": circ.meta["seed"], "planted_peak": [int(b) for b in circ.peak]},
        "config": CFG,
        "oracle": {"bits": [int(b) for b in res.bits], "prob": float(res.prob), "norm2": float(res.norm2),
                   "bond_dims": res.mpo.bond_dims(),
                   "lambdas": [[float(v) for v in l] for l in res.mpo.lam]},
        "brute": {"bits": [int(b) for b in bf.bits_of(x, circ.n)], "prob": float(prob[x])},
    }
    with open(os.path.join(HERE, "config0_fp64.json"), "w") as f:
        json.dump(out, f, indent=1)
    print("wrote config0_fp64.json: bits", out["oracle"]["bits"], "p", out["oracle"]["prob"],
          "brute p", out["brute"]["prob"])


CFG2 = dict(chi_max=1024, cutoff=1e-8, mode="weight", tau=2e4, unswap="parallel", side="both", router="middle")


def config2():
    circ = cg.config_circuit(2, reading="A")
    res = mo.contract(circ.n, circ.gates, mo.OracleConfig(**CFG2))
    out = {
        "circuit": {"workload": 2, "index": 0, "reading": "A", "n": circ.n, "depth": circ.meta["depth"],
                    "seed": circ.meta["seed"], "gates": len(circ.gates), "planted_peak": [int(b) for b in circ.peak]},
        "config": CFG2,
        "oracle": {"bits": [int(b) for b in res.bits], "prob": float(res.prob),
                   "ranks": [int(t["k"]) for t in res.trace if "k" in t],
                   "discarded": float(sum(t.get("discarded", 0.0) for t in res.trace)),
                   "bond_dims": res.mpo.bond_dims(),
                   "lambdas": [[float(v) for v in l] for l in res.mpo.lam]},
        "closed_form_prob": float(bf.peak_probability_closed_form(circ.n, circ.k_gates)),
    }
    with open(os.path.join(HERE, "config2_middle.json"), "w") as f:
        json.dump(out, f)
    print("wrote config2_middle.json: updates", len(out["oracle"]["ranks"]), "p", out["oracle"]["prob"],
          "closed form", out["closed_form_prob"])


if __name__ == "__main__":
    main()
    config2()
