"""Writes the stored expected values of tests/golden/ from the CPU oracle and
the dense brute force only (nothing from the HIP path):

    python tests/golden/make_golden.py

config0_fp64.json: the seeded n = 10 circuit of the CPU-sized workload
(literal reading, R depth 4, chi_max 64, relative cutoff 1e-12, tau 2000,
parallel unswapping), contracted by the oracle (Alg. 1 with App. A.1): the
peak bits and probability of the readout, the final bond dimensions and
singular values; and the argmax of |<x|C|0>|^2 over all 2^10 bitstrings from
the dense statevector, with its probability.
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


if __name__ == "__main__":
    main()
