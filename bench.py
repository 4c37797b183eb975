#!/usr/bin/env python3
"""MPO bond updates/s at chi = 1024 on one MI355X.

One step = one bond update (theta-build, gate pair, truncated SVD, truncation
decision, write-back) at a bond with (chi_l, chi, chi_r) = (1024, 1024, 1024):
theta is a 4096 x 4096 complex matrix and the chi_max = 1024 cap binds.  The
MPO state (random right-canonical site tensors, geometric lambda spectra over
four decades, seed 7) is resident in HBM before timing starts; every step
absorbs a fresh Haar-random SU(4) pair (G_out, G_in).

Prints one JSON line (see the design doc for the roofline and baseline definitions).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "mixed": 2500.0}
DTYPE = {"fp64": "f64", "fp32": "f32", "mixed": "bf16x3+f32"}


def micro_state(chi: int, seed: int = 7):
    """Vidal-form chain whose middle bond has (chi, chi, chi) around it."""
    rng = np.random.default_rng(seed)
    dims = []
    d = 1
    while d * 4 < chi:
        d *= 4
        dims.append(d)
    left = list(dims)
    dims = left + [chi, chi, chi] + left[::-1]
    n = len(dims) + 1
    chis = [1] + dims + [1]
    sites = []
    for i in range(n):
        cl, cr = chis[i], chis[i + 1]
        z = rng.standard_normal((4 * cr, cl)) + 1j * rng.standard_normal((4 * cr, cl))
        q, _ = np.linalg.qr(z)
        sites.append(q.conj().T.reshape(cl, 4, cr))        # rows orthonormal: right-canonical
    lams = []
    for dm in dims:
        l = np.logspace(0, -4, dm)
        lams.append(l / np.linalg.norm(l))
    bond = len(left) + 1                                    # (chi_l, chi, chi_r) = (chi, chi, chi)
    return n, sites, lams, bond


def haar_su4(rng):
    z = (rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))) / np.sqrt(2)
    q, r = np.linalg.qr(z)
    q = q * (np.diag(r) / np.abs(np.diag(r)))[None, :]
    return q / np.linalg.det(q) ** 0.25


def algorithmic_flops(chil, chi, chir, k):
    """Real flops of one bond update counted as a dense SVD would do it
    (theta-build, gate, Gram, tridiagonal-class eigen, back-transform,
    write-back); complex multiply-add = 8 real flops."""
    m, n = 4 * chil, 4 * chir
    if n > m:
        m, n = n, m
    theta = 128.0 * chil * chi * chir
    gate = 2048.0 * chil * chir
    gram = 4.0 * m * n * n
    eig = 16.0 / 3.0 * n ** 3
    back = 8.0 * n * n * k
    wb = 8.0 * m * n * k
    return dict(theta=theta, gate=gate, svd=gram + eig + back, writeback=wb,
                total=theta + gate + gram + eig + back + wb)


def cpu_baseline(n, sites, lams, bond, chi, samples=1):
    """The CPU oracle (complex128 NumPy + LAPACK) on the same update shape."""
    from oracle import mpo_oracle as mo
    try:
        from threadpoolctl import threadpool_info
        cores = max([x.get("num_threads", 1) for x in threadpool_info()] or [os.cpu_count()])
    except Exception:
        cores = os.cpu_count()
    m = mo.OracleMPO(n)
    m.B = [s.copy() for s in sites]
    m.lam = [l.copy() for l in lams]
    rng = np.random.default_rng(99)
    t0 = time.perf_counter()
    for _ in range(samples):
        r = mo.bond_update(m, bond, haar_su4(rng), haar_su4(rng), chi, 1e-8, "weight")
    dt = time.perf_counter() - t0
    return {"value": samples / dt, "unit": "bond updates/s", "cores": int(cores), "kind": "oracle",
            "sample": f"{samples} oracle bond update(s) at (chi_l, chi, chi_r) = ({chi}, {chi}, {chi}), "
                      f"theta {4 * chi}x{4 * chi} complex128, numpy.linalg.svd (LAPACK gesdd); "
                      f"{dt:.1f} s on {os.cpu_count()} host cores", "seconds": dt, "k": int(r.k)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="fp32", choices=["fp64", "fp32", "mixed"])
    ap.add_argument("--chi", type=int, default=1024)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the path is single-GPU, "
              f"see DESIGN.md for how it would shard", file=sys.stderr)
        sys.exit(2)
    rank = int(os.environ.get("RANK", "0"))

    import torch
    from paper_2604_21908_amd import mpo as mpolib

    torch.cuda.set_device(0)
    n, sites, lams, bond = micro_state(args.chi)
    prec = mpolib.PRECISIONS[args.precision]
    h = mpolib.MPO(n, args.chi, 1e-8, mpolib.CUT_WEIGHT, prec)
    h.load_state(sites, lams)
    rng = np.random.default_rng(1234)
    gates = [(haar_su4(rng), haar_su4(rng)) for _ in range(args.warmup + args.steps)]
    dims0 = h.bond_dims()
    for w in range(args.warmup):
        h.absorb(bond, *gates[w])
    h.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ks, sweeps = [], []
    for s in range(args.steps):
        info = h.absorb(bond, *gates[args.warmup + s])
        ks.append(info["k"])
        sweeps.append(info["sweeps"])
    h.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = h.profile(False)
    dims1 = h.bond_dims()
    h.close()
    secs = t1 - t0
    value = args.steps / secs
    chi = args.chi
    flops = algorithmic_flops(chi, chi, chi, chi)
    dom = max(prof, key=lambda c: prof[c][0])
    dom_ms, dom_launches = prof[dom]
    # algorithmic flops attributed to the dominant kernel class, per update
    part = {"jacobi_step": flops["svd"], "theta_gemm": flops["theta"], "writeback_gemm": flops["writeback"],
            "gate": flops["gate"]}.get(dom, flops["total"])
    achieved = part * args.steps / (dom_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS["fp32" if args.precision == "mixed" else args.precision]
    roofline = {"bound": "mfma", "kernel": f"k_{dom}", "achieved": round(achieved, 3), "peak": peak,
                "unit": "TFLOP/s", "frac": round(achieved / peak, 5), "traffic": None,
                "avg_launch_ms": dom_ms / max(dom_launches, 1), "launches_per_update": dom_launches / args.steps,
                "update_roofline_frac": round(flops["total"] / (secs / args.steps) / 1e12 / peak, 5)}
    out = {"metric": "MPO bond updates/s at chi=1024", "value": round(value, 4), "unit": "bond updates/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * secs / args.steps, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[args.precision],
           "data": "synthetic (seeded random Vidal-form MPO bond, Haar SU(4) gate pairs)",
           "config": {"workload": f"MPO bond update (chi_l, chi, chi_r) = ({chi}, {chi}, {chi}), theta "
                                  f"{4 * chi}x{4 * chi} complex, chi_max {chi}, discarded-weight cutoff 1e-8",
                      "precision": args.precision, "kept_rank": ks, "jacobi_sweeps": sweeps,
                      "bond_dims_unchanged": dims0 == dims1},
           "roofline": roofline,
           "kernels_ms_per_update": {c: round(v[0] / args.steps, 3) for c, v in prof.items()}}
    if rank == 0 and not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(n, sites, lams, bond, chi)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
