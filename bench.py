#!/usr/bin/env python3
"""MPO bond updates/s at chi = 1024 on one MI355X.

One step = one bond update (theta-build, gate pair, truncated SVD, truncation
decision, write-back) at a bond with (chi_l, chi, chi_r) = (1024, 1024, 1024):
theta is a 4096 x 4096 complex matrix and the chi_max = 1024 cap binds.  The
MPO state (random right-canonical site tensors, geometric lambda spectra over
four decades, seed 7) is resident in HBM before timing starts; every step
absorbs a fresh Haar-random SU(4) pair (G_out, G_in).

Prints one JSON line: the rate of the timed updates (`value`); the roofline
of the whole update (`roofline`: the dense-SVD algorithmic flops of one
update by work class over each class's MI355X peak, against the measured time
per update); the roofline of the dominant kernel class on its own terms
(`dominant_kernel_roofline`: algorithmic bytes or flops per launch over the
event-measured launch time, with the HBM traffic the counters measured for
it); the CPU oracle timed on the host cores on the first update, and the
error of the GPU forms' first update against it.
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


def svd_route(prec_name):
    """The library's SVD route for a form: FP64 accumulates the rotations
    (operand rows m, plus r rows of V rotated alongside); the FP32 and mixed
    forms run the Jacobi on the triangular factor of a second QR (r rows) and
    take the vectors from its converged columns, unless MPO_SVD=accumulate."""
    if prec_name == "fp64" or os.environ.get("MPO_SVD") == "accumulate":
        return "accumulate"
    return "qr2"


def kernel_bytes(cls, chi, sweeps, rotations, esz, route="accumulate"):
    """Algorithmic HBM bytes one bond update asks of a memory-bound kernel
    class: a rotated panel reads and writes its (m + r) x 32 complex entries
    (the operand's rows and V's rows; r x 32 on the second-QR route, which
    rotates no V); a Gram step reads m x 32 entries per pair."""
    m = r = 4 * chi
    nblk = r // 16
    if cls == "jacobi_rot":
        return rotations * ((m + r) if route == "accumulate" else r) * 32 * 2 * esz
    if cls == "jacobi_gram":
        return sweeps * (nblk - 1) * (nblk // 2) * m * 32 * esz
    return None


def kernel_flops(cls, chi, sweeps, rotations, route="accumulate"):
    """Algorithmic real flops one bond update asks of a kernel class, at
    (chi_l, chi, chi_r) = (chi, chi, chi): m = r = 4 chi rows/columns, 16-column
    blocks, 32-column panels.  Rotation: each rotated panel is an
    (m + r) x 32 x 32 complex product (r x 32 x 32 on the second-QR route);
    Gram: every panel of every step is an m x 32 x 32 complex product;
    QR: the Householder factorisations' flops (one, or two on the second-QR
    route); theta-build and write-back are the GEMMs' flops.  None where no
    such count is meaningful (latency-bound kernels)."""
    m = r = 4 * chi
    nblk = r // 16
    if cls == "jacobi_rot":
        return rotations * ((m + r) if route == "accumulate" else r) * 32 * 32 * 8.0
    if cls == "jacobi_gram":
        return sweeps * (nblk - 1) * (nblk // 2) * m * 32 * 32 * 8.0
    if cls == "qr":
        # complex Householder QR of an n x n matrix, 8 n^3 - (8/3) n^3 real
        # flops; the second-QR route factors twice
        return (2 if route == "qr2" else 1) * 16.0 / 3.0 * r ** 3
    if cls == "theta_gemm":
        return 128.0 * chi ** 3
    if cls == "writeback_gemm":
        return 8.0 * m * r * chi
    return None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(n, sites, lams, bond, chi, gate):
    """The CPU oracle (complex128 NumPy + LAPACK) on the same update: the
    benchmark's initial state and its first gate pair.  Returns the baseline
    entry and the oracle's result (the FP64 reference of the accuracy check)."""
    from oracle import mpo_oracle as mo
    try:
        from threadpoolctl import threadpool_info
        cores = max([x.get("num_threads", 1) for x in threadpool_info()] or [os.cpu_count()])
    except Exception:
        cores = os.cpu_count()
    m = mo.OracleMPO(n)
    m.B = [s.copy() for s in sites]
    m.lam = [l.copy() for l in lams]
    t0 = time.perf_counter()
    r = mo.bond_update(m, bond, gate[0], gate[1], chi, 1e-8, "weight")
    dt = time.perf_counter() - t0
    return {"value": 1 / dt, "unit": "bond updates/s", "cores": int(cores), "cpu_model": cpu_model(),
            "logical_cpus": os.cpu_count(), "kind": "oracle",
            "sample": f"1 oracle bond update at (chi_l, chi, chi_r) = ({chi}, {chi}, {chi}) from the benchmark's "
                      f"initial state with its first gate pair, theta {4 * chi}x{4 * chi} complex128, "
                      f"numpy.linalg.svd (LAPACK gesdd); with vectors and write-back tensors; {dt:.1f} s with "
                      f"{int(cores)} BLAS threads",
            "seconds": dt, "k": int(r.k)}, r


def accuracy(mpolib, prec_name, n, sites, lams, bond, chi, gate, ref):
    """Error of one GPU update (fresh state, first gate pair) against the FP64
    oracle: singular values normwise over the kept range (max |s - s_ref| /
    |s_ref|), the written operator's excess over the optimal discarded weight
    (Eckart-Young, relative to the total weight) and the largest deviation of
    the new right tensor's rows from orthonormality."""
    from oracle import mpo_oracle as mo
    g = mpolib.MPO(n, chi, 1e-8, mpolib.CUT_WEIGHT, mpolib.PRECISIONS[prec_name])
    g.load_state(sites, lams)
    info = g.absorb(bond, *gate)
    s = g.singular_values(bond)
    left, right = g.read_site(bond), g.read_site(bond + 1).reshape(info["k"], -1)
    g.close()
    k = min(len(s), ref.k)
    lam = lams[bond - 1]
    bl, br = sites[bond], sites[bond + 1]
    th = mo.apply_gates_to_theta(np.tensordot(bl, br, axes=([2], [0])), gate[0], gate[1]) * lam[:, None, None, None]
    theta = th.reshape(bl.shape[0] * 4, -1)
    op = (left * lam[:, None, None]).reshape(-1, info["k"]) @ right
    excess = (np.linalg.norm(theta - op) ** 2 - ref.discarded) / ref.total
    return {"kept_rank": int(info["k"]), "oracle_rank": int(ref.k),
            "sv_err_normwise": float(np.max(np.abs(s[:k] - ref.s[:k])) / np.linalg.norm(ref.s[:ref.k])),
            "excess_discarded_rel": float(excess),
            "right_rows_orthonormality": float(np.max(np.abs(right @ right.conj().T - np.eye(info["k"]))))}


def run_precision(mpolib, torch, prec_name, args, n, sites, lams, bond, gates, events=True):
    h = mpolib.MPO(n, args.chi, 1e-8, mpolib.CUT_WEIGHT, mpolib.PRECISIONS[prec_name])
    h.load_state(sites, lams)
    dims0 = h.bond_dims()
    for w in range(args.warmup):
        h.absorb(bond, *gates[w])
    h.profile(events)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = [h.absorb(bond, *gates[args.warmup + s]) for s in range(args.steps)]
    h.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = h.profile(False)
    dims1 = h.bond_dims()
    h.close()
    return dict(secs=t1 - t0, infos=infos, prof=prof, dims_ok=dims0 == dims1)


HBM_PEAK_GBS = 8000.0
KERNEL_NAME = {"jacobi_rot": "k_jac_rot", "jacobi_gram": "k_jac_gram",
               "jacobi_evd": "k_jac_evd", "qr": "k_qr_panel+k_qr_w1+k_qr_w2+k_qr_upd", "theta_gemm": "k_gemm",
               "writeback_gemm": "k_gemm"}
KERNEL_NAME_MIXED = {"jacobi_rot": "k_jac_rot_mixed", "jacobi_gram": "k_jac_gram_bf16"}


def measured_traffic(kernel, route="accumulate", precision="mixed"):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (profiles/*_traffic.md, two rocprofv3 --pmc passes scaled by the copy
    calibration) taken on the same SVD route, or None when there is none or
    the kernel's sources (the comma-separated `source` files, hashed in that
    order) have changed since the counters were taken."""
    import glob
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    for path in glob.glob(os.path.join(here, "profiles", "*_traffic.md")):
        fields = {}
        for line in open(path):
            if ":" in line and not line.startswith(("|", "#", " ", "`")):
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
        if fields.get("kernel") != kernel or "traffic_bytes_per_launch" not in fields:
            continue
        if fields.get("svd_route", "accumulate") != route or fields.get("precision", "mixed") != precision:
            continue
        digest = hashlib.sha256()
        for name in fields.get("source", "").split(","):
            src = os.path.join(here, name.strip())
            if not name.strip() or not os.path.isfile(src):
                return None
            digest.update(open(src, "rb").read())
        if digest.hexdigest() != fields.get("source_sha256"):
            return None
        return float(fields["traffic_bytes_per_launch"])
    return None


def roofline_of(run, prec_name, chi, steps):
    """Roofline of the dominant kernel class (largest event-timed device
    time).  The panel rotation does 32 complex multiply-adds per complex entry
    it reads and writes: 16 real flops per byte in FP32, 8 in FP64, below the
    MFMA ridges (157.3 / 8 and 78.6 / 8 flops per byte), so it is priced in
    bytes against 8 TB/s.  The Gram step reads only (32 flops per byte in
    FP32): MFMA-bound in FP32/FP64, HBM-bound with split-BF16 products.
    GEMM-shaped kernels are priced in flops against the MFMA peak of their
    dtype; the FP64 panel EVD against the FP64 rate."""
    prof = run["prof"]
    dom = max(prof, key=lambda c: prof[c][0])
    ms, launches = prof[dom]
    sweeps = sum(i["sweeps"] for i in run["infos"])
    rots = sum(i["rotations"] for i in run["infos"])
    esz = 16 if prec_name == "fp64" else 8
    hbm_bound = dom == "jacobi_rot" or (dom == "jacobi_gram" and prec_name == "mixed")
    route = svd_route(prec_name)
    byt = kernel_bytes(dom, chi, sweeps, rots, esz, route) if hbm_bound else None
    names = dict(KERNEL_NAME, **(KERNEL_NAME_MIXED if prec_name == "mixed" else {}))
    if prec_name == "mixed" and route == "qr2":
        names["jacobi_rot"] = "k_jac_rot"          # the operand is rotated on FP32 MFMA on this route
    out = {"kernel": names.get(dom, dom), "class": dom, "svd_route": route,
           "avg_launch_ms": round(ms / max(launches, 1), 5),
           "launches_per_update": launches / steps,
           "traffic": measured_traffic(names.get(dom, dom), route, prec_name)}
    if byt:
        achieved = byt / (ms * 1e-3) / 1e9
        out.update({"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "algorithmic_bytes_per_launch": byt / max(launches, 1)})
        f = kernel_flops(dom, chi, sweeps, rots, route)
        out["tflops"] = round(f / (ms * 1e-3) / 1e12, 3)
        return out
    f = kernel_flops(dom, chi, sweeps, rots, route)
    if dom == "jacobi_evd" or f is None:
        peak, bound = PEAK_TFLOPS["fp64"], "alu"
    else:
        peak, bound = PEAK_TFLOPS["fp64" if prec_name == "fp64" else "fp32"], "mfma"
    achieved = (f / (ms * 1e-3) / 1e12) if f else None
    out.update({"bound": bound, "achieved": None if achieved is None else round(achieved, 3), "peak": peak,
                "unit": "TFLOP/s", "frac": None if achieved is None else round(achieved / peak, 5),
                "algorithmic_flops_per_launch": None if not f else f / max(launches, 1)})
    return out


def update_roofline(prec_name, chi, ms_per_update, traffic=None):
    """Roofline of the whole bond update: T_rf = sum over work classes of
    algorithmic flops / the class's peak, against the measured time per
    update.  The algorithmic work is what a dense SVD would do (the Jacobi
    method's own extra work is overhead): the GEMM class (theta-build,
    Hermitian Gram of theta, eigenvector back-transform, write-back) at the
    MFMA peak of the form's contraction dtype (BF16 for split-BF16 products,
    FP32, FP64), the eigen class (tridiagonal-equivalent reduction, (16/3) n^3)
    at the FP64 peak, and the gate pair at the FP32 vector peak.  Compulsory
    HBM traffic (both site tensors in, theta written and read back, both new
    tensors out) is far below any of these at chi = 1024."""
    f = algorithmic_flops(chi, chi, chi, chi)
    m = n = 4 * chi
    gram, eig, back = 4.0 * m * n * n, 16.0 / 3.0 * n ** 3, 8.0 * n * n * chi
    gemm = f["theta"] + gram + back + f["writeback"]
    gemm_peak = {"fp64": 78.6, "fp32": 157.3, "mixed": 2500.0}[prec_name]
    classes = {"gemm": {"flops": gemm, "peak_tflops": gemm_peak},
               "eigen": {"flops": eig, "peak_tflops": 78.6},
               "gate": {"flops": f["gate"], "peak_tflops": 157.3}}
    t_rf = 0.0
    for c in classes.values():
        c["t_ms"] = round(c["flops"] / (c["peak_tflops"] * 1e12) * 1e3, 4)
        t_rf += c["flops"] / (c["peak_tflops"] * 1e12)
    esz = 16 if prec_name == "fp64" else 8
    compulsory = (2 * 4 * chi * chi + 2 * 16 * chi * chi + 2 * 4 * chi * chi) * esz
    t_meas = ms_per_update * 1e-3
    return {"bound": "mfma", "kernel": "bond update (all of its kernels)", "unit": "TFLOP/s",
            "achieved": round(f["total"] / t_meas / 1e12, 3), "peak": round(f["total"] / t_rf / 1e12, 1),
            "frac": round(t_rf / t_meas, 5), "traffic": traffic,
            "algorithmic_flops_per_update": f["total"], "t_roofline_ms": round(t_rf * 1e3, 3),
            "t_measured_ms": round(ms_per_update, 3), "classes": classes,
            "compulsory_hbm_bytes_per_update": compulsory}


def calibrate_copy(nbytes=1 << 30, reps=3):
    """A plain copy of known size for scaling the hardware byte counters."""
    import torch
    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(reps):
        torch.mul(x, 1.0, out=y)      # one elementwise kernel: reads x, writes y
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read_per_launch": nbytes, "copy_bytes_written_per_launch": nbytes,
                      "launches": reps}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="mixed", choices=["fp64", "fp32", "mixed"])
    ap.add_argument("--compare", default="fp32", help="second precision timed in the same run ('' or none: no second)")
    ap.add_argument("--chi", type=int, default=1024)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mirrored", action="store_true", help="skip the mirrored-pair (G_in = G_out^dag) leg")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy three times (the reference kernel "
                         "that scales the FETCH_SIZE / WRITE_SIZE counters to bytes)")
    args = ap.parse_args()
    if args.compare == "none":
        args.compare = ""
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}): the bond update runs on a "
              f"single GPU and there is no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    rank = int(os.environ.get("RANK", "0"))
    if args.calibrate_copy:
        calibrate_copy()
        return

    import torch
    from paper_2604_21908_amd import mpo as mpolib

    torch.cuda.set_device(0)
    n, sites, lams, bond = micro_state(args.chi)
    rng = np.random.default_rng(1234)
    gates = [(haar_su4(rng), haar_su4(rng)) for _ in range(args.warmup + args.steps)]
    chi = args.chi
    # the headline pass has no per-launch events in its timed region (recorded
    # around every launch they cost about a tenth of the step); the same warmup
    # and steps are then run again with HIP events on the library's stream
    # around every launch, for the per-kernel times and the roofline
    run = run_precision(mpolib, torch, args.precision, args, n, sites, lams, bond, gates, events=False)
    prof_run = run_precision(mpolib, torch, args.precision, args, n, sites, lams, bond, gates, events=True)
    secs = run["secs"]
    value = args.steps / secs
    flops = algorithmic_flops(chi, chi, chi, chi)
    out = {"metric": "MPO bond updates/s at chi=1024", "value": round(value, 4), "unit": "bond updates/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * secs / args.steps, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[args.precision],
           "data": "synthetic (seeded random Vidal-form MPO bond, Haar SU(4) gate pairs)",
           "config": {"workload": f"MPO bond update (chi_l, chi, chi_r) = ({chi}, {chi}, {chi}), theta "
                                  f"{4 * chi}x{4 * chi} complex, chi_max {chi}, discarded-weight cutoff 1e-8",
                      "precision": args.precision, "kept_rank": [i["k"] for i in run["infos"]],
                      "jacobi_sweeps": [i["sweeps"] for i in run["infos"]],
                      "bond_dims_unchanged": run["dims_ok"]},
           "roofline": update_roofline(args.precision, chi, 1e3 * secs / args.steps,
                                       measured_traffic("bond_update_" + args.precision, svd_route(args.precision))),
           "dominant_kernel_roofline": roofline_of(prof_run, args.precision, chi, args.steps),
           "roofline_pass_ms_per_step": round(1e3 * prof_run["secs"] / args.steps, 3),
           "kernels_ms_per_update": {c: round(v[0] / args.steps, 3) for c, v in prof_run["prof"].items() if v[1]}}
    if args.compare and args.compare != args.precision:
        cmp_run = run_precision(mpolib, torch, args.compare, args, n, sites, lams, bond, gates, events=False)
        cmp_prof = run_precision(mpolib, torch, args.compare, args, n, sites, lams, bond, gates, events=True)
        out["compare"] = {"precision": args.compare, "value": round(args.steps / cmp_run["secs"], 4),
                          "ms_per_step": round(1e3 * cmp_run["secs"] / args.steps, 3),
                          "jacobi_sweeps": [i["sweeps"] for i in cmp_run["infos"]],
                          "roofline": update_roofline(args.compare, chi, 1e3 * cmp_run["secs"] / args.steps),
                          "dominant_kernel_roofline": roofline_of(cmp_prof, args.compare, chi, args.steps),
                          "kernels_ms_per_update": {c: round(v[0] / args.steps, 3)
                                                    for c, v in cmp_prof["prof"].items() if v[1]},
                          "speedup_of_headline": round(cmp_run["secs"] / secs, 3)}
    if rank == 0 and not args.no_cpu_baseline:
        out["cpu_baseline"], ref = cpu_baseline(n, sites, lams, bond, chi, gates[0])
        precs = [args.precision] + ([args.compare] if args.compare and args.compare != args.precision else [])
        out["accuracy_vs_fp64_oracle"] = {p: accuracy(mpolib, p, n, sites, lams, bond, chi, gates[0], ref)
                                          for p in precs}
    if not args.no_mirrored:
        # the same update with mirrored pairs (G_in = G_out^dag, the structure of
        # the circuits' two halves), headline precision, no per-launch events
        mgates = [(g, g.conj().T.copy()) for g, _ in gates]
        mrun = run_precision(mpolib, torch, args.precision, args, n, sites, lams, bond, mgates, events=False)
        out["mirrored_pair"] = {"value": round(args.steps / mrun["secs"], 4),
                                "ms_per_step": round(1e3 * mrun["secs"] / args.steps, 3),
                                "jacobi_sweeps": [i["sweeps"] for i in mrun["infos"]],
                                "kept_rank": [i["k"] for i in mrun["infos"]]}
    out["paper_context"] = {"value": 4059, "unit": "s", "hardware": "1x NVIDIA A100 80 GB",
                            "what": "the paper's whole contraction and peak readout of its 56-qubit, 1,917-gate "
                                    "circuit (Sec. III); another workload and machine, not comparable to the "
                                    "per-update rate"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
