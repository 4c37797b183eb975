"""Measurements of the batched and served forms (one JSON line each).

    python -m paper_2604_21908_amd.forms_bench batch --count 16
    python -m paper_2604_21908_amd.forms_bench serve --rate 1 --duration 10
    python -m paper_2604_21908_amd.forms_bench peak --config 1 --precisions fp32,mixed

batch: the first `count` circuits of the batching workload (n ~ U{16..48},
depth ~ U{4..10}, chi_max ~ U{128, 256, 512}, literal reading, FP32),
contracted in lockstep with group launches and again with one launch per
update; aggregate bond updates/s and makespan of both.
serve: Poisson arrivals at `rate`/s for `duration` s, n in {24, 40, 56}
(p = 0.5/0.3/0.2), depth n/4, chi_max 512, mixed precision, admission by
projected n chi^2 16 B within `budget_gb`; p50/p99 time-to-peak from arrival
and circuits/s, beside the same arrivals served one at a time in FP32.
peak: time-to-peak of one seeded circuit of a configuration (literal reading;
config 1: n = 32, depth 8, chi_max 256, discarded-weight cutoff 1e-8, parallel
unswapping at size tau) in each precision, with the planted peak checked.
--max-n and --chi-cap bound the batch and serve workloads (widest circuit,
largest chi_max) so a run fits a time budget."""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import batch as bt
from . import circuitgen as cg
from . import driver as dr
from . import serve as sv


def _progress(tag):
    last = [time.perf_counter()]

    def cb(rounds, active):
        now = time.perf_counter()
        if now - last[0] > 3.0:
            print(f"  [{tag}] round {rounds}, resident {active}", flush=True)
            last[0] = now
    return cb


class _TimeLimit(Exception):
    pass


class _Checkpoint(Exception):
    pass


def _save_state(path, c, steps, seconds, max_k):
    """The contraction after a complete unswapping stage: every site tensor
    and bond vector as stored, both wire layouts, the absorption steps done
    and the bookkeeping of the time-to-peak (numpy .npz, no pickles)."""
    n = c.n
    # the MPO's own precision (complex64 values round-trip exactly)
    dt = np.complex128 if c.cfg.precision == "fp64" else np.complex64
    arrs = {f"site{i}": c.m.read_site(i).astype(dt) for i in range(n)}
    arrs.update({f"lam{b}": c.m.singular_values(b) for b in range(n - 1)})
    arrs.update(out_site_of=c.out_w.site_of, out_logical_at=c.out_w.logical_at, in_site_of=c.in_w.site_of,
                in_logical_at=c.in_w.logical_at, steps=np.array(steps), seconds=np.array(seconds),
                max_k=np.array(max_k), bond_updates=np.array(c.bond_updates))
    np.savez(path, **arrs)


def _load_state(path, c):
    """Inverse of _save_state on a fresh Contractor of the same circuit and
    configuration; returns (steps, seconds, max_k)."""
    z = np.load(path)
    steps = int(z["steps"])
    for _ in range(steps):                 # the layers those steps absorbed, innermost first
        if c.c_left:
            c.c_left.pop(0)
        if c.c_right:
            c.c_right.pop(0)
    c.out_w.site_of, c.out_w.logical_at = z["out_site_of"].copy(), z["out_logical_at"].copy()
    c.in_w.site_of, c.in_w.logical_at = z["in_site_of"].copy(), z["in_logical_at"].copy()
    c.m.load_state([z[f"site{i}"] for i in range(c.n)], [z[f"lam{b}"] for b in range(c.n - 1)])
    c.bond_updates = int(z["bond_updates"])
    return steps, float(z["seconds"]), int(z["max_k"])


def p_closed(circ) -> float:
    """|<0^n|K|0^n>|^2, the probability of the planted peak (C = X^b K as an
    operator): the product of K|0^n>'s prefix conditionals P(x_j = 0 | 0..0),
    which the generator already evaluates exactly for its admissibility
    check (K's two brickwork layers in their order)."""
    n = circ.n
    first = len(cg.brickwork_pairs(n, 0))
    layers = [circ.k_gates[:first], circ.k_gates[first:]]
    return float(np.prod(cg.k_prefix_conditionals(n, layers)))


def peak_checks(results, circuits) -> dict:
    """Planted bits bit-exact and p within 1e-3 relative of the closed form
    (plus the discarded weight the run reports) for every finished circuit."""
    bits_ok = p_ok = 0
    worst = 0.0
    for r, circ in zip(results, circuits):
        if r is None:
            continue
        bits_ok += bool((r.bits == circ.peak).all())
        pc = p_closed(circ)
        disc = sum(t.get("discarded", 0.0) for t in r.trace)
        err = abs(r.prob - pc) / pc
        worst = max(worst, err)
        p_ok += err <= 1e-3 + disc / pc
    return {"bits_ok": bits_ok, "p_ok": p_ok, "worst_p_rel_err": worst}


def sample_report(c, circ, count, p_exact, seed=2026):
    """Sec. II.C / Fig. 4 on a contracted circuit: `count` samples of the
    output state (mpo_sample, seeded uniforms), mapped to logical qubits by
    the output layout; the 20 most frequent strings with their counts, the
    planted peak's sampled weight and its exact probability p*."""
    rng = np.random.default_rng(seed)
    u = rng.random((count, c.n))
    t0 = time.perf_counter()
    site_bits, probs = c.m.sample(u)
    secs = time.perf_counter() - t0
    logical = site_bits[:, c.out_w.site_of]               # column q = logical qubit q
    keys = ["".join(map(str, row)) for row in logical]
    hist = {}
    for k in keys:
        hist[k] = hist.get(k, 0) + 1
    top = sorted(hist.items(), key=lambda kv: (-kv[1], kv[0]))[:20]
    peak = "".join(map(str, circ.peak))
    return {"samples": count, "seed": seed, "seconds": round(secs, 3),
            "top20": [[k, v] for k, v in top], "peak": peak, "peak_count": hist.get(peak, 0),
            "sampled_peak_weight": hist.get(peak, 0) / count, "exact_p_peak": p_exact,
            "distinct": len(hist)}


def sawtooth(a):
    """Sec. III.A / Fig. 3 and App. A.1-A.2 on one seeded circuit: for every
    tau, unswapping schedule (sequential, parallel) and acceptance (strict,
    relaxed), size(M) after each absorption step and each unswapping stage
    against the gates absorbed, with time-to-peak, bond updates, SWAP-trial
    SVDs and the peak check.  One JSON line per run, then a summary."""
    circ = cg.config_circuit(a.config, reading=a.reading)
    prec = a.precision or "fp32"
    runs = []
    for tau in [float(x) for x in a.taus.split(",")]:
        for sched in ("sequential", "parallel"):
            for relaxed in (False, True):
                c = dr.Contractor(circ, dr.RunConfig(chi_max=a.chi, cutoff=1e-8, cutoff_mode="weight",
                                                     precision=prec, tau=tau, unswap=sched, relaxed=relaxed,
                                                     side=a.side, router=a.router))
                t0 = time.perf_counter()
                last = [t0]
                orig_step, orig_unswap = c.absorb_step, c.unswap

                def guard(fn, c=c, tag=f"tau {tau:g} {sched}{' relaxed' if relaxed else ''}"):
                    def run_it():
                        now = time.perf_counter()
                        if a.run_limit and now - t0 > a.run_limit:
                            raise _TimeLimit()
                        if now - last[0] > 15:
                            last[0] = now
                            print(f"  [{tag}] {c.gates_absorbed} gates absorbed, size {c.m.total_elements()}, "
                                  f"t = {now - t0:.1f} s", flush=True)
                        return fn()
                    return run_it
                c.absorb_step, c.unswap = guard(orig_step), guard(orig_unswap)
                finished = True
                try:
                    res = c.run()
                except _TimeLimit:
                    finished, res = False, None
                secs = time.perf_counter() - t0
                cnt = c.m.counters()
                c.close()
                if not finished:
                    run = {"tau": tau, "schedule": sched, "relaxed": relaxed, "precision": prec, "finished": False,
                           "seconds": round(secs, 3), "bond_updates": c.bond_updates,
                           "gates_absorbed": c.gates_absorbed, "of_gates": len(circ.gates),
                           "trial_svds": cnt["trials"], "trials_reused": cnt["trials_reused"],
                           "unswap_stages": sum(1 for st, g, sz in c.sizes if st == "unswap"),
                           "max_size": max([sz for st, g, sz in c.sizes] or [0]), "peak_ok": None,
                           "sizes": [[st[0], g, sz] for st, g, sz in c.sizes]}
                    runs.append(run)
                    print(json.dumps(run), flush=True)
                    continue
                stages = [(g, sz) for st, g, sz in c.sizes if st == "unswap"]
                pre = [sz for st, g, sz in c.sizes]
                drops = []
                for j, (st, g, sz) in enumerate(c.sizes):
                    if st == "unswap" and j > 0:
                        drops.append(c.sizes[j - 1][2] - sz)
                run = {"tau": tau, "schedule": sched, "relaxed": relaxed, "precision": prec, "finished": True,
                       "seconds": round(secs, 3), "bond_updates": res.bond_updates,
                       "trial_svds": cnt["trials"], "trials_reused": cnt["trials_reused"],
                       "unswap_stages": len(stages), "max_size": max(pre) if pre else 0,
                       "mean_unswap_drop": round(float(np.mean(drops)), 1) if drops else 0.0,
                       "peak_ok": bool((res.bits == circ.peak).all()), "p_peak": res.prob,
                       "sizes": [[st[0], g, sz] for st, g, sz in c.sizes]}
                runs.append(run)
                print(json.dumps(run), flush=True)
    best = min([r for r in runs if r["finished"]] or runs, key=lambda r: r["seconds"])
    print(json.dumps({"form": "sawtooth", "config": a.config, "n": circ.n, "reading": a.reading,
                      "chi_max": a.chi, "side": a.side, "runs": len(runs),
                      "fastest": {k: best[k] for k in ("tau", "schedule", "relaxed", "seconds")},
                      "all_finished_peaks_ok": all(r["peak_ok"] for r in runs if r["finished"]),
                      "run_limit_s": a.run_limit,
                      "table": [{k: r.get(k) for k in ("tau", "schedule", "relaxed", "finished", "seconds",
                                                       "bond_updates", "trial_svds", "unswap_stages", "max_size",
                                                       "peak_ok", "p_peak")}
                                for r in runs]}), flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("form", choices=["batch", "serve", "peak", "sawtooth"])
    ap.add_argument("--taus", default="5e3,2e4,1e5", help="sawtooth: the tau values to run")
    ap.add_argument("--run-limit", type=float, default=60.0,
                    help="sawtooth: stop a run after this many seconds and report it unfinished")
    ap.add_argument("--reading", default="A", choices=["A", "B"], help="sawtooth/peak: circuit reading")
    ap.add_argument("--config", type=int, default=1)
    ap.add_argument("--chi", type=int, default=256)
    ap.add_argument("--time-limit", type=float, default=0.0,
                    help="peak: stop a precision's run after this many seconds and report how far it got")
    ap.add_argument("--checkpoint-after", type=float, default=0.0,
                    help="peak: after the first unswapping stage that ends past this many seconds, save the "
                         "contraction's state to --state and stop (one precision)")
    ap.add_argument("--checkpoint-at-step", type=int, default=0,
                    help="peak: save to --state and stop at the end of the first unswapping stage after this "
                         "many absorption steps (whatever the time and size)")
    ap.add_argument("--checkpoint-max-elements", type=float, default=4e6,
                    help="peak: checkpoint only at a stage whose MPO holds at most this many elements")
    ap.add_argument("--state", default="", help="peak: checkpoint file (.npz)")
    ap.add_argument("--resume", action="store_true", help="peak: continue from --state")
    ap.add_argument("--precisions", default="fp32,mixed")
    ap.add_argument("--side", default="both", choices=["both", "adaptive", "fixed"],
                    help="peak: side selection of the absorption stage (Alg. 1 alternation, or App. A.3)")
    ap.add_argument("--samples", type=int, default=0,
                    help="peak: after the contraction draw this many seeded samples of the output state (Sec. II.C) "
                         "and report the top-20 histogram and the sampled peak weight beside p*")
    ap.add_argument("--verbose", action="store_true", help="peak: a line for every absorption step over 1 s")
    ap.add_argument("--router", default="middle", choices=["up", "middle"],
                    help="routing of non-adjacent gates (the measured workloads use middle)")
    ap.add_argument("--rewire", default="lazy", choices=["lazy", "eager"], help="peak: rewiring mode")
    ap.add_argument("--n", type=int, default=0, help="peak: a circuit of this width instead of the config's")
    ap.add_argument("--depth", type=int, default=0, help="peak: R depth with --n (default n/4)")
    ap.add_argument("--seed", type=int, default=-1, help="peak: generator seed with --n (default 1000 * config)")
    ap.add_argument("--count", type=int, default=16)
    ap.add_argument("--rounds", type=int, default=0,
                    help="batch: stop both ways after this many lockstep rounds (0: run every circuit to its peak)")
    ap.add_argument("--tau", type=float, default=1e5)
    ap.add_argument("--rate", type=float, default=1.0)
    ap.add_argument("--duration", type=float, default=10.0)
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--light-chi", type=int, default=64,
                    help="serve: round policy (circuits with bonds up to this all step; 0: lockstep)")
    ap.add_argument("--deadline", type=float, default=0.0,
                    help="serve: cancel a request this many seconds after its arrival (0: never)")
    ap.add_argument("--precision", default=None)
    ap.add_argument("--max-n", type=int, default=64, help="skip workload circuits wider than this")
    ap.add_argument("--chi-cap", type=int, default=1024, help="clip the workload's chi_max to this")
    a = ap.parse_args(argv)
    if a.form == "sawtooth":
        sawtooth(a)
        return
    if a.form == "peak":
        import time as _t
        if a.n:
            circ = cg.mirrored_peaked_circuit(a.n, a.depth or a.n // 4, a.seed if a.seed >= 0 else 1000 * a.config,
                                              reading=a.reading)
        else:
            circ = cg.config_circuit(a.config, reading=a.reading)
        tau = a.tau if a.tau != 1e5 else 2e4
        out = {"form": "peak", "config": a.config, "n": circ.n, "chi_max": a.chi, "tau": tau, "runs": []}
        pc = p_closed(circ)
        lams = {}
        for prec in a.precisions.split(","):
            c = dr.Contractor(circ, dr.RunConfig(chi_max=a.chi, cutoff=1e-8, cutoff_mode="weight", precision=prec,
                                                 tau=tau, unswap="parallel", side=a.side, router=a.router,
                                                 rewire=a.rewire))
            steps = [0]
            done_s, max_k0 = 0.0, 1
            if a.resume:
                steps[0], done_s, max_k0 = _load_state(a.state, c)
            t0 = _t.perf_counter()
            last = [t0]
            orig = c.absorb_step

            def step(orig=orig):
                if a.time_limit and _t.perf_counter() - t0 > a.time_limit:
                    raise _TimeLimit()
                ts, tr = _t.perf_counter(), c.trial_absorb_updates
                orig()
                steps[0] += 1
                now = _t.perf_counter()
                if steps[0] % 5 == 0 or now - last[0] > 20 or (a.verbose and now - ts > 1.0):
                    last[0] = now
                    side = ""
                    if c.trace and c.trace[-1].get("stage") == "side":
                        x = c.trace[-1]
                        side = (f", took {x['side']} (sizes L {x['size_left']}, R {x['size_right']}), "
                                f"trial updates {c.trial_absorb_updates - tr}")
                    print(f"  [{prec}] step {steps[0]} of {total_steps}, max chi {max(c.m.bond_dims())}, "
                          f"updates {c.bond_updates}{side}, step {now - ts:.1f} s, t = {done_s + now - t0:.1f} s",
                          flush=True)
            total_steps = steps[0] + (len(c.c_left) + len(c.c_right) if a.side != "both"
                                      else max(len(c.c_left), len(c.c_right)))
            c.absorb_step = step

            def unswap_by_cycle(c=c, prec=prec):
                # one parallel cycle per call until a cycle accepts nothing:
                # with strict acceptance a cycle reduces iff it accepts, so
                # this is the library's own loop, with a line per cycle
                before = c.m.total_elements()
                log = []
                for it in range(c.cfg.max_unswap_iters):
                    got = c.m.unswap(c.cfg.unswap, c.cfg.relaxed, 1)
                    log += got
                    print(f"  [{prec}] unswap cycle {it + 1}: {len(got)} accepted, "
                          f"size {c.m.total_elements()}, t = {done_s + _t.perf_counter() - t0:.1f} s", flush=True)
                    if not got:
                        break
                c.record_unswap(log, before)
                elapsed = done_s + _t.perf_counter() - t0
                at_time = (a.checkpoint_after and elapsed > a.checkpoint_after
                           and c.m.total_elements() <= a.checkpoint_max_elements)
                at_step = a.checkpoint_at_step and steps[0] >= a.checkpoint_at_step
                if (at_time or at_step) and (c.c_left or c.c_right):
                    ks = [x["k"] for x in c.trace if "k" in x]
                    _save_state(a.state, c, steps[0], elapsed, max([max_k0] + ks))
                    raise _Checkpoint()
                return log
            if c.cfg.unswap == "parallel" and not c.cfg.relaxed:
                c.unswap = unswap_by_cycle
            try:
                res = c.run()
            except _Checkpoint:
                z = np.load(a.state)
                out["runs"].append({"precision": prec, "checkpoint": a.state, "seconds": round(float(z["seconds"]), 3),
                                    "absorption_steps": int(z["steps"]), "of_steps": total_steps,
                                    "bond_updates": int(z["bond_updates"]), "max_chi": int(z["max_k"])})
                c.close()
                print(json.dumps(out["runs"][-1]), flush=True)
                continue
            except _TimeLimit:
                ks = [x["k"] for x in c.trace if "k" in x]
                out["runs"].append({"precision": prec, "finished": False, "seconds": round(_t.perf_counter() - t0, 3),
                                    "absorption_steps": steps[0], "of_steps": total_steps,
                                    "bond_updates": c.bond_updates, "max_chi": max(ks) if ks else 1})
                c.close()
                print(json.dumps(out["runs"][-1]), flush=True)
                continue
            sampled = None
            if a.samples:
                sampled = sample_report(c, circ, a.samples, res.prob)
            lams[prec] = [c.m.singular_values(b) for b in range(circ.n - 1)]
            c.close()
            ks = [x["k"] for x in res.trace if "k" in x]
            secs = done_s + res.seconds
            out["runs"].append({"precision": prec, "side": a.side, "router": a.router, "rewire": a.rewire,
                                "finished": True, "time_to_peak_s": round(secs, 3),
                                "resumed": bool(a.resume), "bond_updates": res.bond_updates,
                                "trial_absorb_updates": c.trial_absorb_updates,
                                "max_chi": max([max_k0] + ks),
                                "peak_ok": bool((res.bits == circ.peak).all()), "p_peak": res.prob,
                                "p_rel_err_closed_form": abs(res.prob - pc) / pc,
                                "updates_per_s": round(res.bond_updates / secs, 1)})
            if sampled:
                out["runs"][-1]["sampling"] = sampled
            print(json.dumps(out["runs"][-1]), flush=True)
        if "fp64" in lams:
            # every bond's final values against the FP64 run's (itself within
            # 1e-10 of the oracle), normwise per bond, worst bond
            for run in out["runs"]:
                got = lams.get(run["precision"])
                if got is None or not run.get("finished"):
                    continue
                errs = [float(np.max(np.abs(x - r)) / np.linalg.norm(r)) if len(x) == len(r) else float("inf")
                        for x, r in zip(got, lams["fp64"])]
                run["lambda_err_vs_fp64"] = max(errs)
        print(json.dumps(out), flush=True)
        return
    if a.form == "batch":
        prec = a.precision or "fp32"
        work = []
        for circ, chi in cg.batch_workload(128):
            if len(work) == a.count:
                break
            if circ.n > a.max_n:
                continue
            circ = cg.mirrored_peaked_circuit(circ.n, circ.meta["depth"], circ.meta["seed"], reading="A")
            work.append((circ, dr.RunConfig(chi_max=min(chi, a.chi_cap), cutoff=1e-8, cutoff_mode="weight",
                                            precision=prec, tau=a.tau, side=a.side, router=a.router)))
        print(f"  batch of {len(work)} circuits, n = {[c.n for c, _ in work]}, "
              f"chi_max = {[c.chi_max for _, c in work]}", flush=True)
        orig = bt.run_round
        rounds = [0]
        last = [time.perf_counter()]

        def counted(tasks, group, per_update=False):
            rounds[0] += 1
            if rounds[0] % 10 == 0 or time.perf_counter() - last[0] > 15:
                last[0] = time.perf_counter()
                print(f"  round {rounds[0]} ({'per-update' if per_update else 'grouped'}), "
                      f"{sum(1 for t in tasks if t.done)} of {len(tasks)} finished", flush=True)
            return orig(tasks, group, per_update)
        bt.run_round = counted
        g = bt.run_batched(work, precision=prec, max_rounds=a.rounds)
        rounds[0] = 0
        p = bt.run_batched(work, precision=prec, per_update=True, max_rounds=a.rounds)
        done = [(r, q, c) for r, q, (c, _) in zip(g["results"], p["results"], work) if r is not None and q is not None]
        ok = all((r.bits == c.peak).all() for r, q, c in done)
        same = all((r.bits == q.bits).all() and r.prob == q.prob for r, q, c in done)
        checks = peak_checks(g["results"], [c for c, _ in work])
        print(json.dumps({"form": "batch", "circuits": len(work), "precision": prec, "tau": a.tau, "side": a.side,
                          "router": a.router,
                          "rounds_cap": a.rounds, "n": [c.n for c, _ in work], "chi_max": [c.chi_max for _, c in work],
                          "grouped": {"seconds": round(g["seconds"], 3), "bond_updates": g["bond_updates"],
                                      "rounds": g["rounds"], "finished": g["finished"],
                                      "updates_per_s": round(g["updates_per_s"], 1)},
                          "per_update_launch": {"seconds": round(p["seconds"], 3), "bond_updates": p["bond_updates"],
                                                "rounds": p["rounds"], "finished": p["finished"],
                                                "updates_per_s": round(p["updates_per_s"], 1)},
                          "speedup": round(p["seconds"] / g["seconds"], 3), "finished_both": len(done),
                          "peaks_ok": bool(ok), "grouped_equals_per_update": bool(same),
                          "closed_form_checks": checks}), flush=True)
    else:
        prec = a.precision or "mixed"
        cfg = dr.RunConfig(chi_max=min(512, a.chi_cap), cutoff=1e-8, cutoff_mode="weight", precision=prec,
                           tau=a.tau, side=a.side, router=a.router)
        reqs = [r for r in sv.poisson_requests(a.rate, a.duration) if r.n <= a.max_n]
        print(f"  {len(reqs)} requests, n = {[r.n for r in reqs]}", flush=True)
        out = sv.serve(reqs, cfg, int(a.budget_gb * 2 ** 30), on_round=_progress("serve"), deadline_s=a.deadline,
                       light_chi=a.light_chi)
        print("  sequential FP32 baseline", flush=True)
        base_cfg = dr.RunConfig(chi_max=cfg.chi_max, cutoff=cfg.cutoff, cutoff_mode=cfg.cutoff_mode,
                                precision="fp32", tau=cfg.tau, side=cfg.side, router=cfg.router)
        seq = sv.serve_sequential(reqs, base_cfg, deadline_s=a.deadline,
                                  on_request=lambda i, secs, ok: print(f"  [sequential] request {i}: {secs:.2f} s"
                                                                       f"{'' if ok else ' (deadline)'}", flush=True))
        print(json.dumps({"form": "serve", "rate": a.rate, "duration": a.duration, "requests": len(reqs), "side": a.side,
                          "router": a.router,
                          "chi_max": cfg.chi_max, "max_n": a.max_n,
                          "deadline_s": a.deadline, "tau": a.tau, "light_chi": a.light_chi,
                          "served": len(out["served"]), "timed_out": len(out["timed_out"]),
                          "refused": len(out["refused"]), "precision": prec, "seconds": round(out["seconds"], 3),
                          "circuits_per_s": round(out["circuits_per_s"], 4), "p50_time_to_peak_s": round(out["p50"], 3),
                          "p99_time_to_peak_s": round(out["p99"], 3), "all_peaks_ok": out["all_peaks_ok"],
                          "bond_updates": out["bond_updates"],
                          "peak_projected_gb": round(out["peak_projected_bytes"] / 2 ** 30, 3),
                          "peak_device_gb": round(out["peak_device_bytes"] / 2 ** 30, 3),
                          "sequential_fp32": {"seconds": round(seq["seconds"], 3),
                                              "circuits_per_s": round(seq["circuits_per_s"], 4),
                                              "p50_time_to_peak_s": round(seq["p50"], 3),
                                              "p99_time_to_peak_s": round(seq["p99"], 3),
                                              "finished": seq["finished"], "timed_out": seq["timed_out"],
                                              "all_peaks_ok": seq["all_peaks_ok"]}}), flush=True)


if __name__ == "__main__":
    main()
