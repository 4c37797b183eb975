"""Served form: continuous batching of circuit requests on one GPU.

Requests arrive over time (e.g. Poisson).  A request is admitted when a slot
is free and its projected MPO memory n * chi_max^2 * 16 B fits in what the
admitted requests leave of the budget; admitted circuits stay resident on the
device.  Every scheduling round advances resident circuits by one absorption
step through shared group launches (batch.run_round): all the light ones
(small bond dimensions), and in every few rounds the earliest-arrived heavy
one (pick_round), so
requests that arrive while others are on the GPU join the running batch at
the next round and their work overlaps on the device.  A finished circuit releases its
slot and memory at once.  Time-to-peak is measured from arrival to the end of
its peak readout.
"""
from __future__ import annotations

import dataclasses
import time
from typing import Callable, List, Optional, Sequence

import numpy as np

from . import batch as bt
from . import circuitgen as cg
from . import driver as dr
from . import mpo as _mpo


@dataclasses.dataclass
class Request:
    t_arrival: float
    n: int
    depth: int
    seed: int
    circuit: Optional[cg.Circuit] = None     # built before serving starts (host memory)


def prepare(requests: Sequence[Request], reading: str = "A") -> None:
    """Builds every request's circuit up front: a circuit is already in host
    memory when it arrives, so generation is not part of its time-to-peak."""
    for r in requests:
        if r.circuit is None:
            r.circuit = cg.mirrored_peaked_circuit(r.n, r.depth, r.seed, reading=reading)


def admit(pending: Sequence[Request], used_bytes: int, budget_bytes: int, free_slots: int, chi_max: int):
    """First-come-first-served admission by projected memory: the head of the
    queue is admitted while a slot is free and its n chi_max^2 16 B fits in
    what the resident requests leave of the budget; a request that could not
    fit even alone is refused.  Returns (admitted, refused, still_waiting)."""
    admitted, refused, waiting = [], [], []
    used = used_bytes
    blocked = False
    for r in pending:
        need = projected_bytes(r.n, chi_max)
        if need > budget_bytes:
            refused.append(r)
            continue
        if not blocked and len(admitted) < free_slots and used + need <= budget_bytes:
            admitted.append(r)
            used += need
        else:
            blocked = True          # no overtaking: later requests wait behind the head
            waiting.append(r)
    return admitted, refused, waiting


@dataclasses.dataclass
class Served:
    request: Request
    t_admit: float
    t_done: float
    bits_ok: bool
    prob: float
    updates: int
    bits: Optional[np.ndarray] = None
    lams: Optional[list] = None

    @property
    def time_to_peak(self) -> float:
        return self.t_done - self.request.t_arrival


def projected_bytes(n: int, chi_max: int) -> int:
    return n * chi_max * chi_max * 16


def _device_used_bytes(torch) -> int:
    free, total = torch.cuda.mem_get_info()
    return int(total - free)


def _percentiles(ttp: Sequence[float]):
    ttp = np.asarray(ttp, dtype=np.float64) if len(ttp) else np.zeros(1)
    return float(np.percentile(ttp, 50)), float(np.percentile(ttp, 99))


def pick_round(active: Sequence[tuple], light_chi: int, round_no: int = 0, heavy_every: int = 4) -> List[tuple]:
    """The resident circuits a round advances.  A step costs about the cube
    of the MPO's bond dimensions, so circuits whose largest bond is at most
    `light_chi` ("light") all take a step in every round, sharing the group
    launches, while of the heavier ones only the earliest arrival does, and
    only in every `heavy_every`-th round while light ones are resident: the
    light requests (the short jobs) are not held back by the steps of the
    heavy ones, and the heavy ones are served one after the other, as a
    single queue would.  light_chi <= 0 advances every resident circuit
    (plain lockstep)."""
    if light_chi <= 0:
        return list(active)
    light, heavy = [], []
    for a in active:
        c = a[1].c
        # an adaptive step also absorbs into a copy: the last discarded
        # candidate (held in m2) tells what that costs
        chi = max(max(c.m.bond_dims()), max(c.m2.bond_dims()) if c.m2 is not None else 1)
        (light if chi <= light_chi else heavy).append(a)
    if heavy and (not light or round_no % max(1, heavy_every) == 0):
        light.append(min(heavy, key=lambda a: a[0].t_arrival))
    return light


def serve(requests: Sequence[Request], cfg: dr.RunConfig, budget_bytes: int, max_slots: int = 64,
          reading: str = "A", on_round: Optional[Callable[[int, int], None]] = None,
          keep_lams: bool = False, deadline_s: float = 0.0, light_chi: int = 64) -> dict:
    """Serves `requests` (see the module docstring; `light_chi` is the round
    policy of pick_round).  With `deadline_s` > 0 a request still resident
    that long after its arrival is cancelled (its MPO freed at once) and
    reported in `timed_out`; the percentiles then count it at the deadline,
    so they are lower bounds when any timed out."""
    import torch
    reqs = sorted(requests, key=lambda r: r.t_arrival)
    prepare(reqs, reading)
    group = _mpo.Group(_mpo.PRECISIONS[cfg.precision])
    pending: List[Request] = []
    active: List[tuple] = []
    done: List[Served] = []
    refused: List[Request] = []
    timed_out: List[Request] = []
    used = 0
    peak_used = 0
    torch.cuda.synchronize()
    dev0 = _device_used_bytes(torch)
    dev_peak = 0
    i = 0
    rounds = 0
    t0 = time.perf_counter()
    while i < len(reqs) or pending or active:
        now = time.perf_counter() - t0
        while i < len(reqs) and reqs[i].t_arrival <= now:
            pending.append(reqs[i])
            i += 1
        adm, ref, pending = admit(pending, used, budget_bytes, max_slots - len(active), cfg.chi_max)
        refused += ref
        for r in adm:
            need = projected_bytes(r.n, cfg.chi_max)
            task = bt.CircuitTask(r.circuit, cfg, group_unswap=True, keep_lams=keep_lams)
            active.append((r, task, time.perf_counter() - t0, need))
            used += need
            peak_used = max(peak_used, used)
        if not active:
            if i < len(reqs):
                time.sleep(max(0.0, min(0.05, reqs[i].t_arrival - (time.perf_counter() - t0))))
            continue
        bt.run_round([a[1] for a in pick_round(active, light_chi, rounds)], group)
        rounds += 1
        dev_peak = max(dev_peak, _device_used_bytes(torch) - dev0)
        if on_round:
            on_round(rounds, len(active))
        still = []
        now = time.perf_counter() - t0
        for (r, task, t_adm, need) in active:
            if task.done:
                res = task.result
                done.append(Served(r, t_adm, task.t_done - t0, bool((res.bits == task.circuit.peak).all()),
                                   float(res.prob), res.bond_updates, res.bits, task.lams))
                used -= need
            elif deadline_s > 0 and now - r.t_arrival > deadline_s:
                task.c.close()
                timed_out.append(r)
                used -= need
            else:
                still.append((r, task, t_adm, need))
        active = still
    secs = time.perf_counter() - t0
    group.close()
    p50, p99 = _percentiles([d.time_to_peak for d in done] + [deadline_s] * len(timed_out))
    return dict(served=done, refused=refused, timed_out=timed_out, seconds=secs, rounds=rounds,
                circuits_per_s=len(done) / secs if secs else 0.0, p50=p50, p99=p99,
                all_peaks_ok=all(d.bits_ok for d in done), peak_projected_bytes=peak_used,
                peak_device_bytes=dev_peak, bond_updates=sum(d.updates for d in done))


def poisson_requests(rate: float, duration: float, seed: int = 4000, sizes=(24, 40, 56),
                     probs=(0.5, 0.3, 0.2)) -> List[Request]:
    """Arrivals of the serving workload: exponential gaps at `rate`/s over
    `duration` s; n drawn from `sizes` with `probs`; depth n/4."""
    rng = np.random.Generator(np.random.PCG64(seed + int(rate * 1000)))
    t = 0.0
    out = []
    k = 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        n = int(rng.choice(list(sizes), p=list(probs)))
        out.append(Request(t, n, max(1, n // 4), seed + 17 * k + 1))
        k += 1
    return out


class _Deadline(Exception):
    pass


def _contract_within(circ, cfg: dr.RunConfig, limit_s: float):
    """dr.contract with a limit on the wall time (checked before every
    absorption step); None when the limit is reached."""
    c = dr.Contractor(circ, cfg)
    t0 = time.perf_counter()
    if limit_s > 0:
        step = c.absorb_step

        def bounded():
            if time.perf_counter() - t0 > limit_s:
                raise _Deadline()
            step()
        c.absorb_step = bounded
    try:
        return c.run()
    except _Deadline:
        return None
    finally:
        c.close()


def serve_sequential(requests: Sequence[Request], cfg: dr.RunConfig, reading: str = "A",
                     deadline_s: float = 0.0, on_request: Optional[Callable[[int, float, bool], None]] = None) -> dict:
    """Baseline for the served form: the same arrivals handled one circuit at
    a time, first come first served, each contracted alone with one launch per
    update wave.  The solo service time of every circuit is measured; the
    queue is then exact for a single server: a request starts when it has
    arrived and the previous one has finished.  With `deadline_s` > 0 the
    deadline counts from arrival, as in serve(): a request is served for at
    most what is left of it when it starts (none if nothing is left) and is
    counted at the deadline when it does not finish."""
    reqs = sorted(requests, key=lambda r: r.t_arrival)
    prepare(reqs, reading)
    service = []
    solo_done = []
    ok = []
    updates = 0
    for r in reqs:
        circ = r.circuit
        t0 = time.perf_counter()
        res = _contract_within(circ, cfg, deadline_s)
        service.append(time.perf_counter() - t0)
        solo_done.append(res is not None)
        if on_request:
            on_request(len(service), service[-1], res is not None)
        if res is not None:
            ok.append(bool((res.bits == circ.peak).all()))
            updates += res.bond_updates
    done = []
    t_free = 0.0
    finished = 0
    for r, s, res_ok in zip(reqs, service, solo_done):
        start = max(r.t_arrival, t_free)
        left = deadline_s - (start - r.t_arrival) if deadline_s > 0 else float("inf")
        if left <= 0:
            done.append(deadline_s)           # expired while waiting
            continue
        if res_ok and s <= left:
            t_free = start + s
            done.append(t_free - r.t_arrival)
            finished += 1
        else:
            t_free = start + min(s, left)
            done.append(deadline_s)
    makespan = t_free if reqs else 0.0
    p50, p99 = _percentiles(done)
    return dict(seconds=makespan, circuits_per_s=finished / makespan if makespan else 0.0,
                p50=p50, p99=p99, finished=finished, timed_out=len(reqs) - finished,
                all_peaks_ok=all(ok), bond_updates=updates, service_s=service)
