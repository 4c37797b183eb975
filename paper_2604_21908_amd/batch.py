"""Batched and served forms: many resident circuits advanced in lockstep.

Each circuit keeps its own device-resident MPO and follows Alg. 1 exactly as
alone (driver.Contractor: absorb at least one layer pair, keep absorbing while
size(M) < tau, unswap, repeat; then read the peak).  What changes is only how
the bond updates reach the GPU: in every round each circuit that is absorbing
contributes the ordered updates of its next absorption step; those are split
into waves of mutually distant bonds per circuit, the waves of all circuits are
merged, sorted by operand shape (chi_l, chi_r) and issued as group launches
(mpo_group_absorb, up to 32 updates per launch).  Circuits that reach their
unswapping stage in the same round run the parallel schedule together
(mpo_group_unswap: the trial and commit updates of one (side, parity) batch of
all of them share launches).  Per-update arithmetic is the same as alone, so
every circuit's result is identical to its lone run.
"""
from __future__ import annotations

import dataclasses
import time
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np

from . import driver as dr
from . import mpo as _mpo

GROUP_MAX = 32
UNSWAP = object()      # next_step(): the circuit waits for its unswapping stage


class CircuitTask:
    """Alg. 1 for one circuit as a resumable state machine."""

    def __init__(self, circuit, cfg: dr.RunConfig, tag=None, group_unswap: bool = False, keep_lams: bool = False):
        self.circuit = circuit
        self.cfg = cfg
        self.tag = tag
        self.keep_lams = keep_lams
        self.lams: Optional[List[np.ndarray]] = None
        self.group_unswap = group_unswap and cfg.unswap == "parallel"
        if cfg.rewire != "lazy":
            raise ValueError("the lockstep runner uses lazy rewiring")
        self.c = dr.Contractor(circuit, cfg)
        self.phase_started = False
        self.result: Optional[dr.RunResult] = None
        self.t_start = time.perf_counter()
        self.t_done: Optional[float] = None

    @property
    def done(self) -> bool:
        return self.result is not None

    def next_step(self):
        """(MPO handle, updates) candidates of the next absorption step (two
        for an adaptive step, Contractor.step_candidates); runs the unswap
        stage (or, with group unswapping, returns UNSWAP and waits for
        unswap_done) and the final readout when Alg. 1 reaches them.  None
        once finished."""
        c = self.c
        while True:
            if not (c.c_left or c.c_right):
                if self.phase_started:
                    if self.group_unswap:
                        return UNSWAP
                    c.unswap()
                    self.phase_started = False
                self.result = c.finish()
                self.t_done = time.perf_counter()
                if self.keep_lams:
                    self.lams = c.lambdas()
                c.close()
                return None
            if not self.phase_started:
                self.phase_started = True
                return c.step_candidates()
            if not c.m.tau_reached():
                return c.step_candidates()
            if self.group_unswap:
                return UNSWAP
            c.unswap()
            self.phase_started = False

    def unswap_done(self, log, before: int) -> None:
        self.c.record_unswap(log, before)
        self.phase_started = False

    def shape(self, bond: int):
        dims = self.c.m.bond_dims()
        return (1 if bond == 0 else dims[bond - 1], dims[bond + 1] if bond + 1 < len(dims) else 1)


def run_round(tasks: Sequence[CircuitTask], group: Optional[_mpo.Group], per_update: bool = False) -> int:
    """Advances every unfinished task by one absorption step; returns the
    number of bond updates issued."""
    steps = []
    pend = []
    for t in tasks:
        if t.done:
            continue
        ups = t.next_step()
        if ups is UNSWAP:
            pend.append(t)
        elif ups:
            steps.append((t, ups))
    if pend and per_update:
        # the same stage, each circuit's sweep launched on its own
        for t in pend:
            before = t.c.m.total_elements()
            log = t.c.m.unswap(t.cfg.unswap, t.cfg.relaxed, t.cfg.max_unswap_iters)
            t.unswap_done(log, before)
    elif pend:
        by_opts: Dict[tuple, list] = {}
        for t in pend:
            by_opts.setdefault((t.cfg.relaxed, t.cfg.max_unswap_iters), []).append(t)
        for (relaxed, iters), ts in by_opts.items():
            before = [t.c.m.total_elements() for t in ts]
            logs = group.unswap([t.c.m for t in ts], relaxed, iters)
            for t, log, b0 in zip(ts, logs, before):
                t.unswap_done(log, b0)
    issued = 0
    if per_update:
        for t, cands in steps:
            infos = [[m.absorb(u.bond, u.g_out, u.g_in) for u in ups] for m, ups in cands]
            t.c.step_commit(cands, infos)
            issued += sum(len(ups) for m, ups in cands)
        return issued
    # merge the waves of every candidate of every circuit, shape-sorted, into
    # group launches (the candidates of an adaptive step act on different MPOs)
    results = {(id(t), c): [None] * len(ups) for t, cands in steps for c, (m, ups) in enumerate(cands)}
    waves: List[list] = []
    for t, cands in steps:
        for c, (m, ups) in enumerate(cands):
            dims = m.bond_dims()
            for w, idxs in enumerate(dr.wave_split([u.bond for u in ups])):
                while len(waves) <= w:
                    waves.append([])
                for i in idxs:
                    b = ups[i].bond
                    key = (1 if b == 0 else dims[b - 1], dims[b + 1] if b + 1 < len(dims) else 1)
                    waves[w].append((key, (id(t), c), m, ups[i], i))
    for wave in waves:
        wave.sort(key=lambda x: x[0])
        for j in range(0, len(wave), GROUP_MAX):
            chunk = wave[j:j + GROUP_MAX]
            infos = group.absorb([x[2] for x in chunk], [x[3].bond for x in chunk], [x[3].g_out for x in chunk],
                                 [x[3].g_in for x in chunk])
            for (key, rk, m, u, i), inf in zip(chunk, infos):
                results[rk][i] = inf
            issued += len(chunk)
    for t, cands in steps:
        t.c.step_commit(cands, [results[(id(t), c)] for c in range(len(cands))])
    return issued


def run_batched(circuits_cfgs, precision: str = "fp32", per_update: bool = False, keep_lams: bool = False,
                max_rounds: int = 0) -> dict:
    """Contracts (circuit, RunConfig) pairs in lockstep; returns results and
    aggregate throughput (with keep_lams, also every circuit's final bond
    vectors, read after its peak readout).  With max_rounds > 0 it stops after
    that many rounds (the same work in the grouped and the per-update way);
    unfinished circuits have result None."""
    group = None if per_update else _mpo.Group(_mpo.PRECISIONS[precision])
    t0 = time.perf_counter()
    # both ways take the unswapping stage as a round of its own (the grouped
    # way batches it across circuits), so a round is the same work in both
    tasks = [CircuitTask(c, cfg, tag=i, group_unswap=True, keep_lams=keep_lams)
             for i, (c, cfg) in enumerate(circuits_cfgs)]
    updates = 0
    rounds = 0
    while not all(t.done for t in tasks) and not (max_rounds and rounds >= max_rounds):
        updates += run_round(tasks, group, per_update)
        rounds += 1
    secs = time.perf_counter() - t0
    for t in tasks:
        if not t.done:
            t.c.close()
    if group is not None:
        group.close()
    return dict(results=[t.result for t in tasks], seconds=secs, bond_updates=updates, rounds=rounds,
                updates_per_s=updates / secs if secs > 0 else 0.0, lams=[getattr(t, "lams", None) for t in tasks],
                finished=sum(1 for t in tasks if t.done))
