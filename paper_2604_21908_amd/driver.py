"""Host driver of the middle-MPO contraction over libmpo (Alg. 1).

The driver owns only integer bookkeeping: layering, the midpoint split, the
order of the updates of one absorption step, layouts (rewiring) and lazy
routing.  Every tensor operation is a libmpo call.

Update order of one absorption step (the innermost layer of C_L, whose gates
act on the output legs, then the innermost layer of C_R, input legs):
  for each C_L gate in layer order: route it with output-side SWAPs moving the
  qubit on the lower site upwards; absorb it, together with the first not yet
  absorbed C_R gate of the step that already sits on the same bond;
  then route and absorb the remaining C_R gates with input-side SWAPs.
Updates on bonds at distance >= 2 commute exactly (they touch disjoint
tensors), so the ordered list is executed as waves of mutually distant bonds
through mpo_absorb_batch; the result equals the one-by-one execution.
"""
from __future__ import annotations

import dataclasses
import time
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import mpo as _mpo

SWAP = np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]], dtype=np.complex128)


@dataclasses.dataclass
class RunConfig:
    chi_max: int = 64
    cutoff: float = 1e-12
    cutoff_mode: str = "rel_sv"       # "rel_sv" | "weight"
    precision: str = "fp64"           # "fp64" | "fp32" | "mixed"
    tau: float = float("inf")
    unswap: str = "parallel"          # "parallel" | "sequential" | "none"
    relaxed: bool = False
    max_unswap_iters: int = 20
    waves: bool = True                # batch independent updates
    side: str = "both"                # "both" (Alg. 1), "adaptive" or "fixed" (App. A.3)
    fixed_freq: Tuple[int, int] = (1, 1)   # fixed mode: layers of C_L, then of C_R, per period
    rewire: str = "lazy"              # "lazy" routing per absorbed layer, or "eager" (Alg. 1: transpile,
                                      # strip transpilation SWAPs, reindex, re-transpile after unswapping)
    router: str = "up"                # routing of non-adjacent gates: "up" or "middle" (see route_bonds)


@dataclasses.dataclass
class Update:
    bond: int
    g_out: Optional[np.ndarray]
    g_in: Optional[np.ndarray]
    stage: str
    gids: Tuple[int, ...] = ()        # circuit gates this update absorbs (eager rewiring bookkeeping)


@dataclasses.dataclass
class RunResult:
    bits: np.ndarray
    prob: float
    norm2: float
    site_bits: np.ndarray
    out_layout: List[int]
    in_layout: List[int]
    trace: List[Dict]
    seconds: float
    bond_updates: int
    trial_updates: int


def time_layers(gates: Sequence[Tuple[int, int, np.ndarray]], n: int) -> List[list]:
    """Gates grouped into layers; a gate is placed right after the last layer
    that uses one of its wires."""
    front = np.zeros(n, dtype=np.int64)
    out: List[list] = []
    for q0, q1, u in gates:
        layer = int(max(front[q0], front[q1]))
        while len(out) <= layer:
            out.append([])
        out[layer].append((q0, q1, u))
        front[q0] = front[q1] = layer + 1
    return out


class Wires:
    """site_of[logical] and logical_at[site] of one side of the MPO."""

    def __init__(self, n: int):
        self.site_of = np.arange(n)
        self.logical_at = np.arange(n)

    def copy(self) -> "Wires":
        w = Wires.__new__(Wires)
        w.site_of = self.site_of.copy()
        w.logical_at = self.logical_at.copy()
        return w

    def exchange(self, bond: int) -> None:
        a, b = self.logical_at[bond], self.logical_at[bond + 1]
        self.logical_at[bond], self.logical_at[bond + 1] = b, a
        self.site_of[a] = bond + 1
        self.site_of[b] = bond


def _on_bond(u: np.ndarray, sa: int, sb: int) -> Tuple[int, np.ndarray]:
    if sb - sa == 1:
        return sa, u
    if sa - sb == 1:
        return sb, SWAP @ u @ SWAP
    raise ValueError("gate is not nearest-neighbour on the sites")


def _kind(g) -> Tuple[bool, Optional[int]]:
    """(is a transpilation SWAP, circuit gate id) of a layer entry: plain
    (a, b, u) circuit gates, or (a, b, u, is_swap, gid) from transpile()."""
    return (bool(g[3]), g[4]) if len(g) > 3 else (False, None)


def route_bonds(lo: int, hi: int, router: str = "up") -> List[int]:
    """Bonds of the SWAPs that make sites lo < hi neighbours, in order.
    "up": the qubit on the lower site climbs to hi - 1.  "middle": it climbs
    half the gap (rounded up), then the upper qubit descends the rest."""
    if router == "up":
        return list(range(lo, hi - 1))
    k = (hi - lo) // 2
    return list(range(lo, lo + k)) + list(range(hi - 1, lo + k, -1))


def plan_step(lgates, rgates, out_w: Wires, in_w: Wires, router: str = "up") -> List[Update]:
    """Ordered updates of one absorption step; routing changes the layouts.
    Entries flagged as transpilation SWAPs (eager rewiring) are absorbed as
    SWAP updates on their side and exchange the two sites in the layout."""
    ups: List[Update] = []

    def route(w: Wires, a: int, b: int, side: str):
        lo, hi = sorted((int(w.site_of[a]), int(w.site_of[b])))
        for j in route_bonds(lo, hi, router):
            ups.append(Update(j, SWAP if side == "L" else None, SWAP if side == "R" else None, "route"))
            w.exchange(j)

    def tswap(w: Wires, a: int, b: int, side: str):
        bond, _ = _on_bond(SWAP, int(w.site_of[a]), int(w.site_of[b]))
        ups.append(Update(bond, SWAP if side == "L" else None, SWAP if side == "R" else None, "route"))
        w.exchange(bond)

    waiting = list(rgates)
    for g in lgates:
        a, b, u = g[0], g[1], g[2]
        is_swap, gid = _kind(g)
        if is_swap:
            tswap(out_w, a, b, "L")
            continue
        route(out_w, a, b, "L")
        bond, gl = _on_bond(u, int(out_w.site_of[a]), int(out_w.site_of[b]))
        partner = None
        for j, rg in enumerate(waiting):
            if _kind(rg)[0]:
                continue
            sa, sb = int(in_w.site_of[rg[0]]), int(in_w.site_of[rg[1]])
            if abs(sa - sb) == 1 and min(sa, sb) == bond:
                partner = j
                break
        if partner is None:
            ups.append(Update(bond, gl, None, "absorb", (gid,) if gid is not None else ()))
        else:
            rg = waiting.pop(partner)
            _, gr = _on_bond(rg[2], int(in_w.site_of[rg[0]]), int(in_w.site_of[rg[1]]))
            rid = _kind(rg)[1]
            ups.append(Update(bond, gl, gr, "absorb", tuple(x for x in (gid, rid) if x is not None)))
    for g in waiting:
        a, b, u = g[0], g[1], g[2]
        is_swap, gid = _kind(g)
        if is_swap:
            tswap(in_w, a, b, "R")
            continue
        route(in_w, a, b, "R")
        bond, gr = _on_bond(u, int(in_w.site_of[a]), int(in_w.site_of[b]))
        ups.append(Update(bond, None, gr, "absorb", (gid,) if gid is not None else ()))
    return ups


def transpile(gates, w: Wires, router: str = "up") -> List[list]:
    """Alg. 1 "transpile to linear connectivity", for one half of the
    circuit from the layout `w` (not changed): the gates, in absorption order,
    each preceded by the SWAPs that bring its qubits next to each other (the
    qubit on the lower site moves up, as in lazy routing), then layered as
    soon as possible by the sites they touch.  Entries are
    (a, b, u, is_swap, gid) on logical qubits: a SWAP carries the two qubits
    it exchanges and gid None; a circuit gate its id."""
    w = w.copy()
    items = []
    for (a, b, u, gid) in gates:
        lo, hi = sorted((int(w.site_of[a]), int(w.site_of[b])))
        for j in route_bonds(lo, hi, router):
            items.append((j, (int(w.logical_at[j]), int(w.logical_at[j + 1]), SWAP, True, None)))
            w.exchange(j)
        items.append((min(int(w.site_of[a]), int(w.site_of[b])), (a, b, u, False, gid)))
    front = np.zeros(len(w.site_of) + 1, dtype=np.int64)
    layers: List[list] = []
    for lo, it in items:
        l = int(max(front[lo], front[lo + 1]))
        while len(layers) <= l:
            layers.append([])
        layers[l].append(it)
        front[lo] = front[lo + 1] = l + 1
    return layers


def wave_split(bonds: Sequence[int]) -> List[List[int]]:
    """Indices of `bonds` grouped into waves: an update goes one wave after the
    latest earlier update on a bond at distance <= 1."""
    last: Dict[int, int] = {}
    waves: List[List[int]] = []
    for idx, b in enumerate(bonds):
        w = 1 + max(last.get(b - 1, -1), last.get(b, -1), last.get(b + 1, -1))
        while len(waves) <= w:
            waves.append([])
        waves[w].append(idx)
        last[b] = w
    return waves


class Contractor:
    def __init__(self, circuit, cfg: RunConfig, stream=None):
        self.n = circuit.n
        self.cfg = cfg
        layers = time_layers(circuit.gates, self.n)
        cut = (len(layers) + 1) // 2
        self.c_left = layers[cut:]                     # innermost first
        self.c_right = layers[:cut][::-1]              # innermost first
        self.out_w = Wires(self.n)
        self.in_w = Wires(self.n)
        self.trace: List[Dict] = []
        self.bond_updates = 0
        mode = _mpo.CUT_REL_SV if cfg.cutoff_mode == "rel_sv" else _mpo.CUT_WEIGHT
        if np.isfinite(cfg.tau) and cfg.tau <= 0:
            raise ValueError("tau must be positive (or inf for no unswapping)")
        # size(M) is an integer, so size >= ceil(tau) exactly when size >= tau
        tau_elems = int(np.ceil(cfg.tau)) if np.isfinite(cfg.tau) else 0
        self._mk = lambda: _mpo.MPO(self.n, cfg.chi_max, cfg.cutoff, mode, _mpo.PRECISIONS[cfg.precision],
                                    stream=stream, tau_elems=tau_elems)
        self.m = self._mk()
        self.m2 = None                  # the second copy of adaptive side selection
        self.steps = 0
        self.trial_absorb_updates = 0
        self.gates_absorbed = 0
        self.sizes: List[Tuple[str, int, int]] = []
        if cfg.side not in ("both", "adaptive", "fixed"):
            raise ValueError(f"side must be both, adaptive or fixed, not {cfg.side!r}")
        if cfg.rewire not in ("lazy", "eager"):
            raise ValueError(f"rewire must be lazy or eager, not {cfg.rewire!r}")
        if cfg.rewire == "eager":
            # the halves as circuit gates with ids, in absorption order; the
            # absorption queues become their transpiled layers
            gid = 0
            self.gates_left, self.gates_right = [], []
            for dst, layers in ((self.gates_left, self.c_left), (self.gates_right, self.c_right)):
                for layer in layers:
                    for (a, b, u) in layer:
                        dst.append((a, b, u, gid))
                        gid += 1
            self.absorbed = set()
            self.retranspile()

    def close(self):
        self.m.close()
        if self.m2 is not None:
            self.m2.close()

    def _run_updates(self, m, ups: List[Update]) -> List[dict]:
        infos: List[Optional[dict]] = [None] * len(ups)
        if not ups:
            return infos
        if self.cfg.waves:
            for wave in wave_split([u.bond for u in ups]):
                res = m.absorb_batch([ups[i].bond for i in wave], [ups[i].g_out for i in wave],
                                     [ups[i].g_in for i in wave])
                for i, r in zip(wave, res):
                    infos[i] = r
        else:
            for i, u in enumerate(ups):
                infos[i] = m.absorb(u.bond, u.g_out, u.g_in)
        return infos

    def _execute(self, ups: List[Update]):
        if ups:
            self.record(ups, self._run_updates(self.m, ups))

    def plan_absorb(self) -> List[Update]:
        """Pops the innermost layer of each side and returns the ordered
        updates of that absorption step (layouts change by routing)."""
        lg = self.c_left.pop(0) if self.c_left else []
        rg = self.c_right.pop(0) if self.c_right else []
        return plan_step(lg, rg, self.out_w, self.in_w, self.cfg.router)

    def retranspile(self) -> None:
        """Rewiring of Alg. 1 in the eager mode: the circuit gates not yet
        absorbed (transpilation SWAPs stripped), on the current layouts (the
        accepted swaps reindex the qubits), transpiled again."""
        left = [g for g in self.gates_left if g[3] not in self.absorbed]
        right = [g for g in self.gates_right if g[3] not in self.absorbed]
        self.c_left = transpile(left, self.out_w, self.cfg.router)
        self.c_right = transpile(right, self.in_w, self.cfg.router)

    def record(self, ups: List[Update], infos: List[dict]) -> None:
        for u, r in zip(ups, infos):
            self.trace.append(dict(stage=u.stage, bond=u.bond, k=r["k"], discarded=r["discarded"],
                                   total=r["total"], sweeps=r["sweeps"]))
            if u.stage == "absorb":      # a fused update absorbs one gate of each half
                self.gates_absorbed += (u.g_out is not None) + (u.g_in is not None)
            if self.cfg.rewire == "eager":
                self.absorbed.update(u.gids)
        self.bond_updates += len(ups)

    def note_size(self, stage: str) -> None:
        """size(M) against the circuit gates absorbed so far (the sawtooth
        of Sec. III.A): one point after every absorption step and unswap stage."""
        self.sizes.append((stage, self.gates_absorbed, self.m.total_elements()))

    def step_candidates(self) -> List[Tuple[object, List[Update]]]:
        """The updates of the next absorption step under the configured side
        selection (App. A.3), as (MPO handle, ordered updates) pairs: one pair,
        or for an adaptive step two -- the next C_L layer on this MPO and the
        next C_R layer on a fresh copy of it.  Alg. 1's alternation takes a
        layer of each side; the fixed mode takes f_L layers of C_L, then f_R
        of C_R, in turn.  Once one side has no layers left, every mode takes
        the other.  step_commit() must follow with the updates' results."""
        mode = self.cfg.side
        if mode == "both" or not (self.c_left and self.c_right):
            self._pending = ("plain", "L" if self.c_left else "R", None)
            return [(self.m, self.plan_absorb())]
        if mode == "fixed":
            fl, fr = self.cfg.fixed_freq
            if self.steps % (fl + fr) < fl:
                self._pending = ("plain", "L", None)
                return [(self.m, plan_step(self.c_left.pop(0), [], self.out_w, self.in_w, self.cfg.router))]
            self._pending = ("plain", "R", None)
            return [(self.m, plan_step([], self.c_right.pop(0), self.out_w, self.in_w, self.cfg.router))]
        if self.m2 is None:
            self.m2 = self._mk()
        self.m2.copy_from(self.m)
        wl = (self.out_w.copy(), self.in_w.copy())
        ups_l = plan_step(self.c_left[0], [], *wl, self.cfg.router)
        wr = (self.out_w.copy(), self.in_w.copy())
        ups_r = plan_step([], self.c_right[0], *wr, self.cfg.router)
        self._pending = ("adaptive", None, (wl, wr))
        return [(self.m, ups_l), (self.m2, ups_r)]

    def step_commit(self, cands, infos) -> None:
        """Records the step planned by step_candidates(); an adaptive step
        keeps the copy with the smaller size(M) (equal: the left one), the
        other layer stays pending."""
        kind, taken, extra = self._pending
        self._pending = None
        if kind == "plain":
            self.record(cands[0][1], infos[0])
            if self.cfg.side == "fixed":
                self.trace.append(dict(stage="layer", taken=taken))
        else:
            (ups_l, ups_r), (inf_l, inf_r), (wl, wr) = (cands[0][1], cands[1][1]), infos, extra
            sl, sr = self.m.total_elements(), self.m2.total_elements()
            if sl <= sr:
                self.c_left.pop(0)
                self.out_w, self.in_w = wl
                self.record(ups_l, inf_l)
                self.trial_absorb_updates += len(ups_r)
            else:
                self.c_right.pop(0)
                self.out_w, self.in_w = wr
                self.m, self.m2 = self.m2, self.m
                self.record(ups_r, inf_r)
                self.trial_absorb_updates += len(ups_l)
            self.trace.append(dict(stage="side", side="L" if sl <= sr else "R", size_left=sl, size_right=sr))
        self.steps += 1

    def absorb_step(self):
        """One absorption step (step_candidates, the updates, step_commit)."""
        cands = self.step_candidates()
        self.step_commit(cands, [self._run_updates(m, ups) for m, ups in cands])

    def finish(self) -> RunResult:
        site_bits, p, n2 = self.m.extract_peak()
        bits = site_bits[self.out_w.site_of]
        return RunResult(bits.astype(np.uint8), p, n2, site_bits, list(map(int, self.out_w.site_of)),
                         list(map(int, self.in_w.site_of)), self.trace, 0.0, self.bond_updates,
                         self.m.counters()["trials"])

    def lambdas(self) -> List[np.ndarray]:
        return [self.m.singular_values(b) for b in range(self.n - 1)]

    def unswap(self):
        if self.cfg.unswap == "none":
            return []
        before = self.m.total_elements()
        log = self.m.unswap(self.cfg.unswap, self.cfg.relaxed, self.cfg.max_unswap_iters)
        self.record_unswap(log, before)
        return log

    def record_unswap(self, log, before: int) -> None:
        """Rewiring (Sec. II.B.2): fold the accepted swaps into the layouts."""
        for side, b in log:
            if side in ("L", "B"):
                self.out_w.exchange(b)
            if side in ("R", "B"):
                self.in_w.exchange(b)
        self.trace.append(dict(stage="unswap", accepted=len(log), size_before=before,
                               size=self.m.total_elements(), log=list(log)))
        if self.cfg.rewire == "eager":
            self.retranspile()

    def run(self) -> RunResult:
        t0 = time.perf_counter()
        while self.c_left or self.c_right:
            # at least one layer pair per phase (so the loop progresses when
            # unswapping cannot get below tau); with eager rewiring, until a
            # circuit gate is absorbed (leading layers of only transpilation
            # SWAPs would be unswapped and put back by rewiring, forever)
            before = self.gates_absorbed
            self.absorb_step()
            self.note_size("absorb")
            while self.cfg.rewire == "eager" and self.gates_absorbed == before and (self.c_left or self.c_right):
                self.absorb_step()
                self.note_size("absorb")
            while not self.m.tau_reached() and (self.c_left or self.c_right):
                self.absorb_step()
                self.note_size("absorb")
            self.unswap()
            self.note_size("unswap")
        site_bits, p, n2 = self.m.extract_peak()
        secs = time.perf_counter() - t0
        bits = site_bits[self.out_w.site_of]
        return RunResult(bits.astype(np.uint8), p, n2, site_bits, list(map(int, self.out_w.site_of)),
                         list(map(int, self.in_w.site_of)), self.trace, secs, self.bond_updates,
                         self.m.counters()["trials"])


def contract(circuit, cfg: RunConfig, stream=None) -> RunResult:
    c = Contractor(circuit, cfg, stream=stream)
    try:
        return c.run()
    finally:
        c.close()
