"""CPU oracle of the middle-MPO contraction -- TEST INFRASTRUCTURE ONLY.

Only tests, the smoke check and the benchmark's CPU-baseline leg may import
this module.  It is a plain, slow, complex128 NumPy implementation written
from the paper's statement of the method, and it shares no code with the GPU
path (it imports nothing from the product package; circuits reach it as
plain gate lists).

What it follows:
* Alg. 1 (MPO iterative cancellation with unswapping): split at the temporal
  midpoint, identity MPO, absorb innermost layers from both sides while the
  MPO size is below tau, then unswap, then rewire, until no layers remain;
  finally apply the MPO to |0...0>.
* Sec. II.B.1 (absorption): each two-qubit gate next to the MPO is contracted
  with the two site tensors, followed by an SVD with a singular-value cutoff
  and a bond-dimension cap (App. A.4).
* Sec. II.B.2 and Eq. (1) (unswapping): greedy SWAP trials from the left,
  the right or both sides on the largest available bond, accepted only when
  they lower that bond's dimension; M = P_L M~ P_R.
* App. A.1 (parallel swap selection) and A.2 (relaxed acceptance).
* Sec. II.B.3 (rewiring): the accepted swaps relabel the remaining circuits.
  The workload circuits are nearest-neighbour from the start, so "strip the
  transpilation SWAPs" is empty; the relabelling is held as layout maps and
  re-routing to the line is done lazily by SWAPs absorbed on the same side.
* Sec. II.C (sampling): the MPO applied to |0...0> is an MPS; the peak is
  read out by a greedy left-to-right conditional argmax.
* App. A.3 (side selection): besides Alg. 1's alternation (a layer of C_L,
  then a layer of C_R, per absorption step), an adaptive mode that absorbs
  the next layer of each side into its own copy of the MPO and keeps the
  copy with the smaller size(M), and a fixed-frequency mode that takes f_L
  layers of C_L, then f_R layers of C_R, in turn.

Representation: site i is B_i[a, s, b] with s = 2*o + p (o output bit,
p input bit); the MPO is kept as a vectorised MPS in Vidal/Hastings form:
right-canonical B_i plus bond vectors lam_i (operator-Schmidt values).  The
identity MPO has B_i = (1, 0, 0, 1)/sqrt(2), so |vec(M)| = 1.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

SQRT_HALF = np.sqrt(0.5)
SWAP4 = np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]], dtype=np.complex128)

# bond-weight ties in the choice among L/R/B trials are resolved by side order
# when the discarded weights differ by less than this (relative to sum s^2)
WEIGHT_TIE_REL = 1e-9


# --------------------------------------------------------------------------
# truncation rule (Sec. II.B.1; App. A.4 "SVD cutoff", "maximum bond dimension")
# --------------------------------------------------------------------------
def truncation_rank(s: np.ndarray, chi_max: int, cutoff: float, mode: str) -> int:
    """Number of singular values kept.

    mode "rel_sv": keep s_j > cutoff * s_0.
    mode "weight": smallest k with sum_{j>=k} s_j^2 <= cutoff * sum_j s_j^2.
    Then k <- min(k, chi_max) and k >= 1.  ``s`` is sorted descending.
    """
    s = np.asarray(s, dtype=np.float64)
    if s.size == 0:
        return 1
    if mode == "rel_sv":
        k = int(np.count_nonzero(s > cutoff * s[0]))
    elif mode == "weight":
        sq = s * s
        total = float(np.sum(sq))
        # tail[k] = sum_{j>=k} s_j^2, accumulated from the smallest value
        tail = np.concatenate([np.cumsum(sq[::-1])[::-1], [0.0]])
        k = int(np.argmax(tail <= cutoff * total))
    else:
        raise ValueError(mode)
    return max(1, min(k, chi_max, s.size))


# --------------------------------------------------------------------------
# the MPO (Alg. 1 "Initialize MPO M <- I^{(x)N}")
# --------------------------------------------------------------------------
class OracleMPO:
    def __init__(self, n: int):
        if n < 2:
            raise ValueError("n >= 2")
        self.n = n
        w = np.zeros((1, 4, 1), dtype=np.complex128)
        w[0, 0, 0] = SQRT_HALF      # o=0, p=0
        w[0, 3, 0] = SQRT_HALF      # o=1, p=1
        self.B = [w.copy() for _ in range(n)]
        self.lam = [np.ones(1) for _ in range(n - 1)]

    def copy(self) -> "OracleMPO":
        m = OracleMPO.__new__(OracleMPO)
        m.n = self.n
        m.B = [b.copy() for b in self.B]
        m.lam = [l.copy() for l in self.lam]
        return m

    def chi(self, i: int) -> int:
        return int(self.lam[i].size)

    def bond_dims(self) -> List[int]:
        return [self.chi(i) for i in range(self.n - 1)]

    def size(self) -> int:
        """size(M): total number of MPO tensor elements (Alg. 1, Sec. II.B.1)."""
        return int(sum(b.size for b in self.B))

    # ------------------------------------------------------------ dense view
    def dense_vector(self) -> np.ndarray:
        """Full contraction of the vectorised MPO, axes (s_0, ..., s_{n-1})."""
        t = self.B[0][0]                      # (4, chi_0)
        for i in range(1, self.n):
            t = np.tensordot(t, self.B[i], axes=([t.ndim - 1], [0]))
        return t[..., 0]

    def dense_operator(self) -> np.ndarray:
        """2^n x 2^n matrix of the (normalised) operator, rows = outputs in
        site order, columns = inputs in site order, site 0 most significant."""
        n = self.n
        v = self.dense_vector().reshape([2, 2] * n)          # o0 p0 o1 p1 ...
        v = v.transpose(list(range(0, 2 * n, 2)) + list(range(1, 2 * n, 2)))
        return v.reshape(2 ** n, 2 ** n)


# --------------------------------------------------------------------------
# two-site update (Sec. II.B.1; Vidal/Hastings form)
# --------------------------------------------------------------------------
@dataclasses.dataclass
class UpdateResult:
    bond: int
    k: int
    s: np.ndarray              # all singular values, descending
    discarded: float           # sum of the dropped s_j^2 (absolute)
    total: float               # sum of all s_j^2
    new_left: Optional[np.ndarray] = None
    new_right: Optional[np.ndarray] = None


def apply_gates_to_theta(theta: np.ndarray, g_out: Optional[np.ndarray],
                         g_in: Optional[np.ndarray]) -> np.ndarray:
    """theta[a, s1, s2, b] -> gate pair applied on the physical legs.

    g_out acts on the output legs (M <- G M):  o' = G o.
    g_in  acts on the input legs  (M <- M G):  p' = sum_p p G[p, p'].
    Both are 4x4 in the basis |q_i q_{i+1}>, site i most significant.
    """
    a, _, _, b = theta.shape
    t = theta.reshape(a, 2, 2, 2, 2, b)          # a o1 p1 o2 p2 b
    if g_out is not None:
        g = np.asarray(g_out, dtype=np.complex128).reshape(2, 2, 2, 2)   # o1' o2' o1 o2
        t = np.einsum("xyuv,aupvqb->axpyqb", g, t)
    if g_in is not None:
        g = np.asarray(g_in, dtype=np.complex128).reshape(2, 2, 2, 2)    # p1 p2 p1' p2'
        t = np.einsum("aoxpyb,xyuv->aoupvb", t, g)
    return t.reshape(a, 4, 4, b)


def bond_update(m: OracleMPO, i: int, g_out: Optional[np.ndarray], g_in: Optional[np.ndarray],
                chi_max: int, cutoff: float, mode: str, vectors: bool = True) -> UpdateResult:
    """One bond update at (i, i+1): theta = (G_out (x) G_in^T) Lam_{i-1} B_i B_{i+1},
    SVD, truncation; with ``vectors`` the new site tensors are returned
    (B_{i+1}' = V_k^dag, B_i' = theta_noLam V_k) but nothing is written to ``m``."""
    bl, br = m.B[i], m.B[i + 1]
    chil, chir = bl.shape[0], br.shape[2]
    theta_nolam = np.tensordot(bl, br, axes=([2], [0]))                 # a s1 s2 b
    theta_nolam = apply_gates_to_theta(theta_nolam, g_out, g_in)
    lam_left = m.lam[i - 1] if i > 0 else np.ones(1)
    theta = theta_nolam * lam_left[:, None, None, None]
    mat = theta.reshape(chil * 4, 4 * chir)
    try:
        if vectors:
            _, s, vh = np.linalg.svd(mat, full_matrices=False)
        else:
            s = np.linalg.svd(mat, compute_uv=False)
    except np.linalg.LinAlgError:
        # LAPACK's divide-and-conquer driver occasionally fails to converge;
        # the QR-iteration driver computes the same decomposition
        import scipy.linalg
        _, s, vh = scipy.linalg.svd(mat, full_matrices=False, lapack_driver="gesvd")
    k = truncation_rank(s, chi_max, cutoff, mode)
    sq = s * s
    res = UpdateResult(bond=i, k=k, s=s, discarded=float(np.sum(sq[k:])), total=float(np.sum(sq)))
    if vectors:
        vk = vh[:k]                                                     # k x 4chir
        res.new_right = vk.reshape(k, 4, chir)
        res.new_left = (theta_nolam.reshape(chil * 4, 4 * chir) @ vk.conj().T).reshape(chil, 4, k)
    return res


def commit(m: OracleMPO, res: UpdateResult) -> None:
    i = res.bond
    m.B[i] = res.new_left
    m.B[i + 1] = res.new_right
    m.lam[i] = res.s[:res.k].copy()


# --------------------------------------------------------------------------
# peak extraction (Alg. 1 "apply M to |0>"; Sec. II.C)
# --------------------------------------------------------------------------
def extract_peak(m: OracleMPO) -> Tuple[np.ndarray, float, float]:
    """Greedy conditional argmax of |<x|M|0...0>|^2 over site bits.

    A_i[a, o, b] = B_i[a, 2o + 0, b] (input leg projected on |0>).  Right
    environments E_i = sum_o A_o E_{i+1} A_o^dag are exact; from the left the
    bit with the larger conditional weight is taken (ties -> 0).  Returns
    (site bits, p = prod of conditionals, <psi|psi>)."""
    n = m.n
    A = [m.B[i][:, 0::2, :] for i in range(n)]          # s = 0 (o=0,p=0), s = 2 (o=1,p=0)
    env = [None] * (n + 1)
    env[n] = np.ones((1, 1), dtype=np.complex128)
    for i in range(n - 1, -1, -1):
        e = np.zeros((A[i].shape[0], A[i].shape[0]), dtype=np.complex128)
        for o in range(2):
            ao = A[i][:, o, :]
            e += ao @ env[i + 1] @ ao.conj().T
        env[i] = e
    norm2 = float(env[0][0, 0].real)
    v = np.ones((1,), dtype=np.complex128)
    bits = np.zeros(n, dtype=np.uint8)
    logp = 0.0
    for i in range(n):
        w = [v @ A[i][:, o, :] for o in range(2)]
        p = [float((w[o] @ env[i + 1] @ w[o].conj()).real) for o in range(2)]
        o = 1 if p[1] > p[0] else 0
        bits[i] = o
        logp += np.log(p[o] / (p[0] + p[1]))
        v = w[o] / np.linalg.norm(w[o])
    return bits, float(np.exp(logp)), norm2


def sample(m: OracleMPO, uniforms: np.ndarray, with_q: bool = False):
    """Sec. II.C sampling of M|0...0>: one sample per row of ``uniforms``
    (shape count x n, values in [0, 1)).  From the left, site i's bit is 0
    when u_i < P(0 | bits so far) = p_0 / (p_0 + p_1), with
    p_o = w_o E_{i+1} w_o^dag, w_o = v A_i[:, o, :] and v the normalised left
    vector of the bits chosen so far; E are the exact right environments of
    extract_peak.  Returns (site bits, count x n; probability of each sampled
    string, the product of its conditionals) and, with ``with_q``, the
    thresholds P(0 | prefix) each decision compared u_i with (count x n)."""
    n = m.n
    u = np.asarray(uniforms, dtype=np.float64)
    A = [m.B[i][:, 0::2, :] for i in range(n)]
    env = [None] * (n + 1)
    env[n] = np.ones((1, 1), dtype=np.complex128)
    for i in range(n - 1, -1, -1):
        env[i] = sum(A[i][:, o, :] @ env[i + 1] @ A[i][:, o, :].conj().T for o in range(2))
    bits = np.zeros(u.shape, dtype=np.uint8)
    probs = np.zeros(u.shape[0])
    qs = np.zeros(u.shape)
    for s in range(u.shape[0]):
        v = np.ones((1,), dtype=np.complex128)
        logp = 0.0
        for i in range(n):
            w = [v @ A[i][:, o, :] for o in range(2)]
            p = [float((w[o] @ env[i + 1] @ w[o].conj()).real) for o in range(2)]
            qs[s, i] = p[0] / (p[0] + p[1])
            o = 0 if u[s, i] < qs[s, i] else 1
            bits[s, i] = o
            logp += np.log(p[o] / (p[0] + p[1]))
            v = w[o] / np.sqrt(p[o])
        probs[s] = np.exp(logp)
    return (bits, probs, qs) if with_q else (bits, probs)


# --------------------------------------------------------------------------
# unswapping (Sec. II.B.2, Eq. (1); App. A.1, A.2)
# --------------------------------------------------------------------------
SIDES = ("L", "R", "B")


def swap_gates(side: str):
    return (SWAP4 if side in ("L", "B") else None, SWAP4 if side in ("R", "B") else None)


def unswap_sequential(m: OracleMPO, cfg: "OracleConfig") -> List[Tuple[str, int]]:
    """Alg. 1 unswapping block: pick the available bond with the largest
    dimension (ties -> smallest index), try a SWAP from the left, the right and
    both sides, accept the best if it lowers that bond (relaxed: does not raise
    it), then retire the bond and re-enable its neighbours; a rejected bond is
    only retired.  The best trial has the smallest k, then the smaller
    discarded weight, then the order L, R, B."""
    n = m.n
    avail = set(range(n - 1))
    log: List[Tuple[str, int]] = []
    cap = cfg.max_unswap_iters * (n - 1)
    while avail and len(log) < cap:
        i = max(sorted(avail), key=lambda j: (m.chi(j), -j))
        chi_i = m.chi(i)
        best = None
        for side in SIDES:
            go, gi = swap_gates(side)
            r = bond_update(m, i, go, gi, cfg.chi_max, cfg.cutoff, cfg.mode, vectors=True)
            if best is None:
                best = (side, r)
                continue
            rb = best[1]
            tol = WEIGHT_TIE_REL * max(r.total, rb.total)
            if r.k < rb.k or (r.k == rb.k and r.discarded < rb.discarded - tol):
                best = (side, r)
        side, r = best
        ok = r.k < chi_i or (cfg.relaxed and r.k == chi_i)
        avail.discard(i)
        if ok:
            commit(m, r)
            log.append((side, i))
            if i - 1 >= 0:
                avail.add(i - 1)
            if i + 1 <= n - 2:
                avail.add(i + 1)
    return log


PARALLEL_ORDER = (("B", 0), ("B", 1), ("L", 0), ("L", 1), ("R", 0), ("R", 1))


def unswap_parallel(m: OracleMPO, cfg: "OracleConfig") -> List[Tuple[str, int]]:
    """App. A.1: cycle through (side, parity) in the order both-even, both-odd,
    left-even, left-odd, right-even, right-odd; in each batch every bond of that
    parity gets an independent SWAP trial (the bonds are disjoint) and keeps it
    only if it lowers (relaxed: does not raise) its bond.  Stop after a full
    cycle without a strict reduction, or after ``max_unswap_iters`` cycles."""
    n = m.n
    log: List[Tuple[str, int]] = []
    for _cycle in range(cfg.max_unswap_iters):
        reduced = False
        for side, parity in PARALLEL_ORDER:
            go, gi = swap_gates(side)
            results = []
            for i in range(parity, n - 1, 2):
                results.append((i, m.chi(i), bond_update(m, i, go, gi, cfg.chi_max, cfg.cutoff,
                                                         cfg.mode, vectors=True)))
            for i, chi_i, r in results:
                if r.k < chi_i or (cfg.relaxed and r.k == chi_i):
                    commit(m, r)
                    log.append((side, i))
                    if r.k < chi_i:
                        reduced = True
        if not reduced:
            break
    return log


# --------------------------------------------------------------------------
# circuit side: layers, split, layouts, routing (Alg. 1 split; Sec. II.B.3)
# --------------------------------------------------------------------------
def asap_layers(gates: Sequence[Tuple[int, int, np.ndarray]], n: int) -> List[list]:
    """As-soon-as-possible layering: a gate goes one layer after the latest
    gate on either of its wires."""
    depth = [0] * n
    layers: List[list] = []
    for q0, q1, u in gates:
        l = max(depth[q0], depth[q1])
        if l == len(layers):
            layers.append([])
        layers[l].append((q0, q1, u))
        depth[q0] = depth[q1] = l + 1
    return layers


@dataclasses.dataclass
class OracleConfig:
    chi_max: int = 64
    cutoff: float = 1e-12
    mode: str = "rel_sv"            # "rel_sv" or "weight"
    tau: float = float("inf")       # size(M) threshold that triggers unswapping
    unswap: str = "parallel"        # "parallel" (App. A.1), "sequential" (Alg. 1) or "none"
    relaxed: bool = False           # App. A.2
    max_unswap_iters: int = 20      # App. A.4
    side: str = "both"              # "both" (Alg. 1), "adaptive" or "fixed" (App. A.3)
    fixed_freq: Tuple[int, int] = (1, 1)   # fixed mode: layers of C_L, then of C_R, per period
    rewire: str = "lazy"            # "lazy" or "eager" (Alg. 1 / Sec. II.B.3 taken literally)
    router: str = "up"              # "up": the lower qubit climbs; "middle": both meet halfway


class Layout:
    """Site <-> logical-qubit maps of one side of the MPO."""

    def __init__(self, n: int):
        self.site_of = list(range(n))      # logical -> site
        self.logical_at = list(range(n))   # site -> logical

    def swap_sites(self, i: int) -> None:
        a, b = self.logical_at[i], self.logical_at[i + 1]
        self.logical_at[i], self.logical_at[i + 1] = b, a
        self.site_of[a], self.site_of[b] = i + 1, i


def orient(u: np.ndarray, sa: int, sb: int) -> Tuple[int, np.ndarray]:
    """Bond index and 4x4 matrix in the (site i, site i+1) basis of a gate whose
    first logical qubit sits at site sa and second at sb = sa +- 1."""
    if sb == sa + 1:
        return sa, u
    assert sa == sb + 1
    return sb, SWAP4 @ u @ SWAP4


def transpile_linear(gates, lay: "Layout", router: str = "up") -> List[list]:
    """Alg. 1 "transpile C to linear connectivity" for the gates of one half
    (in the order they are absorbed), starting from layout `lay` (left as
    is).  Before each gate, SWAPs on consecutive sites carry the qubit on
    the lower site up until the two are neighbours; the resulting gate
    sequence is then layered as soon as possible by the sites each entry
    touches.  Entries: (a, b, u, is_swap, gate id) on logical qubits."""
    site_of, logical_at = list(lay.site_of), list(lay.logical_at)
    seq = []                                  # (lower site, entry)
    for (a, b, u, gid) in gates:
        climb = None
        while abs(site_of[a] - site_of[b]) > 1:
            lo, hi = min(site_of[a], site_of[b]), max(site_of[a], site_of[b])
            if climb is None:               # SWAPs the lower qubit makes ("middle": half the gap)
                climb = hi - lo - 1 if router == "up" else (hi - lo) // 2
            if climb > 0:
                j, climb = lo, climb - 1
            else:
                j = hi - 1
            x, y = logical_at[j], logical_at[j + 1]
            seq.append((j, (x, y, SWAP4, True, None)))
            logical_at[j], logical_at[j + 1] = y, x
            site_of[x], site_of[y] = j + 1, j
        seq.append((min(site_of[a], site_of[b]), (a, b, u, False, gid)))
    busy = [0] * (len(site_of) + 1)
    layers: List[list] = []
    for j, e in seq:
        depth = max(busy[j], busy[j + 1])
        if depth == len(layers):
            layers.append([])
        layers[depth].append(e)
        busy[j] = busy[j + 1] = depth + 1
    return layers


@dataclasses.dataclass
class OracleResult:
    bits: np.ndarray            # peak bitstring on logical qubits
    prob: float
    norm2: float
    site_bits: np.ndarray
    layout_left: List[int]
    layout_right: List[int]
    trace: List[Dict]
    mpo: OracleMPO


class Contraction:
    """Alg. 1 driver with the update sequence spelled out:

    * the circuit is layered ASAP and split at the temporal midpoint: C_R is the
      first ceil(D/2) layers (applied first), C_L the rest;
    * each absorption step takes C_L's innermost layer (gates act on output
      legs) and then C_R's innermost layer (input legs).  For every C_L gate in
      layer order: route it (SWAPs on the output side) and, if a not yet
      absorbed C_R gate of this step lands on the same bond without routing,
      absorb both in one update; then route and absorb the remaining C_R gates;
    * routing moves the qubit on the lower site rightwards by SWAPs, each an
      ordinary bond update plus a layout change;
    * after the inner loop, unswap; accepted swaps change the layouts;
    * an absorption phase always takes at least one step (Alg. 1 would
      otherwise repeat unswapping forever once it cannot get below tau).
    """

    def __init__(self, n: int, gates, cfg: OracleConfig):
        self.n = n
        self.cfg = cfg
        layers = asap_layers(gates, n)
        h = (len(layers) + 1) // 2
        self.right = list(reversed(layers[:h]))     # innermost first
        self.left = layers[h:]
        self.m = OracleMPO(n)
        self.lay_l = Layout(n)
        self.lay_r = Layout(n)
        self.trace: List[Dict] = []
        self.updates = 0
        self.steps = 0                  # absorption steps taken (fixed-frequency phase)
        if cfg.rewire == "eager":
            # Alg. 1 taken literally: each half is transpiled to the line, and
            # after every unswapping stage its remaining circuit gates (the
            # transpilation SWAPs stripped) are reindexed by the layouts and
            # transpiled again
            ids = iter(range(len(gates)))
            self.half_l = [(a, b, u, next(ids)) for layer in self.left for (a, b, u) in layer]
            self.half_r = [(a, b, u, next(ids)) for layer in self.right for (a, b, u) in layer]
            self.done_ids = set()
            self._retranspile()
        elif cfg.rewire != "lazy":
            raise ValueError(cfg.rewire)

    def _retranspile(self):
        self.left = transpile_linear([g for g in self.half_l if g[3] not in self.done_ids], self.lay_l, self.cfg.router)
        self.right = transpile_linear([g for g in self.half_r if g[3] not in self.done_ids], self.lay_r,
                                      self.cfg.router)

    # ------------------------------------------------------------- updates
    def _update(self, i, g_out, g_in, stage, fused=False):
        cfg = self.cfg
        chil, chir = self.m.B[i].shape[0], self.m.B[i + 1].shape[2]
        chi_old = self.m.chi(i)
        r = bond_update(self.m, i, g_out, g_in, cfg.chi_max, cfg.cutoff, cfg.mode)
        commit(self.m, r)
        self.updates += 1
        self.trace.append(dict(stage=stage, bond=i, chi_l=chil, chi=chi_old, chi_r=chir, k=r.k,
                               discarded=r.discarded, total=r.total, size=self.m.size(),
                               s=r.s[:r.k].copy(), fused=fused))

    def _route(self, lay: Layout, a: int, b: int, side: str) -> Tuple[int, int]:
        sa, sb = lay.site_of[a], lay.site_of[b]
        lo, hi = min(sa, sb), max(sa, sb)
        if self.cfg.router == "up":
            bonds = list(range(lo, hi - 1))
        else:
            # the lower qubit climbs ceil((gap - 1) / 2) sites, the upper one
            # comes down the rest
            up = (hi - lo) // 2
            bonds = [lo + t for t in range(up)] + [hi - 1 - t for t in range(hi - lo - 1 - up)]
        for j in bonds:
            if side == "L":
                self._update(j, SWAP4, None, "route")
            else:
                self._update(j, None, SWAP4, "route")
            lay.swap_sites(j)
        return lay.site_of[a], lay.site_of[b]

    def absorb_step(self):
        """One absorption step under the configured side selection."""
        mode = self.cfg.side
        if mode == "both" or not (self.left and self.right):
            taken = "L" if self.left else "R"
            self.absorb_layers(self.left.pop(0) if self.left else [],
                               self.right.pop(0) if self.right else [])
            if mode == "fixed":                # one side is used up
                self.trace.append(dict(stage="layer", taken=taken))
        elif mode == "fixed":
            fl, fr = self.cfg.fixed_freq
            if self.steps % (fl + fr) < fl:
                self.absorb_layers(self.left.pop(0), [])
                self.trace.append(dict(stage="layer", taken="L"))
            else:
                self.absorb_layers([], self.right.pop(0))
                self.trace.append(dict(stage="layer", taken="R"))
        elif mode == "adaptive":
            self.absorb_adaptive()
        else:
            raise ValueError(mode)
        self.steps += 1

    def absorb_adaptive(self):
        """App. A.3: the next C_L layer and the next C_R layer are each
        absorbed into a copy of the current state; the copy with the smaller
        size(M) is kept (equal sizes: the left one) and the other layer stays
        pending.  Updates of the discarded copy are counted as trials."""
        cands = []
        for side in ("L", "R"):
            c = Contraction.__new__(Contraction)
            c.n, c.cfg = self.n, self.cfg
            c.left, c.right = list(self.left), list(self.right)
            c.m = self.m.copy()
            c.lay_l, c.lay_r = Layout(self.n), Layout(self.n)
            c.lay_l.site_of, c.lay_l.logical_at = list(self.lay_l.site_of), list(self.lay_l.logical_at)
            c.lay_r.site_of, c.lay_r.logical_at = list(self.lay_r.site_of), list(self.lay_r.logical_at)
            c.trace, c.updates, c.steps = [], 0, self.steps
            if self.cfg.rewire == "eager":
                c.half_l, c.half_r, c.done_ids = self.half_l, self.half_r, set(self.done_ids)
            if side == "L":
                c.absorb_layers(c.left.pop(0), [])
            else:
                c.absorb_layers([], c.right.pop(0))
            cands.append(c)
        sizes = [c.m.size() for c in cands]
        keep = cands[0] if sizes[0] <= sizes[1] else cands[1]
        other = cands[1] if keep is cands[0] else cands[0]
        self.left, self.right, self.m = keep.left, keep.right, keep.m
        self.lay_l, self.lay_r = keep.lay_l, keep.lay_r
        if self.cfg.rewire == "eager":
            self.done_ids = keep.done_ids
        self.trace.extend(keep.trace)
        self.updates += keep.updates
        self.trial_absorb_updates = getattr(self, "trial_absorb_updates", 0) + other.updates
        self.trace.append(dict(stage="side", side="L" if keep is cands[0] else "R",
                               size_left=sizes[0], size_right=sizes[1]))

    def absorb_layers(self, lgates, rgates):
        """One absorption step's updates.  Entries of eager (transpiled)
        layers carry a flag: a transpilation SWAP is absorbed as a SWAP update
        on its side and exchanges the two sites in that side's layout; a
        circuit gate's id is noted as absorbed."""
        def flag(g):
            return (g[3], g[4]) if len(g) == 5 else (False, None)

        pending = list(rgates)
        for g in lgates:
            a, b, u = g[:3]
            is_swap, gid = flag(g)
            if is_swap:
                i = min(self.lay_l.site_of[a], self.lay_l.site_of[b])
                assert abs(self.lay_l.site_of[a] - self.lay_l.site_of[b]) == 1
                self._update(i, SWAP4, None, "route")
                self.lay_l.swap_sites(i)
                continue
            sa, sb = self._route(self.lay_l, a, b, "L")
            i, ul = orient(u, sa, sb)
            fused = None
            for idx, rg in enumerate(pending):
                if flag(rg)[0]:
                    continue
                xa, xb = self.lay_r.site_of[rg[0]], self.lay_r.site_of[rg[1]]
                if abs(xa - xb) == 1 and min(xa, xb) == i:
                    fused = idx
                    break
            if fused is not None:
                rg = pending.pop(fused)
                _, ur = orient(rg[2], self.lay_r.site_of[rg[0]], self.lay_r.site_of[rg[1]])
                self._update(i, ul, ur, "absorb", fused=True)
                self._note_done(gid, flag(rg)[1])
            else:
                self._update(i, ul, None, "absorb")
                self._note_done(gid)
        for g in pending:
            a, b, u = g[:3]
            is_swap, gid = flag(g)
            if is_swap:
                i = min(self.lay_r.site_of[a], self.lay_r.site_of[b])
                assert abs(self.lay_r.site_of[a] - self.lay_r.site_of[b]) == 1
                self._update(i, None, SWAP4, "route")
                self.lay_r.swap_sites(i)
                continue
            sa, sb = self._route(self.lay_r, a, b, "R")
            i, ur = orient(u, sa, sb)
            self._update(i, None, ur, "absorb")
            self._note_done(gid)

    def _note_done(self, *gids):
        if self.cfg.rewire == "eager":
            self.done_ids.update(x for x in gids if x is not None)

    def unswap(self):
        cfg = self.cfg
        before = self.m.size()
        if cfg.unswap == "none":
            return []
        if cfg.unswap == "sequential":
            log = unswap_sequential(self.m, cfg)
        elif cfg.unswap == "parallel":
            log = unswap_parallel(self.m, cfg)
        else:
            raise ValueError(cfg.unswap)
        # rewiring (Sec. II.B.3): fold the accepted swaps into the layouts
        for side, i in log:
            if side in ("L", "B"):
                self.lay_l.swap_sites(i)
            if side in ("R", "B"):
                self.lay_r.swap_sites(i)
        self.trace.append(dict(stage="unswap", accepted=len(log), size_before=before,
                               size=self.m.size(), log=list(log)))
        if cfg.rewire == "eager":
            self._retranspile()
        return log

    def gates_absorbed(self) -> int:
        return sum(2 if t.get("fused") else 1 for t in self.trace if t.get("stage") == "absorb")

    def run(self) -> OracleResult:
        cfg = self.cfg
        # size(M) against gates absorbed after every absorption step and
        # unswapping stage: the sawtooth of Sec. III.A
        self.sizes = []
        while self.left or self.right:
            # every absorption phase takes at least one layer pair, so the loop
            # progresses even when unswapping cannot bring size(M) below tau;
            # with eager rewiring a phase goes on until it has absorbed a circuit
            # gate (its first layers may hold only transpilation SWAPs, which
            # unswapping would take out again, and rewiring put back)
            before = self.gates_absorbed()
            self.absorb_step()
            self.sizes.append(("absorb", self.gates_absorbed(), self.m.size()))
            while cfg.rewire == "eager" and self.gates_absorbed() == before and (self.left or self.right):
                self.absorb_step()
                self.sizes.append(("absorb", self.gates_absorbed(), self.m.size()))
            while self.m.size() < cfg.tau and (self.left or self.right):
                self.absorb_step()
                self.sizes.append(("absorb", self.gates_absorbed(), self.m.size()))
            self.unswap()
            self.sizes.append(("unswap", self.gates_absorbed(), self.m.size()))
        site_bits, p, norm2 = extract_peak(self.m)
        bits = np.array([site_bits[self.lay_l.site_of[q]] for q in range(self.n)], dtype=np.uint8)
        res = OracleResult(bits, p, norm2, site_bits, list(self.lay_l.site_of),
                           list(self.lay_r.site_of), self.trace, self.m)
        res.sizes = list(self.sizes)
        return res


def contract(n: int, gates, cfg: OracleConfig) -> OracleResult:
    return Contraction(n, gates, cfg).run()


def full_operator(res: OracleResult) -> np.ndarray:
    """Dense P_L M~ P_R on logical qubits (Eq. (1)), normalised like M."""
    n = res.mpo.n
    mat = res.mpo.dense_operator().reshape([2] * (2 * n))     # out sites..., in sites...
    # output axis of logical q is site layout_left[q]; input axis likewise with layout_right
    perm = [res.layout_left[q] for q in range(n)] + [n + res.layout_right[q] for q in range(n)]
    return mat.transpose(perm).reshape(2 ** n, 2 ** n)
