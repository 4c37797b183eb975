"""Seeded synthetic mirrored peaked circuits (input generator only).

This module produces the *inputs* of the middle-MPO contraction: a time-ordered
list of two-qubit gates on a line of qubits.  It holds none of the contraction
arithmetic (no MPO, no SVD, no truncation, no schedule); both the GPU path and
the CPU oracle read the circuits it writes.

Construction (a stand-in for the mirrored, swap-obfuscated peaked circuits the
paper attacks, Sec. I and Sec. II.A):

    C = X^b . K . R^dag . S_inv . S . R          (time runs right to left)

* R      -- ``depth`` brickwork layers of Haar-random SU(4) gates on adjacent
            pairs; layer l uses pairs (2j, 2j+1) when l is even and
            (2j+1, 2j+2) when l is odd.
* S      -- the SWAP network of an odd-even transposition sort of a random
            permutation pi.
* S_inv  -- reading "B" (default): the odd-even transposition network of
            pi^{-1}, built independently of S, so S_inv . S = I as operators
            while no gate of S_inv mirrors a gate of S.  Reading "A": the gate
            reversal of S (a literal mirror).
* K      -- two brickwork layers of near-identity gates exp(i sum_k t_k P_k)
            over the 15 non-identity two-qubit Paulis, t_k ~ N(0, std).
* X^b    -- a planted bitstring b; X on qubit q is folded into the last gate
            that touches q.

Obfuscation: a SWAP whose preceding gate on both its wires is one gate on the
same pair is multiplied into that gate; afterwards every wire segment between
two consecutive gates receives a Haar U(2) u, put into the earlier gate's
output leg and u^dag into the later gate's input leg.  The circuit operator is
unchanged by both steps, so C = X^b K as an operator and the peak is b.

Admissibility: K is redrawn from the same stream until every conditional
P(x_j = 0 | x_<j = 0) of K|0^n> exceeds 1/2, so that a greedy conditional
argmax of C|0^n> (the peak readout, Sec. II.C) lands on b.  Seeds whose first
K passes are unaffected.

Conventions: a gate (q0, q1, U) acts on |q0 q1> with q0 the most significant
bit of the 4x4 row-major matrix U.  In dense vectors qubit 0 is the most
significant bit.  Random draws come from numpy's PCG64 in the fixed order
pi, R, K (and its redraws), b, dressing.
"""
from __future__ import annotations

import dataclasses
import hashlib
import io
from typing import List, Optional, Tuple

import numpy as np

Gate = Tuple[int, int, np.ndarray]

SWAP = np.array([[1, 0, 0, 0],
                 [0, 0, 1, 0],
                 [0, 1, 0, 0],
                 [0, 0, 0, 1]], dtype=np.complex128)

_PAULI1 = [np.eye(2, dtype=np.complex128),
           np.array([[0, 1], [1, 0]], dtype=np.complex128),
           np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
           np.array([[1, 0], [0, -1]], dtype=np.complex128)]
_X = _PAULI1[1]


@dataclasses.dataclass
class Circuit:
    """A time-ordered gate list on ``n`` qubits plus the generator's metadata."""
    n: int
    gates: List[Gate]
    peak: np.ndarray                 # planted bitstring b (uint8, length n)
    k_gates: List[Gate]              # undressed K gates (for closed forms)
    perm: np.ndarray                 # pi
    meta: dict

    # ------------------------------------------------------------------ io
    def to_npz_bytes(self) -> bytes:
        buf = io.BytesIO()
        np.savez(buf,
                 n=np.int64(self.n),
                 qubits=np.array([[g[0], g[1]] for g in self.gates], dtype=np.int32).reshape(-1, 2),
                 mats=np.array([g[2] for g in self.gates], dtype=np.complex128).reshape(-1, 4, 4),
                 peak=self.peak.astype(np.uint8),
                 k_qubits=np.array([[g[0], g[1]] for g in self.k_gates], dtype=np.int32).reshape(-1, 2),
                 k_mats=np.array([g[2] for g in self.k_gates], dtype=np.complex128).reshape(-1, 4, 4),
                 perm=self.perm.astype(np.int64),
                 meta=np.array(repr(sorted(self.meta.items()))))
        return buf.getvalue()

    def save(self, path: str) -> None:
        with open(path, "wb") as f:
            f.write(self.to_npz_bytes())

    @staticmethod
    def load(path: str) -> "Circuit":
        z = np.load(path, allow_pickle=False)
        gates = [(int(q[0]), int(q[1]), m) for q, m in zip(z["qubits"], z["mats"])]
        kg = [(int(q[0]), int(q[1]), m) for q, m in zip(z["k_qubits"], z["k_mats"])]
        return Circuit(int(z["n"]), gates, z["peak"].astype(np.uint8), kg,
                       z["perm"].astype(np.int64), {"loaded_from": path})

    def digest(self) -> str:
        h = hashlib.sha256()
        h.update(np.int64(self.n).tobytes())
        for q0, q1, m in self.gates:
            h.update(np.array([q0, q1], dtype=np.int32).tobytes())
            h.update(np.ascontiguousarray(m, dtype=np.complex128).tobytes())
        h.update(self.peak.astype(np.uint8).tobytes())
        return h.hexdigest()

    @property
    def peak_string(self) -> str:
        return "".join(str(int(x)) for x in self.peak)


# ---------------------------------------------------------------- primitives
def haar_unitary(rng: np.random.Generator, d: int) -> np.ndarray:
    """Haar-distributed U(d): QR of a complex Ginibre matrix with the phases of
    R's diagonal folded back into Q (Mezzadri's recipe)."""
    z = (rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    dg = np.diag(r)
    return q * (dg / np.abs(dg))[None, :]


def haar_su4(rng: np.random.Generator) -> np.ndarray:
    u = haar_unitary(rng, 4)
    return u / np.linalg.det(u) ** 0.25


def near_identity_gate(rng: np.random.Generator, std: float) -> np.ndarray:
    """exp(i sum_k t_k P_k) over the 15 non-identity two-qubit Paulis."""
    h = np.zeros((4, 4), dtype=np.complex128)
    for a in range(4):
        for b in range(4):
            if a == 0 and b == 0:
                continue
            h += rng.normal(0.0, std) * np.kron(_PAULI1[a], _PAULI1[b])
    w, v = np.linalg.eigh(h)
    return (v * np.exp(1j * w)[None, :]) @ v.conj().T


def brickwork_pairs(n: int, layer: int) -> List[Tuple[int, int]]:
    start = layer % 2
    return [(q, q + 1) for q in range(start, n - 1, 2)]


def oets_swaps(arr: np.ndarray) -> List[List[Tuple[int, int]]]:
    """Rounds of an odd-even transposition sort of ``arr``.  Round r
    compare-exchanges pairs (i, i+1) with i = r mod 2; a SWAP is recorded
    whenever the pair is out of order.  Empty rounds are dropped."""
    a = list(int(x) for x in arr)
    n = len(a)
    rounds = []
    r = 0
    while any(a[i] > a[i + 1] for i in range(n - 1)):
        sw = []
        for i in range(r % 2, n - 1, 2):
            if a[i] > a[i + 1]:
                a[i], a[i + 1] = a[i + 1], a[i]
                sw.append((i, i + 1))
        if sw:
            rounds.append(sw)
        r += 1
    return rounds


def transposition_swaps(arr: np.ndarray) -> List[List[Tuple[int, int]]]:
    """A selection sort of ``arr`` as SWAPs on arbitrary pairs (all-to-all
    connectivity): for position i in order, the value i is swapped in from
    wherever it sits.  One SWAP per round; the pair is (i, j), i < j."""
    a = list(int(x) for x in arr)
    where = {v: k for k, v in enumerate(a)}
    rounds = []
    for i in range(len(a)):
        j = where[i]
        if j != i:
            vi = a[i]
            a[i], a[j] = a[j], a[i]
            where[vi], where[i] = j, i
            rounds.append([(i, j)])
    return rounds


def matching_pairs(rng: np.random.Generator, n: int) -> List[Tuple[int, int]]:
    """A random perfect matching of the n qubits (one qubit idle when n is
    odd), each pair in random order: one layer of an all-to-all circuit."""
    q = rng.permutation(n)
    return [(int(q[2 * j]), int(q[2 * j + 1])) for j in range(n // 2)]


def embed_1q(u: np.ndarray, which: int) -> np.ndarray:
    """4x4 matrix of a single-qubit u on the first (which=0, MSB) or second qubit."""
    return np.kron(u, np.eye(2)) if which == 0 else np.kron(np.eye(2), u)


# ---------------------------------------------------------------- admissibility
def k_prefix_conditionals(n: int, k_layers) -> np.ndarray:
    """P(x_j = 0 | x_<j = 0), j = 0..n-1, of the state K|0^n> (input check).

    The planted peak is read greedily (a deterministic conditional argmax):
    it returns b when every one of these conditionals exceeds 1/2, because
    C = X^b K as an operator.  K has two brickwork layers, so K|0^n> is a
    chain of 2 x 2 x 2 tensors per qubit whose bonds (at most 4) come from
    writing each gate's output on its two qubits with the right qubit's value
    carried in the bond: an exact rewriting, no decomposition.  The prefix
    probability P(0^j) is the prefix-projected amplitude row times the right
    environment of the chain."""
    chain = []
    for _ in range(n):
        t = np.zeros((1, 2, 1), dtype=np.complex128)
        t[0, 0, 0] = 1.0
        chain.append(t)
    for layer in k_layers:
        for (q0, q1, u) in layer:
            a, b = chain[q0], chain[q1]
            dl, dr = a.shape[0], b.shape[2]
            # (l, y, m) (m, y', r) -> (l, y, y', r), then the gate on (y, y')
            pair = np.einsum("lym,mzr->lyzr", a, b)
            out = np.einsum("xwyz,lyzr->lxwr", u.reshape(2, 2, 2, 2), pair)
            # left tensor keeps x and carries (w, r) in its right bond; the
            # right tensor reads w back out of the bond
            chain[q0] = out.reshape(dl, 2, 2 * dr)
            right = np.zeros((2 * dr, 2, dr), dtype=np.complex128)
            for w in range(2):
                right[w * dr:(w + 1) * dr, w, :] = np.eye(dr)
            chain[q1] = right
    env = [np.ones((1, 1), dtype=np.complex128)]
    for t in reversed(chain):
        e = env[-1]
        env.append(t[:, 0, :] @ e @ t[:, 0, :].conj().T + t[:, 1, :] @ e @ t[:, 1, :].conj().T)
    env = env[::-1]                                   # env[j]: right environment of qubits >= j
    row = np.ones((1, 1), dtype=np.complex128)
    cond = np.zeros(n)
    for j in range(n):
        p_prefix = float((row @ env[j] @ row.conj().T).real[0, 0])
        nxt = row @ chain[j][:, 0, :]
        p_next = float((nxt @ env[j + 1] @ nxt.conj().T).real[0, 0])
        cond[j] = p_next / p_prefix
        row = nxt / np.sqrt(p_next)
    return cond


# ---------------------------------------------------------------- generator
def mirrored_peaked_circuit(n: int, depth: int, seed: int, *, reading: str = "B",
                            k_std: float = 0.1, with_k: bool = True,
                            with_peak: bool = True, with_swaps: bool = True,
                            fuse_swaps: bool = True, dress: bool = True,
                            min_margin: float = 0.5, max_k_draws: int = 64,
                            connectivity: str = "line") -> Circuit:
    """Build C = X^b K R^dag S_inv S R (see the module docstring).  K is
    redrawn until every prefix conditional of K|0^n> exceeds `min_margin`.

    connectivity "all": an all-to-all stand-in for circuits that are not
    nearest-neighbour (the paper's input before transpilation, Sec. II.A):
    R's layers are random perfect matchings and S, S_inv are selection-sort
    SWAP sequences on arbitrary pairs; K stays a nearest-neighbour brickwork
    (so the closed form of the peak is unchanged)."""
    if n < 2:
        raise ValueError("need at least two qubits")
    if reading not in ("A", "B"):
        raise ValueError("reading must be 'A' or 'B'")
    if connectivity not in ("line", "all"):
        raise ValueError("connectivity must be 'line' or 'all'")
    rng = np.random.Generator(np.random.PCG64(seed))

    perm = rng.permutation(n) if with_swaps else np.arange(n)
    if connectivity == "line":
        r_layers = [[(q0, q1, haar_su4(rng)) for (q0, q1) in brickwork_pairs(n, l)]
                    for l in range(depth)]
    else:
        r_layers = [[(q0, q1, haar_su4(rng)) for (q0, q1) in matching_pairs(rng, n)]
                    for _ in range(depth)]
    sort_net = oets_swaps if connectivity == "line" else transposition_swaps
    k_layers = []
    if with_k:
        # K is drawn again (same stream) until the planted peak is readable by
        # the greedy conditional argmax: every prefix conditional of K|0^n>
        # above min_margin
        for _ in range(max_k_draws):
            k_layers = [[(q0, q1, near_identity_gate(rng, k_std)) for (q0, q1) in brickwork_pairs(n, l)]
                        for l in range(2)]
            if k_prefix_conditionals(n, k_layers).min() > min_margin:
                break
        else:
            raise RuntimeError(f"no admissible K after {max_k_draws} draws (n={n}, seed={seed})")
    peak = rng.integers(0, 2, size=n).astype(np.uint8) if with_peak else np.zeros(n, np.uint8)

    seq: List[list] = []          # mutable [q0, q1, U, is_bare_swap]
    for layer in r_layers:
        seq += [[q0, q1, u.copy(), False] for (q0, q1, u) in layer]
    s_rounds = sort_net(perm)
    if reading == "B":
        inv = np.empty(n, dtype=np.int64)
        inv[perm] = np.arange(n)
        sinv_rounds = sort_net(inv)
    else:
        sinv_rounds = [list(reversed(r)) for r in reversed(s_rounds)]
    for rnd in s_rounds + sinv_rounds:
        seq += [[q0, q1, SWAP.copy(), True] for (q0, q1) in rnd]
    for layer in reversed(r_layers):
        seq += [[q0, q1, u.conj().T.copy(), False] for (q0, q1, u) in layer]
    for layer in k_layers:
        seq += [[q0, q1, u.copy(), False] for (q0, q1, u) in layer]

    # fuse each SWAP into its predecessor when that predecessor is one gate on the same pair
    if fuse_swaps:
        out: List[list] = []
        last = [-1] * n
        for g in seq:
            q0, q1, u, bare = g
            if bare and last[q0] >= 0 and last[q0] == last[q1]:
                prev = out[last[q0]]
                if prev[0] == q0 and prev[1] == q1:
                    prev[2] = SWAP @ prev[2]
                    prev[3] = False
                    continue
            out.append(g)
            last[q0] = last[q1] = len(out) - 1
        seq = out

    # fold X^b into the last gate touching each flipped qubit
    if with_peak:
        for q in range(n):
            if not peak[q]:
                continue
            idx = max(i for i, g in enumerate(seq) if q in (g[0], g[1]))
            g = seq[idx]
            g[2] = embed_1q(_X, 0 if g[0] == q else 1) @ g[2]
            g[3] = False

    # u / u^dag dressing of every wire segment between two consecutive gates
    if dress:
        last = [-1] * n
        for i, g in enumerate(seq):
            for w in (g[0], g[1]):
                j = last[w]
                if j >= 0:
                    u = haar_unitary(rng, 2)
                    pg = seq[j]
                    pg[2] = embed_1q(u, 0 if pg[0] == w else 1) @ pg[2]
                    g[2] = g[2] @ embed_1q(u.conj().T, 0 if g[0] == w else 1)
                    pg[3] = False
                    g[3] = False
                last[w] = i

    gates = [(int(g[0]), int(g[1]), np.ascontiguousarray(g[2])) for g in seq]
    k_gates = [(q0, q1, u.copy()) for layer in k_layers for (q0, q1, u) in layer]
    meta = dict(n=n, depth=depth, seed=seed, reading=reading, k_std=k_std, connectivity=connectivity,
                with_k=with_k, with_peak=with_peak, with_swaps=with_swaps,
                fuse_swaps=fuse_swaps, dress=dress,
                swaps_s=sum(len(r) for r in s_rounds),
                swaps_sinv=sum(len(r) for r in sinv_rounds))
    return Circuit(n, gates, peak, k_gates, np.asarray(perm, dtype=np.int64), meta)


def mirror_only_circuit(n: int, depth: int, seed: int, *, dress: bool = True) -> Circuit:
    """An un-obfuscated mirror R^dag R (with optional u/u^dag dressing): the
    collapse case, whose contraction from the exact centre stays at bond
    dimension one."""
    return mirrored_peaked_circuit(n, depth, seed, with_k=False, with_peak=False,
                                   with_swaps=False, fuse_swaps=False, dress=dress)


# ---------------------------------------------------------------- workloads
def config_circuit(config: int, index: int = 0, reading: str = "B") -> Circuit:
    """The seeded circuits of the measured workloads; circuit ``index`` of
    workload ``config`` uses seed 1000*config + index."""
    seed = 1000 * config + index
    if config == 0:
        return mirrored_peaked_circuit(10, 4, seed, reading=reading)
    if config == 1:
        return mirrored_peaked_circuit(32, 8, seed, reading=reading)
    if config == 2:
        return mirrored_peaked_circuit(56, 12, seed, reading=reading)
    if config == 3:
        rng = np.random.Generator(np.random.PCG64(seed))
        n = int(rng.integers(16, 49))
        depth = int(rng.integers(4, 11))
        return mirrored_peaked_circuit(n, depth, seed, reading=reading)
    raise ValueError(f"no fixed circuit for workload {config}")


def batch_workload(count: int = 128, seed: int = 3000):
    """(circuit, chi_max) pairs of the batching workload: n ~ U{16..48},
    depth ~ U{4..10}, chi_max ~ U{128, 256, 512}."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(count):
        n = int(rng.integers(16, 49))
        depth = int(rng.integers(4, 11))
        chi = int(rng.choice([128, 256, 512]))
        out.append((mirrored_peaked_circuit(n, depth, seed + 1 + i), chi))
    return out


def serving_arrivals(rate: float, duration: float, seed: int = 4000):
    """Poisson arrivals over ``duration`` seconds: list of (t_arrival, n, depth, seed)."""
    rng = np.random.Generator(np.random.PCG64(seed + int(rate * 1000)))
    t = 0.0
    out = []
    i = 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        n = int(rng.choice([24, 40, 56], p=[0.5, 0.3, 0.2]))
        out.append((t, n, n // 4, seed + 17 * i + 1))
        i += 1
    return out
