"""Dense brute force and closed forms -- TEST INFRASTRUCTURE ONLY.

Pins for the oracle in :mod:`oracle.mpo_oracle` that do not go through the
MPO method at all:

* dense circuit unitaries and statevectors (n <= 12 / n <= 20);
* the operator-Schmidt values of a two-qubit gate in canonical (KAK) form,
  which are the singular values one absorption of that gate into the
  identity MPO must produce (Sec. II.B.1 on a single gate);
* the peak probability |<0|K|0>|^2 of the planted circuit C = X^b K as a
  bond-2 transfer product over K's two brickwork layers;
* the conditional marginals of K|0> along 0...0, which decide whether a
  greedy left-to-right readout (Sec. II.C, deterministic variant) returns the
  planted peak.
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np

PAULI = [np.eye(2, dtype=np.complex128),
         np.array([[0, 1], [1, 0]], dtype=np.complex128),
         np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
         np.array([[1, 0], [0, -1]], dtype=np.complex128)]


# ------------------------------------------------------------------ dense
def apply_gate_state(psi: np.ndarray, n: int, q0: int, q1: int, u: np.ndarray) -> np.ndarray:
    """psi has shape (2,)*n (qubit 0 first); u acts on |q0 q1>, q0 the MSB."""
    g = np.asarray(u).reshape(2, 2, 2, 2)
    out = np.tensordot(g, psi, axes=([2, 3], [q0, q1]))        # (q0', q1', rest...)
    rest = [q for q in range(n) if q not in (q0, q1)]
    order = [q0, q1] + rest
    inv = np.argsort(order)
    return out.transpose(inv)


def circuit_unitary(n: int, gates: Sequence[Tuple[int, int, np.ndarray]]) -> np.ndarray:
    """Dense 2^n x 2^n unitary of the time-ordered gate list."""
    u = np.eye(2 ** n, dtype=np.complex128).reshape([2] * n + [2 ** n])
    for q0, q1, g in gates:
        gg = np.asarray(g).reshape(2, 2, 2, 2)
        out = np.tensordot(gg, u, axes=([2, 3], [q0, q1]))
        rest = [q for q in range(n) if q not in (q0, q1)]
        order = [q0, q1] + rest + [n]
        u = out.transpose(np.argsort(order))
    return u.reshape(2 ** n, 2 ** n)


def circuit_state(n: int, gates) -> np.ndarray:
    psi = np.zeros([2] * n, dtype=np.complex128)
    psi[(0,) * n] = 1.0
    for q0, q1, g in gates:
        psi = apply_gate_state(psi, n, q0, q1, g)
    return psi.reshape(-1)


def bits_of(index: int, n: int) -> np.ndarray:
    return np.array([(index >> (n - 1 - q)) & 1 for q in range(n)], dtype=np.uint8)


# ------------------------------------------------------------ KAK closed form
def kak_gate(a: float, b: float, c: float) -> np.ndarray:
    h = a * np.kron(PAULI[1], PAULI[1]) + b * np.kron(PAULI[2], PAULI[2]) + c * np.kron(PAULI[3], PAULI[3])
    w, v = np.linalg.eigh(h)
    return (v * np.exp(1j * w)[None, :]) @ v.conj().T


def kak_schmidt_values(a: float, b: float, c: float) -> np.ndarray:
    """Operator-Schmidt values of exp(i(a XX + b YY + c ZZ)) normalised to unit
    2-norm.  XX, YY, ZZ commute and XX.YY = -ZZ, YY.ZZ = -XX, ZZ.XX = -YY,
    XX.YY.ZZ = -II, so the product of the three exponentials expands on
    {II, XX, YY, ZZ} with the coefficients below; the four Pauli products are
    Hilbert-Schmidt orthogonal, so their moduli are the Schmidt values."""
    ca, sa, cb, sb, cc, sc = np.cos(a), np.sin(a), np.cos(b), np.sin(b), np.cos(c), np.sin(c)
    coef = np.array([ca * cb * cc + 1j * sa * sb * sc,
                     ca * sb * sc + 1j * sa * cb * cc,
                     sa * cb * sc + 1j * ca * sb * cc,
                     sa * sb * cc + 1j * ca * cb * sc])
    return np.sort(np.abs(coef))[::-1]


# ------------------------------------------------------- planted-peak forms
def _k_layers(k_gates, n):
    even = {q0: u for (q0, q1, u) in k_gates if q0 % 2 == 0}
    odd = {q0: u for (q0, q1, u) in k_gates if q0 % 2 == 1}
    return even, odd


def peak_amplitude_closed_form(n: int, k_gates) -> complex:
    """<0^n| K1 K0 |0^n> by a transfer product with a 2-dim carry.

    K0 (pairs (2j,2j+1)) maps |00> to a pair state phi_j; K1 (pairs (2j+1,2j+2))
    is then projected on <00|.  The carry is the value of the odd qubit 2j+1
    entering K1's gate on (2j+1, 2j+2)."""
    even, odd = _k_layers(k_gates, n)

    def phi(j):                       # pair state of qubits (2j, 2j+1), or |0> for a lone last qubit
        if 2 * j + 1 < n:
            return even[2 * j][:, 0].reshape(2, 2)
        return np.array([[1.0], [0.0]], dtype=np.complex128)    # (x_{2j}, dummy)

    # qubit 0 is never touched by K1: project it on <0| right away
    carry = phi(0)[0, :].copy() if n > 1 else None              # over x_1
    j = 0
    while True:
        q = 2 * j + 1                                           # carry lives on qubit q
        if q >= n - 1 or q not in odd:
            # no K1 gate on (q, q+1): q is projected on <0| directly
            amp = carry[0]
            # remaining qubits after q (none for a well-formed brickwork)
            return complex(amp)
        nxt = phi(j + 1)                                        # (x_{q+1}, x_{q+2})
        g = odd[q].reshape(2, 2, 2, 2)[0, 0]                     # <00| K1 |x_q x_{q+1}>
        if 2 * (j + 1) + 1 < n:
            carry = np.einsum("x,xy,yz->z", carry, g, nxt)
        else:
            return complex(np.einsum("x,xy,y->", carry, g, nxt[:, 0]))
        j += 1


def peak_probability_closed_form(n: int, k_gates) -> float:
    return float(abs(peak_amplitude_closed_form(n, k_gates)) ** 2)


def k_state_margins(n: int, k_gates) -> np.ndarray:
    """Conditional probabilities P(x_i = 0 | x_<i = 0) of K|0^n>, exact.

    K|0> is written as a chain of small tensors (bond <= 4) without any
    truncation: K0's pair states, then each K1 gate contracted into its two
    qubits by a full-rank split.  Right environments give the marginals."""
    even, odd = _k_layers(k_gates, n)
    # start: product of pair states, each split into two site tensors (a, x, b)
    sites: List[np.ndarray] = []
    q = 0
    while q < n:
        if q + 1 < n and q in even:
            ph = even[q][:, 0].reshape(2, 2)
            u, s, vh = np.linalg.svd(ph)
            sites.append(u.reshape(1, 2, 2))
            sites.append((np.diag(s) @ vh).reshape(2, 2, 1))
            q += 2
        else:
            t = np.zeros((1, 2, 1), dtype=np.complex128)
            t[0, 0, 0] = 1.0
            sites.append(t)
            q += 1
    for q0, u in sorted(odd.items()):
        a, b = sites[q0], sites[q0 + 1]
        th = np.tensordot(a, b, axes=([2], [0]))                 # (l, x, y, r)
        th = np.einsum("xyuv,luvr->lxyr", u.reshape(2, 2, 2, 2), th)
        l, r = th.shape[0], th.shape[3]
        uu, s, vh = np.linalg.svd(th.reshape(l * 2, 2 * r), full_matrices=False)
        sites[q0] = uu.reshape(l, 2, -1)
        sites[q0 + 1] = (np.diag(s) @ vh).reshape(-1, 2, r)
    env = [None] * (n + 1)
    env[n] = np.ones((1, 1), dtype=np.complex128)
    for i in range(n - 1, -1, -1):
        t = sites[i]
        env[i] = sum(t[:, x, :] @ env[i + 1] @ t[:, x, :].conj().T for x in range(2))
    v = np.ones((1,), dtype=np.complex128)
    out = np.zeros(n)
    for i in range(n):
        w = [v @ sites[i][:, x, :] for x in range(2)]
        p = [float((w[x] @ env[i + 1] @ w[x].conj()).real) for x in range(2)]
        out[i] = p[0] / (p[0] + p[1])
        v = w[0] / np.linalg.norm(w[0])
    return out
