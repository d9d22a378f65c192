"""Density-matrix simulation for tiny qubit counts -- TEST INFRASTRUCTURE ONLY.

Written independently of ``tusq_oracle.c`` to pin it: full 2^n x 2^n
operators built with Kronecker products, rotations from the matrix
exponential of their Pauli generator, and the channel applied as
rho -> (1 - sum p) rho + sum_k p_k P_k rho P_k (TUSQ Sec. II; the
2-qubit channel uses the 15 non-identity two-qubit Paulis).  Bit q of a basis
index is qubit q, so qubit 0 is the rightmost Kronecker factor.
"""

from __future__ import annotations

import itertools
import math
from typing import Iterable, List, Sequence, Tuple

import numpy as np
from scipy.linalg import expm

I2 = np.eye(2, dtype=np.complex128)
PX = np.array([[0, 1], [1, 0]], dtype=np.complex128)
PY = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
PZ = np.array([[1, 0], [0, -1]], dtype=np.complex128)
PAULIS = (I2, PX, PY, PZ)


def gate_2x2(kind: str, params: Sequence[float]) -> np.ndarray:
    t = params[0] if params else 0.0
    if kind == "RX":
        return expm(-0.5j * t * PX)
    if kind == "RY":
        return expm(-0.5j * t * PY)
    if kind == "RZ":
        return expm(-0.5j * t * PZ)
    if kind == "U3":
        th, ph, la = params[:3]
        # U3 is RZ(phi) RY(theta) RZ(lambda) up to the phase e^{i(phi+lambda)/2}
        return np.exp(0.5j * (ph + la)) * (expm(-0.5j * ph * PZ) @ expm(-0.5j * th * PY)
                                             @ expm(-0.5j * la * PZ))
    if kind == "H":
        return (PX + PZ) / math.sqrt(2)
    if kind == "S":
        return expm(0.25j * math.pi * (I2 - PZ))        # diag(1, i)
    if kind == "SDG":
        return expm(-0.25j * math.pi * (I2 - PZ))
    if kind == "T":
        return expm(0.125j * math.pi * (I2 - PZ))       # diag(1, e^{i pi/4})
    if kind == "TDG":
        return expm(-0.125j * math.pi * (I2 - PZ))
    if kind == "X":
        return PX.copy()
    if kind == "Y":
        return PY.copy()
    if kind == "Z":
        return PZ.copy()
    raise ValueError(kind)


def embed_1q(n: int, q: int, m: np.ndarray) -> np.ndarray:
    out = np.array([[1.0 + 0j]])
    for k in range(n - 1, -1, -1):
        out = np.kron(out, m if k == q else I2)
    return out


def cx_full(n: int, c: int, t: int) -> np.ndarray:
    """CX as |0><0|_c (x) I + |1><1|_c (x) X_t."""
    p0 = np.array([[1, 0], [0, 0]], dtype=np.complex128)
    p1 = np.array([[0, 0], [0, 1]], dtype=np.complex128)
    a = np.array([[1.0 + 0j]])
    b = np.array([[1.0 + 0j]])
    for k in range(n - 1, -1, -1):
        a = np.kron(a, p0 if k == c else I2)
        b = np.kron(b, p1 if k == c else (PX if k == t else I2))
    return a + b


def _matrix_of(params: Sequence[float], d: int) -> np.ndarray:
    v = np.asarray(params, dtype=np.float64)
    return (v[0::2] + 1j * v[1::2]).reshape(d, d)


def embed_2q(n: int, qa: int, qb: int, m: np.ndarray) -> np.ndarray:
    """A 4x4 acting on qubits (qa, qb), index 2 * bit(qa) + bit(qb), as a
    2^n x 2^n matrix, entry by entry."""
    N = 1 << n
    U = np.zeros((N, N), dtype=np.complex128)
    for i in range(N):
        col = 2 * ((i >> qa) & 1) + ((i >> qb) & 1)
        base = i & ~((1 << qa) | (1 << qb))
        for row in range(4):
            j = base | ((row >> 1) << qa) | ((row & 1) << qb)
            U[j, i] = m[row, col]
    return U


def gate_full(n: int, kind: str, qubits: Sequence[int], params: Sequence[float]) -> np.ndarray:
    if kind == "CX":
        return cx_full(n, qubits[0], qubits[1])
    if kind == "UNITARY2":
        return embed_2q(n, qubits[0], qubits[1], _matrix_of(params, 4))
    if kind == "UNITARY1":
        return embed_1q(n, qubits[0], _matrix_of(params, 2))
    return embed_1q(n, qubits[0], gate_2x2(kind, params))


def pauli_full(n: int, paulis: Iterable[Tuple[int, int]]) -> np.ndarray:
    """Product of single-qubit Paulis [(qubit, code)], code I=0 X=1 Y=2 Z=3."""
    m = np.eye(1 << n, dtype=np.complex128)
    for q, p in paulis:
        m = embed_1q(n, q, PAULIS[p]) @ m
    return m


def channel_terms(kind: str, qubits, probs) -> List[Tuple[float, List[Tuple[int, int]]]]:
    """(probability, paulis) for every non-identity outcome of a channel."""
    terms = []
    if len(probs) == 3:
        for k in range(3):
            terms.append((probs[k], [(qubits[0], k + 1)]))
    else:
        for k in range(1, 16):
            a, b = k >> 2, k & 3
            ps = []
            if a:
                ps.append((qubits[0], a))
            if b:
                ps.append((qubits[1], b))
            terms.append((probs[k - 1], ps))
    return terms


def measure_kraus(n: int, qubits: Sequence[int], reset: bool) -> List[np.ndarray]:
    """Kraus operators of a Z-basis measurement of `qubits` whose outcome is
    discarded: the projectors onto each outcome pattern, each followed (for a
    reset) by the X flips that return the measured qubits to 0."""
    out = []
    N = 1 << n
    for o in range(1 << len(qubits)):
        K = np.zeros((N, N), dtype=np.complex128)
        for i in range(N):
            if all(((i >> q) & 1) == ((o >> b) & 1) for b, q in enumerate(qubits)):
                j = i
                if reset:
                    for q in qubits:
                        j &= ~(1 << q)
                K[j, i] = 1.0
        out.append(K)
    return out


def density_matrix(circ) -> np.ndarray:
    n = circ.n
    rho = np.zeros((1 << n, 1 << n), dtype=np.complex128)
    rho[0, 0] = 1.0
    for kind, qs, pr, noise in zip(circ.kinds, circ.qubits, circ.params, circ.noise):
        if kind in ("M", "MR"):
            rho = sum(K @ rho @ K.conj().T for K in measure_kraus(n, qs, kind == "MR"))
            continue
        U = gate_full(n, kind, qs, pr)
        rho = U @ rho @ U.conj().T
        if noise is not None:
            terms = channel_terms(kind, qs, noise)
            new = (1.0 - sum(p for p, _ in terms)) * rho
            for p, ps in terms:
                P = pauli_full(n, ps)
                new = new + p * (P @ rho @ P.conj().T)
            rho = new
    return rho


def circuit_unitary(circ, events=()) -> np.ndarray:
    """Unitary of the circuit with Pauli events (slot, qubit, pauli) applied
    just before the gate of their slot (slot G: after the last gate)."""
    n = circ.n
    ev = sorted(events)
    U = np.eye(1 << n, dtype=np.complex128)
    e = 0
    G = circ.n_gates
    for s in range(G + 1):
        while e < len(ev) and ev[e][0] == s:
            U = pauli_full(n, [(ev[e][1], ev[e][2])]) @ U
            e += 1
        if s < G:
            U = gate_full(n, circ.kinds[s], circ.qubits[s], circ.params[s]) @ U
    return U


def equal_up_to_phase(A: np.ndarray, B: np.ndarray, tol: float = 1e-10) -> bool:
    idx = np.unravel_index(np.argmax(np.abs(B)), B.shape)
    if abs(B[idx]) < 1e-12:
        return np.allclose(A, B, atol=tol)
    ph = A[idx] / B[idx]
    if abs(abs(ph) - 1.0) > tol:
        return False
    return np.allclose(A, ph * B, atol=tol)


def enumerate_ers(circ):
    """Every error realisation with its exact probability: yields
    (probability, raw events with slot = gate + 1)."""
    chans = [(g, noise) for g, noise in enumerate(circ.noise) if noise is not None]
    options = []
    for g, probs in chans:
        opts = [(1.0 - sum(probs), [])]
        qs = circ.qubits[g]
        if len(probs) == 3:
            for k in range(3):
                opts.append((probs[k], [(g + 1, qs[0], k + 1)]))
        else:
            for k in range(1, 16):
                a, b = k >> 2, k & 3
                ev = []
                if a:
                    ev.append((g + 1, qs[0], a))
                if b:
                    ev.append((g + 1, qs[1], b))
                opts.append((probs[k - 1], ev))
        options.append(opts)
    for combo in itertools.product(*options):
        p = 1.0
        ev = []
        for pk, e in combo:
            p *= pk
            ev.extend(e)
        yield p, sorted(ev)
