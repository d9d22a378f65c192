"""Circuit descriptions and the seeded generators for the synthetic workloads.

A :class:`Circuit` is plain data.  Gate ``g`` has a kind name, one or two
qubit indices (for CX the first is the control), up to three real parameters,
and optionally the probabilities of a Pauli channel applied right after it:

* 1-qubit channel: ``(pX, pY, pZ)``;
* 2-qubit channel: 15 probabilities, entry ``k - 1`` for ``k = 4a + b``
  (``a`` the Pauli on the gate's first qubit, ``b`` on its second, with
  I=0, X=1, Y=2, Z=3; ``k = 0`` is the identity and carries the rest).

Random numbers here only pick circuit angles and job parameters; they use
numpy's PCG64 seeded by the integers given, so a circuit is fully determined
by its family, sizes and seed.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

GATE_NAMES = ("U3", "RX", "RY", "RZ", "H", "S", "SDG", "T", "TDG", "X", "Y", "Z", "CX")
TWO_QUBIT = frozenset({"CX"})
N_PARAMS = {"U3": 3, "RX": 1, "RY": 1, "RZ": 1}
# a caller's unitary (add_unitary): the gate's params are the matrix,
# row-major, as (re, im) pairs; UNITARY2's basis index is
# 2 * bit(first qubit) + bit(second qubit)
UNITARY_KINDS = ("UNITARY1", "UNITARY2")
# mid-circuit Z-basis measurement layers: "M" keeps the measured qubits in
# their outcome, "MR" resets them to |0> afterwards
MEASURE_KINDS = ("M", "MR")
MAX_MEASURED = 8


@dataclass
class Circuit:
    n: int
    kinds: List[str] = field(default_factory=list)
    qubits: List[tuple] = field(default_factory=list)
    params: List[tuple] = field(default_factory=list)
    noise: List[Optional[tuple]] = field(default_factory=list)
    name: str = ""

    def add(self, kind: str, qubits: Sequence[int], params: Sequence[float] = (),
            noise: Optional[Sequence[float]] = None) -> int:
        if kind not in GATE_NAMES:
            raise ValueError(f"unknown gate kind {kind!r}")
        arity = 2 if kind in TWO_QUBIT else 1
        if len(qubits) != arity:
            raise ValueError(f"{kind} takes {arity} qubit(s)")
        p = tuple(float(x) for x in params) + (0.0,) * (3 - len(params))
        self.kinds.append(kind)
        self.qubits.append(tuple(int(q) for q in qubits))
        self.params.append(p)
        if noise is not None:
            noise = tuple(float(x) for x in noise)
            if len(noise) != (3 if arity == 1 else 15):
                raise ValueError("noise must have 3 (1q) or 15 (2q) probabilities")
        self.noise.append(noise)
        return len(self.kinds) - 1

    def add_unitary(self, qubits: Sequence[int], matrix,
                    noise: Optional[Sequence[float]] = None) -> int:
        """A caller's 2x2 (one qubit) or 4x4 (two qubits, basis index
        2 * bit(qubits[0]) + bit(qubits[1])) unitary, optionally followed by
        a Pauli channel of 3 or 15 probabilities."""
        qs = tuple(int(q) for q in qubits)
        d = 2 if len(qs) == 1 else 4
        m = np.asarray(matrix, dtype=np.complex128)
        if len(qs) not in (1, 2) or m.shape != (d, d):
            raise ValueError("add_unitary takes 1 qubit and a 2x2, or 2 qubits and a 4x4")
        if len(set(qs)) != len(qs) or min(qs) < 0 or max(qs) >= self.n:
            raise ValueError("qubits out of range or repeated")
        if not np.all(np.isfinite(m)) or \
                np.max(np.abs(m.conj().T @ m - np.eye(d))) > 1e-10:
            raise ValueError("matrix is not unitary")
        if noise is not None:
            noise = tuple(float(x) for x in noise)
            if len(noise) != (3 if d == 2 else 15):
                raise ValueError("noise must have 3 (1q) or 15 (2q) probabilities")
        self.kinds.append("UNITARY1" if d == 2 else "UNITARY2")
        self.qubits.append(qs)
        self.params.append(tuple(float(v) for z in m.ravel() for v in (z.real, z.imag)))
        self.noise.append(noise)
        return len(self.kinds) - 1

    def add_readout_noise(self, qubit: int, p: float) -> int:
        """Read-out flip of probability p on `qubit`: an X error just before
        the final read-out, written as RZ(0) (the identity) carrying the
        channel (p, 0, 0).  Append it after the qubit's last gate."""
        if not 0.0 <= p <= 1.0:
            raise ValueError("read-out flip probability outside [0, 1]")
        return self.add("RZ", (qubit,), (0.0,), (float(p), 0.0, 0.0))

    def add_measure(self, qubits: Sequence[int], reset: bool = True) -> int:
        """A layer of concurrent Z-basis measurements of `qubits` (at most
        8, distinct), one non-invertible edge of the circuit tree; with
        `reset` the measured qubits are returned to |0>.  Carries no noise
        channel."""
        qs = tuple(sorted(int(q) for q in qubits))
        if not qs or len(qs) > MAX_MEASURED or len(set(qs)) != len(qs):
            raise ValueError(f"a measurement layer takes 1..{MAX_MEASURED} distinct qubits")
        if qs[0] < 0 or qs[-1] >= self.n:
            raise ValueError("measured qubit out of range")
        self.kinds.append("MR" if reset else "M")
        self.qubits.append(qs)
        self.params.append((0.0, 0.0, 0.0))
        self.noise.append(None)
        return len(self.kinds) - 1

    @property
    def n_gates(self) -> int:
        return len(self.kinds)

    @property
    def n_measure_layers(self) -> int:
        return sum(1 for k in self.kinds if k in MEASURE_KINDS)

    @property
    def n_channels(self) -> int:
        return sum(1 for x in self.noise if x is not None)

    def expected_errors(self) -> float:
        """Mean number of non-identity channel outcomes per shot (lambda)."""
        return float(sum(sum(x) for x in self.noise if x is not None))

    def arrays(self):
        """Flat arrays: kind names, q0, q1, params (G,3), noise count, probs."""
        G = self.n_gates
        q0 = np.zeros(G, dtype=np.uint32)
        q1 = np.zeros(G, dtype=np.uint32)
        for g, qs in enumerate(self.qubits):
            if self.kinds[g] in MEASURE_KINDS:
                # a measurement layer's qubit set as a 64-bit mask split
                # over the two qubit fields (low word, high word)
                mask = sum(1 << q for q in qs)
                q0[g] = mask & 0xFFFFFFFF
                q1[g] = mask >> 32
                continue
            q0[g] = qs[0]
            q1[g] = qs[1] if len(qs) > 1 else 0
        params = np.array([(0.0, 0.0, 0.0) if k in UNITARY_KINDS else p
                           for k, p in zip(self.kinds, self.params)],
                          dtype=np.float64).reshape(G, 3)
        nprob = np.array([0 if x is None else len(x) for x in self.noise], dtype=np.uint8)
        probs = np.array([v for x in self.noise if x is not None for v in x], dtype=np.float64)
        return list(self.kinds), q0, q1, params, nprob, probs

    def unitary_arrays(self):
        """The matrices of UNITARY1 / UNITARY2 gates concatenated as (re, im)
        doubles, and per gate its offset there (0 for other gates)."""
        off = np.zeros(self.n_gates, dtype=np.uint64)
        vals = []
        for g, (k, p) in enumerate(zip(self.kinds, self.params)):
            if k in UNITARY_KINDS:
                off[g] = len(vals)
                vals.extend(p)
        return np.array(vals, dtype=np.float64), off


def depol1(p: float) -> tuple:
    return (p / 3.0,) * 3


def depol2(p: float) -> tuple:
    return (p / 15.0,) * 15


def brickwork(n: int, layers: int, p1: float, p2: float, seed: int) -> Circuit:
    """Random brickwork: per layer, U3 with uniform angles on every qubit in
    ascending order, then CX(i, i+1) for every i with i = layer (mod 2)."""
    rng = np.random.default_rng(seed)
    c = Circuit(n, name=f"brickwork_n{n}_L{layers}")
    two_pi = 2.0 * math.pi
    for layer in range(layers):
        for q in range(n):
            ang = rng.random(3) * two_pi
            c.add("U3", (q,), ang, depol1(p1) if p1 > 0 else None)
        for i in range(layer % 2, n - 1, 2):
            c.add("CX", (i, i + 1), (), depol2(p2) if p2 > 0 else None)
    return c


def ising(n: int, steps: int, p1: float, p2: float, theta: float = 0.1,
          rx: float = 0.2) -> Circuit:
    """Trotterised transverse-field Ising chain: per step, RZZ(theta) on each
    neighbour pair as CX, RZ(theta) on the second qubit, CX; then RX(rx) on
    every qubit."""
    c = Circuit(n, name=f"ising_n{n}_T{steps}")
    for _ in range(steps):
        for i in range(n - 1):
            c.add("CX", (i, i + 1), (), depol2(p2) if p2 > 0 else None)
            c.add("RZ", (i + 1,), (theta,), depol1(p1) if p1 > 0 else None)
            c.add("CX", (i, i + 1), (), depol2(p2) if p2 > 0 else None)
        for q in range(n):
            c.add("RX", (q,), (rx,), depol1(p1) if p1 > 0 else None)
    return c


def bell_pair(p_h: float = 0.0, p_cx: float = 0.0) -> Circuit:
    """H on qubit 0 then CX(0, 1), with optional depolarising noise on each."""
    c = Circuit(2, name="bell")
    c.add("H", (0,), (), depol1(p_h) if p_h > 0 else None)
    c.add("CX", (0, 1), (), depol2(p_cx) if p_cx > 0 else None)
    return c


def syndrome_rounds(d: int, rounds: int, p1: float, p2: float, theta: float = 0.0,
                    reset: bool = True) -> Circuit:
    """Repetition-code memory: data qubits 0..d-1, ancillas d..2d-2; an
    optional RY(theta) on every data qubit first (theta != 0 makes the
    measurement outcomes random), then per round CX(i, d+i), CX(i+1, d+i)
    for every neighbour pair and one measurement layer of all ancillas
    (with reset unless told otherwise).  Stands in for the surface-code
    memory circuits with d rounds of mid-circuit measurement."""
    if d < 2 or 2 * d - 1 > 64 or d - 1 > MAX_MEASURED:
        raise ValueError("need 2 <= d <= 9")
    c = Circuit(2 * d - 1, name=f"syndrome_d{d}_r{rounds}")
    if theta:
        for q in range(d):
            c.add("RY", (q,), (theta,), depol1(p1) if p1 > 0 else None)
    for _ in range(rounds):
        for i in range(d - 1):
            c.add("CX", (i, d + i), (), depol2(p2) if p2 > 0 else None)
            c.add("CX", (i + 1, d + i), (), depol2(p2) if p2 > 0 else None)
        c.add_measure(range(d, 2 * d - 1), reset=reset)
    return c


def random_small_circuit(n: int, n_gates: int, seed: int, p1: float = 0.05,
                         p2: float = 0.05, kinds: Sequence[str] = GATE_NAMES,
                         noisy_fraction: float = 1.0) -> Circuit:
    """Random gate soup over the full gate set, for small-n tests."""
    rng = np.random.default_rng(seed)
    kinds = [k for k in kinds if not (k in TWO_QUBIT and n < 2)]
    c = Circuit(n, name=f"random_n{n}_G{n_gates}_s{seed}")
    for _ in range(n_gates):
        k = kinds[int(rng.integers(len(kinds)))]
        noisy = rng.random() < noisy_fraction
        if k in TWO_QUBIT:
            a, b = rng.choice(n, size=2, replace=False)
            c.add(k, (int(a), int(b)), (), depol2(p2) if (noisy and p2 > 0) else None)
        else:
            q = int(rng.integers(n))
            params = rng.random(N_PARAMS.get(k, 0)) * 2 * math.pi
            c.add(k, (q,), params, depol1(p1) if (noisy and p1 > 0) else None)
    return c


def haar_unitary(d: int, rng) -> np.ndarray:
    """A d x d unitary drawn from the Haar measure (QR of a complex Gaussian
    matrix with the phases of R's diagonal divided out)."""
    z = rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))
    q, r = np.linalg.qr(z)
    return q * (np.diag(r) / np.abs(np.diag(r)))


def unitary_mix(n: int, n_gates: int, seed: int, p1: float = 0.02,
                p2: float = 0.05) -> Circuit:
    """Named gates (U3, CX) mixed with a caller's UNITARY1 / UNITARY2 gates
    (Haar-random), each followed by depolarising noise."""
    rng = np.random.default_rng(seed)
    c = Circuit(n, name=f"unitary_mix_n{n}_G{n_gates}_s{seed}")
    for _ in range(n_gates):
        r = rng.random()
        if r < 0.25:
            c.add("U3", (int(rng.integers(n)),), rng.random(3) * 2 * math.pi, depol1(p1))
        elif r < 0.45:
            a, b = rng.choice(n, 2, replace=False)
            c.add("CX", (int(a), int(b)), (), depol2(p2))
        elif r < 0.7:
            c.add_unitary((int(rng.integers(n)),), haar_unitary(2, rng), depol1(p1))
        else:
            a, b = rng.choice(n, 2, replace=False)
            c.add_unitary((int(a), int(b)), haar_unitary(4, rng), depol2(p2))
    return c


@dataclass
class JobParams:
    index: int
    n: int
    layers: int
    p2: float
    p1: float
    shots: int
    circuit_seed: int
    noise_seed: int


def batch_job_params(n_jobs: int = 4096, base_seed: int = 3, shots: int = 10_000) -> List[JobParams]:
    """Many independent small brickwork jobs: n ~ U{10..16}, layers ~
    U{10..60}, p2 ~ U[1e-3, 2e-2], p1 = p2 / 10."""
    out = []
    for j in range(n_jobs):
        rng = np.random.default_rng((base_seed, j))
        n = int(rng.integers(10, 17))
        layers = int(rng.integers(10, 61))
        p2 = float(rng.uniform(1e-3, 2e-2))
        out.append(JobParams(j, n, layers, p2, p2 / 10.0, shots, 1000 + j, 100_000 + j))
    return out


def batch_jobs(params: Sequence[JobParams]) -> List[Circuit]:
    return [brickwork(p.n, p.layers, p.p1, p.p2, p.circuit_seed) for p in params]


@dataclass
class Request:
    index: int
    arrival_s: float
    family: str
    n: int
    depth: int
    shots: int
    precision: str
    seed: int

    def circuit(self) -> Circuit:
        if self.family == "brickwork":
            return brickwork(self.n, self.depth, 1e-3, 1e-2, self.seed)
        return ising(self.n, self.depth, 5e-4, 5e-3)


def serving_requests(count: int, rate_hz: float, seed: int = 4, n_min: int = 12,
                     n_max: int = 30, shots_exp=(4.0, 6.0)) -> List[Request]:
    """Poisson arrivals; n = floor(exp(u)), u ~ U[ln n_min, ln(n_max+1));
    family and precision 50/50; shots = floor(10^U[a, b])."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        t += float(rng.exponential(1.0 / rate_hz))
        n = int(math.floor(math.exp(rng.uniform(math.log(n_min), math.log(n_max + 1)))))
        n = max(n_min, min(n_max, n))
        fam = "brickwork" if rng.random() < 0.5 else "ising"
        depth = int(rng.integers(10, 21)) if fam == "brickwork" else int(rng.integers(5, 11))
        shots = int(math.floor(10 ** rng.uniform(*shots_exp)))
        prec = "c64" if rng.random() < 0.5 else "c128"
        out.append(Request(i, t, fam, n, depth, shots, prec, 5000 + i))
    return out
