"""ctypes wrapper around ``liboracle.so`` (built from ``tusq_oracle.c`` with
gcc).  Test infrastructure only."""

from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass
from typing import List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tusq_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

KIND_CODES = {name: i for i, name in enumerate(
    ("U3", "RX", "RY", "RZ", "H", "S", "SDG", "T", "TDG", "X", "Y", "Z", "CX", "M", "MR",
     "UNITARY1", "UNITARY2"))}


def build_library(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off",
                               "-fcx-limited-range", "-shared", "-fPIC", "-o", tmp, _SRC,
                               "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Circuit(C.Structure):
    _fields_ = [("n", C.c_uint32), ("G", C.c_uint32),
                ("kind", C.c_void_p), ("q0", C.c_void_p), ("q1", C.c_void_p),
                ("params", C.c_void_p), ("nprob", C.c_void_p), ("probs", C.c_void_p),
                ("mats", C.c_void_p), ("mat_off", C.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build_library())
        L = _lib
        L.oc_ecm.restype = C.c_void_p
        L.oc_ecm.argtypes = [C.c_void_p, C.c_uint64, C.c_uint64, C.c_int, C.c_int,
                             C.c_uint32, C.c_uint32, C.c_uint32]
        L.oc_tree_free.argtypes = [C.c_void_p]
        for f in ("oc_tree_num_leaves", "oc_tree_num_events", "oc_tree_num_raw"):
            getattr(L, f).restype = C.c_uint64
            getattr(L, f).argtypes = [C.c_void_p]
        L.oc_tree_serialize.restype = C.c_size_t
        L.oc_tree_serialize.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t]
        L.oc_run.argtypes = [C.c_void_p, C.c_void_p, C.c_uint64, C.c_int, C.c_uint64,
                             C.c_uint64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.oc_run_margins.argtypes = [C.c_void_p, C.c_void_p, C.c_uint64, C.c_int, C.c_uint64,
                                     C.c_uint64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_void_p]
        L.oc_trajectory.argtypes = [C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_uint64, C.c_void_p]
        L.oc_roundtrip.argtypes = [C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p,
                                   C.c_void_p, C.c_uint64, C.c_void_p]
        L.oc_leaf_margins.argtypes = [C.c_void_p, C.c_void_p, C.c_uint64, C.c_uint64,
                                      C.c_uint64, C.c_void_p, C.c_void_p]
        L.oc_sample_shot.argtypes = [C.c_void_p, C.c_uint64, C.c_uint32, C.c_void_p,
                                     C.c_void_p, C.c_void_p]
        L.oc_commute.argtypes = [C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p, C.c_int,
                                 C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.oc_run_mcm.argtypes = [C.c_void_p, C.c_void_p, C.c_uint64, C.c_uint32, C.c_uint64,
                                 C.c_uint64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.oc_set_checkpoint_slots.argtypes = [C.c_uint64]
        L.oc_prune_select.argtypes = [C.c_uint64, C.c_uint64, C.c_uint32, C.c_void_p]
        L.oc_apportion.argtypes = [C.c_uint64, C.c_void_p, C.c_uint32, C.c_void_p]
        L.oc_bounded.restype = C.c_uint64
        L.oc_bounded.argtypes = [C.c_uint64, C.c_uint32, C.c_uint64]
        L.oc_uniform53.restype = C.c_double
        L.oc_uniform53.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32,
                                   C.c_int]
    return _lib


def set_threads(t: int) -> None:
    lib().oc_set_threads(int(t))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


class _CircuitHandle:
    """Keeps the numpy arrays alive next to the ctypes struct."""

    def __init__(self, circ):
        kinds, q0, q1, params, nprob, probs = circ.arrays()
        self.kind = np.array([KIND_CODES[k] for k in kinds], dtype=np.uint8)
        self.q0, self.q1 = np.ascontiguousarray(q0), np.ascontiguousarray(q1)
        self.params = np.ascontiguousarray(params, dtype=np.float64)
        self.nprob = np.ascontiguousarray(nprob)
        self.probs = np.ascontiguousarray(probs if probs.size else np.zeros(1))
        mats, mat_off = circ.unitary_arrays()
        self.mats = np.ascontiguousarray(mats if mats.size else np.zeros(1))
        self.mat_off = np.ascontiguousarray(mat_off if mat_off.size else np.zeros(1, np.uint64))
        self.n = circ.n
        self.G = len(kinds)
        self.s = _Circuit(circ.n, self.G, _ptr(self.kind) if self.G else None,
                          _ptr(self.q0) if self.G else None, _ptr(self.q1) if self.G else None,
                          _ptr(self.params) if self.G else None,
                          _ptr(self.nprob) if self.G else None, _ptr(self.probs),
                          _ptr(self.mats), _ptr(self.mat_off))

    @property
    def ref(self):
        return C.byref(self.s)


def prune_select(seed: int, nins: int, beta: int) -> List[int]:
    """Positions (ascending) of the beta insignificant circuits the pruning
    stage keeps out of nins (Sec. III-A.4; the oracle's selection step)."""
    out = np.zeros(max(nins, 1), dtype=np.uint64)
    lib().oc_prune_select(int(seed), int(nins), int(beta), _ptr(out))
    return [int(x) for x in out[:beta]]


def apportion(s_insig: int, counts: Sequence[int]) -> List[int]:
    """Integer shots of the selected circuits (the oracle's largest-remainder
    step of Eq. (2))."""
    cnt = np.ascontiguousarray(np.array(counts, dtype=np.uint64))
    out = np.zeros(max(len(counts), 1), dtype=np.uint64)
    lib().oc_apportion(int(s_insig), _ptr(cnt), len(counts), _ptr(out))
    return [int(x) for x in out[:len(counts)]]


def bounded(seed: int, t: int, m: int) -> int:
    """The oracle's uniform integer in [0, m) from stream 1 (draw t)."""
    return int(lib().oc_bounded(int(seed), int(t), int(m)))


def philox(ctr: Sequence[int], key: Sequence[int]) -> Tuple[int, int, int, int]:
    c = (C.c_uint32 * 4)(*ctr)
    k = (C.c_uint32 * 2)(*key)
    o = (C.c_uint32 * 4)()
    lib().oc_philox(c, k, o)
    return tuple(int(x) for x in o)


def thresholds(p: Sequence[float]) -> List[int]:
    a = np.ascontiguousarray(p, dtype=np.float64)
    out = np.zeros(len(a), dtype=np.uint64)
    lib().oc_thresholds(_ptr(a), C.c_int(len(a)), _ptr(out))
    return [int(x) for x in out]


def thermal_probs(t: float, t1: float, t2: float, two_qubit: bool = False) -> List[float]:
    """Pauli-twirled thermal-relaxation channel (Sec. VI-A, Eq. (4)): 3
    probabilities (pX, pY, pZ), or the 15 of the same channel on both qubits
    of a CX.  Raises ValueError outside t >= 0, T1 > 0, 0 < T2 <= 2 T1."""
    out = np.zeros(15 if two_qubit else 3, dtype=np.float64)
    f = lib().oc_thermal_probs2 if two_qubit else lib().oc_thermal_probs
    if f(C.c_double(t), C.c_double(t1), C.c_double(t2), _ptr(out)) != 0:
        raise ValueError("need t >= 0, T1 > 0, 0 < T2 <= 2 T1")
    return [float(x) for x in out]


def sample_shot(circ, seed: int, shot: int):
    h = _CircuitHandle(circ)
    nch = max(1, circ.n_channels)
    ch = np.zeros(nch, dtype=np.uint32)
    out = np.zeros(nch, dtype=np.uint8)
    n = C.c_uint32()
    rc = lib().oc_sample_shot(h.ref, C.c_uint64(seed), C.c_uint32(shot), _ptr(ch), _ptr(out),
                              C.byref(n))
    if rc:
        raise ValueError("invalid circuit")
    return ch[: n.value].copy(), out[: n.value].copy()


def commute(circ, chan, outc, do_commute: bool = True):
    """Canonical event list (slot, qubit, pauli) of one raw ER."""
    h = _CircuitHandle(circ)
    chan = np.ascontiguousarray(chan, dtype=np.uint32)
    outc = np.ascontiguousarray(outc, dtype=np.uint8)
    cap = circ.n * (circ.n_gates + 2) + 2 * len(chan) + 1
    slot = np.zeros(cap, np.uint32)
    qub = np.zeros(cap, np.uint32)
    pau = np.zeros(cap, np.uint8)
    n = C.c_uint32()
    rc = lib().oc_commute(h.ref, C.c_uint32(len(chan)), _ptr(chan) if len(chan) else None,
                          _ptr(outc) if len(outc) else None, C.c_int(int(do_commute)),
                          _ptr(slot), _ptr(qub), _ptr(pau), C.byref(n))
    if rc:
        raise ValueError("invalid circuit")
    k = n.value
    return [(int(slot[i]), int(qub[i]), int(pau[i])) for i in range(k)]


def _events_arrays(events):
    ev = list(events)
    slot = np.array([e[0] for e in ev] or [0], dtype=np.uint32)
    qub = np.array([e[1] for e in ev] or [0], dtype=np.uint32)
    pau = np.array([e[2] for e in ev] or [0], dtype=np.uint8)
    return len(ev), slot, qub, pau


def trajectory(circ, events=(), max_tokens: int = 0) -> np.ndarray:
    """Statevector U_e |0...0> with the events (slot, qubit, pauli) applied
    before the gate of their slot (the whole leaf, or its first tokens)."""
    h = _CircuitHandle(circ)
    ne, slot, qub, pau = _events_arrays(events)
    out = np.zeros(1 << circ.n, dtype=np.complex128)
    rc = lib().oc_trajectory(h.ref, C.c_uint32(ne), _ptr(slot), _ptr(qub), _ptr(pau),
                             C.c_uint64(max_tokens), _ptr(out))
    if rc:
        raise ValueError("invalid circuit or unsorted events")
    return out


def roundtrip(circ, events, depth: int) -> float:
    h = _CircuitHandle(circ)
    ne, slot, qub, pau = _events_arrays(events)
    d = C.c_double()
    rc = lib().oc_roundtrip(h.ref, C.c_uint32(ne), _ptr(slot), _ptr(qub), _ptr(pau),
                            C.c_uint64(depth), C.byref(d))
    if rc:
        raise ValueError("invalid circuit")
    return d.value


@dataclass
class OracleTree:
    circ: object
    handle: int
    n_leaves: int
    ev_off: np.ndarray
    slot: np.ndarray
    qubit: np.ndarray
    pauli: np.ndarray
    count: np.ndarray
    shots: np.ndarray
    wnum: np.ndarray
    wden: np.ndarray
    stats: dict
    _h: object = None

    def events(self, leaf: int):
        a, b = int(self.ev_off[leaf]), int(self.ev_off[leaf + 1])
        return [(int(self.slot[i]), int(self.qubit[i]), int(self.pauli[i])) for i in range(a, b)]

    def weights(self) -> np.ndarray:
        return self.wnum.astype(np.float64) / self.wden.astype(np.float64)

    def serialize(self) -> bytes:
        L = lib()
        size = L.oc_tree_serialize(C.c_void_p(self.handle), None, C.c_size_t(0))
        buf = (C.c_uint8 * size)()
        L.oc_tree_serialize(C.c_void_p(self.handle), buf, C.c_size_t(size))
        return bytes(buf)

    def raw_events(self):
        L = lib()
        n = int(L.oc_tree_num_raw(C.c_void_p(self.handle)))
        shot = np.zeros(max(n, 1), np.uint32)
        chan = np.zeros(max(n, 1), np.uint32)
        out = np.zeros(max(n, 1), np.uint8)
        L.oc_tree_raw(C.c_void_p(self.handle), _ptr(shot), _ptr(chan), _ptr(out))
        return shot[:n], chan[:n], out[:n]

    def __del__(self):
        try:
            if self.handle:
                lib().oc_tree_free(C.c_void_p(self.handle))
                self.handle = 0
        except Exception:
            pass


def ecm(circ, shots: int, seed: int, do_commute: bool = True, prune: bool = True,
        alpha=(1, 100), beta: int = 100) -> OracleTree:
    h = _CircuitHandle(circ)
    L = lib()
    t = L.oc_ecm(h.ref, C.c_uint64(shots), C.c_uint64(seed), C.c_int(int(do_commute)),
                 C.c_int(int(prune)), C.c_uint32(alpha[0]), C.c_uint32(alpha[1]),
                 C.c_uint32(beta))
    if not t:
        raise ValueError("invalid circuit or options")
    nl = int(L.oc_tree_num_leaves(C.c_void_p(t)))
    ne = int(L.oc_tree_num_events(C.c_void_p(t)))
    ev_off = np.zeros(nl + 1, np.uint64)
    slot = np.zeros(max(ne, 1), np.uint32)
    qub = np.zeros(max(ne, 1), np.uint32)
    pau = np.zeros(max(ne, 1), np.uint8)
    cnt = np.zeros(max(nl, 1), np.uint64)
    sh = np.zeros(max(nl, 1), np.uint64)
    wn = np.zeros(max(nl, 1), np.uint64)
    wd = np.zeros(max(nl, 1), np.uint64)
    L.oc_tree_leaves(C.c_void_p(t), _ptr(ev_off), _ptr(slot), _ptr(qub), _ptr(pau), _ptr(cnt),
                     _ptr(sh), _ptr(wn), _ptr(wd))
    st = np.zeros(8, np.uint64)
    L.oc_tree_stats(C.c_void_p(t), _ptr(st))
    names = ("raw_unique", "canonical_unique", "significant", "insignificant", "s_insig",
             "d_selected", "s_max", "kept")
    stats = {k: int(v) for k, v in zip(names, st)}
    return OracleTree(circ, t, nl, ev_off, slot[:ne], qub[:ne], pau[:ne], cnt[:nl], sh[:nl],
                      wn[:nl], wd[:nl], stats, h)


COUNTER_NAMES = ("fwd_gates", "inv_gates", "fwd_paulis", "inv_paulis", "resets", "leaves",
                 "draws", "ret_gates", "ret_paulis", "checkpoint_saves", "checkpoint_restores",
                 "mcm_edges", "paper_ops")
TRAVERSAL = {"dftt": 0, "naive": 1, "hybrid": 2, "checkpoint": 3}


def run(circ, tree: OracleTree, seed: int, traversal: str = "dftt", leaf_begin: int = 0,
        leaf_end: int = 0, want_dist: bool = True, want_samples: bool = True,
        checkpoint_slots: int = 0):
    """Walk the tree: returns (dist or None, samples or None, counters dict,
    per-leaf norms).  checkpoint_slots bounds the states the checkpoint
    traversal keeps (0 = no bound)."""
    h = _CircuitHandle(circ)
    lib().oc_set_checkpoint_slots(C.c_uint64(checkpoint_slots))
    le = leaf_end or tree.n_leaves
    dist = np.zeros(1 << circ.n, np.float64) if want_dist else None
    nshots = int(tree.shots[leaf_begin:le].sum())
    samples = np.zeros(max(nshots, 1), np.uint64) if want_samples else None
    ctr = np.zeros(len(COUNTER_NAMES), np.uint64)
    norms = np.zeros(max(le - leaf_begin, 1), np.float64)
    rc = lib().oc_run(h.ref, C.c_void_p(tree.handle), C.c_uint64(seed),
                      C.c_int(TRAVERSAL[traversal]), C.c_uint64(leaf_begin), C.c_uint64(le),
                      _ptr(dist) if dist is not None else None,
                      _ptr(samples) if samples is not None else None, _ptr(ctr), _ptr(norms))
    if rc:
        raise ValueError("oracle run failed")
    counters = {k: int(v) for k, v in zip(COUNTER_NAMES, ctr)}
    return dist, (samples[:nshots] if samples is not None else None), counters, \
        norms[: le - leaf_begin]


def run_with_margins(circ, tree: OracleTree, seed: int, traversal: str = "dftt",
                     leaf_begin: int = 0, leaf_end: int = 0, want_dist: bool = True):
    """run() with samples, also returning each draw's margin to the nearer
    CDF boundary of its index: (dist or None, samples, margins, counters,
    norms)."""
    h = _CircuitHandle(circ)
    lib().oc_set_checkpoint_slots(C.c_uint64(0))
    le = leaf_end or tree.n_leaves
    dist = np.zeros(1 << circ.n, np.float64) if want_dist else None
    nshots = int(tree.shots[leaf_begin:le].sum())
    samples = np.zeros(max(nshots, 1), np.uint64)
    margins = np.zeros(max(nshots, 1), np.float64)
    ctr = np.zeros(len(COUNTER_NAMES), np.uint64)
    norms = np.zeros(max(le - leaf_begin, 1), np.float64)
    rc = lib().oc_run_margins(h.ref, C.c_void_p(tree.handle), C.c_uint64(seed),
                              C.c_int(TRAVERSAL[traversal]), C.c_uint64(leaf_begin),
                              C.c_uint64(le), _ptr(dist) if dist is not None else None,
                              _ptr(samples), _ptr(margins), _ptr(ctr), _ptr(norms))
    if rc:
        raise ValueError("oracle run failed")
    counters = {k: int(v) for k, v in zip(COUNTER_NAMES, ctr)}
    return dist, samples[:nshots], margins[:nshots], counters, norms[: le - leaf_begin]


def run_mcm(circ, tree: OracleTree, seed: int, cache_capacity: int, leaf_begin: int = 0,
            leaf_end: int = 0, want_dist: bool = True, want_samples: bool = True):
    """DFTT+Caching over a tree whose circuit has measurement layers (Sec.
    III-B.2) with a LIFO cache of `cache_capacity` pre-measurement states
    (0: every leaf from the root).  Returns (dist or None, samples or None,
    counters dict, most states cached at once).  Checkpoint saves/restores
    count cache pushes/fetches; paper_ops is the operation count of Eq. (3)."""
    h = _CircuitHandle(circ)
    le = leaf_end or tree.n_leaves
    dist = np.zeros(1 << circ.n, np.float64) if want_dist else None
    nshots = int(tree.shots[leaf_begin:le].sum())
    samples = np.zeros(max(nshots, 1), np.uint64) if want_samples else None
    ctr = np.zeros(len(COUNTER_NAMES), np.uint64)
    st = np.zeros(1, np.uint64)
    rc = lib().oc_run_mcm(h.ref, C.c_void_p(tree.handle), C.c_uint64(seed),
                          C.c_uint32(cache_capacity), C.c_uint64(leaf_begin), C.c_uint64(le),
                          _ptr(dist) if dist is not None else None,
                          _ptr(samples) if samples is not None else None, _ptr(ctr), _ptr(st))
    if rc:
        raise ValueError(f"oracle measurement walk failed ({rc})")
    counters = {k: int(v) for k, v in zip(COUNTER_NAMES, ctr)}
    return dist, (samples[:nshots] if samples is not None else None), counters, int(st[0])


def uniform53(seed: int, sub: int, primary: int, aux: int, stream: int, half: int = 0) -> float:
    """(v >> 11) 2^-53 of one Philox draw with counter (sub, primary, aux,
    stream) and key seed."""
    return float(lib().oc_uniform53(C.c_uint64(seed), C.c_uint32(sub), C.c_uint32(primary),
                                    C.c_uint32(aux), C.c_uint32(stream), C.c_int(half)))


def leaf_margins(circ, state: np.ndarray, seed: int, leaf: int, shots: int):
    h = _CircuitHandle(circ)
    st = np.ascontiguousarray(state, dtype=np.complex128)
    idx = np.zeros(max(shots, 1), np.uint64)
    mar = np.zeros(max(shots, 1), np.float64)
    lib().oc_leaf_margins(h.ref, _ptr(st), C.c_uint64(seed), C.c_uint64(leaf),
                          C.c_uint64(shots), _ptr(idx), _ptr(mar))
    return idx[:shots], mar[:shots]
