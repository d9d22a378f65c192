"""Writes ``ising30_leaves_1_3.json``: what the oracle computes for the
depth-first leaves [1, 3) of the 30-qubit noisy Trotter-Ising workload (20
steps of CX-RZ(0.1)-CX on neighbours and RX(0.2) on every qubit, 1-qubit
depolarising p = 5e-4 after each RZ and RX, 2-qubit p = 5e-3 after each CX,
10^6 shots, seed 2, pruned tree with alpha = 1/100 and beta = 100), walked
with plain DFTT in complex128 (Sec. III-B).  A complex128 state of 2^30
amplitudes is 16 GiB and the walk takes the better part of an hour on a
few cores, so the GPU test reads these stored figures instead of running
the oracle:

* the SHA-256 of the oracle's serialised tree (the engine's must match);
* the walk's counters and per-leaf FP64 norms;
* the 30 one-qubit marginals P(bit q = 1) and the total of the distribution;
* the probabilities at 4096 seeded random indices and at the 64 largest;
* every sample of the two leaves with the draws whose margin to a CDF
  boundary is below 1e-9 (the margin rule excuses those below 1e-11).

Only ``oracle/`` computes; ``workloads`` supplies the circuit.  Run from
the repository root:  python tests/golden/make_ising30_golden.py [threads]
"""

import base64
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from workloads import ising  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "ising30_leaves_1_3.json")
N_QUBITS, STEPS, P1, P2, SHOTS, SEED = 30, 20, 5e-4, 5e-3, 1_000_000, 2
LB, LE = 1, 3
PROBE_SEED, N_PROBE, N_TOP, SMALL_MARGIN = 12345, 4096, 64, 1e-9


def b64(a: np.ndarray) -> str:
    return base64.b64encode(np.ascontiguousarray(a).tobytes()).decode()


def main() -> None:
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 1)
    oracle.set_threads(threads)
    c = ising(N_QUBITS, STEPS, P1, P2)
    t0 = time.time()
    ot = oracle.ecm(c, SHOTS, SEED)
    tree_hash = hashlib.sha256(ot.serialize()).hexdigest()
    print(f"ecm {time.time() - t0:.1f}s, {ot.n_leaves} leaves", flush=True)
    t0 = time.time()
    dist, samples, margins, counters, norms = oracle.run_with_margins(
        c, ot, SEED, leaf_begin=LB, leaf_end=LE)
    print(f"walk {time.time() - t0:.1f}s", flush=True)
    marg = []
    for q in range(N_QUBITS):
        v = dist.reshape(1 << (N_QUBITS - q - 1), 2, 1 << q)[:, 1, :].sum()
        marg.append(float(v))
    rng = np.random.default_rng(PROBE_SEED)
    probe = np.unique(rng.integers(0, 1 << N_QUBITS, N_PROBE, dtype=np.uint64))
    top = np.argsort(dist)[-N_TOP:].astype(np.uint64)
    idx = np.concatenate([probe, top])
    small = np.nonzero(margins < SMALL_MARGIN)[0]
    rec = {
        "workload": {"family": "ising", "n": N_QUBITS, "steps": STEPS, "p1": P1, "p2": P2,
                     "shots": SHOTS, "seed": SEED, "alpha": [1, 100], "beta": 100,
                     "traversal": "dftt", "leaf_begin": LB, "leaf_end": LE},
        "n_leaves": int(ot.n_leaves),
        "tree_sha256": tree_hash,
        "shots": [int(x) for x in ot.shots[LB:LE]],
        "counters": counters,
        "norms": [float(x).hex() for x in norms],
        "total": float(dist.sum()).hex(),
        "marginals": [x.hex() for x in marg],
        "index_u64_b64": b64(idx.astype("<u8")),
        "prob_f64_b64": b64(dist[idx].astype("<f8")),
        "samples_u32_b64": b64(samples.astype("<u4")),
        "small_margin_positions": [int(i) for i in small],
        "small_margins": [float(margins[i]).hex() for i in small],
    }
    with open(OUT, "w") as f:
        json.dump(rec, f, indent=1)
    print(f"wrote {OUT}: {len(samples)} samples, {len(small)} draws with margin < "
          f"{SMALL_MARGIN}", flush=True)


if __name__ == "__main__":
    main()
