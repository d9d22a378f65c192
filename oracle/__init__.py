"""CPU oracle for the noisy-simulation pipeline -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU engine never calls it and
shares no code with it.

``tusq_oracle.c`` holds the plain C implementation (complex128 statevector,
literal per-qubit-stack error commutation, left-to-right FP64 sums);
``dms.py`` holds an independent NumPy density-matrix simulator used only to
pin the oracle for tiny qubit counts.
"""

from .oracle import (  # noqa: F401
    KIND_CODES,
    OracleTree,
    apportion,
    bounded,
    build_library,
    commute,
    ecm,
    leaf_margins,
    lib,
    philox,
    prune_select,
    roundtrip,
    run,
    run_mcm,
    run_with_margins,
    sample_shot,
    set_threads,
    thermal_probs,
    thresholds,
    trajectory,
    uniform53,
)
