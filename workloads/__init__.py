"""Seeded synthetic workloads for the noisy-simulation engine and its oracle.

This package only *describes* circuits: gate lists, rotation angles and the
probabilities of the Pauli noise channels attached to gates.  It contains none
of the simulation method's arithmetic (no error sampling, no commutation, no
statevector math), so both the GPU engine's binding and the CPU oracle can take
its output as their common input.

Families (the paper evaluates on a benchmark suite that is not available here;
these two synthetic families stand in for it and span the two extremes for the
error-characterisation stages):

* random brickwork: U3 on every qubit with uniform angles, then CX on
  alternating nearest-neighbour pairs of a linear chain;
* Trotterised transverse-field Ising chain: RZZ(theta) on neighbours
  (decomposed as CX, RZ, CX) followed by RX on every qubit.

Noise is the depolarising Pauli channel of the paper's Section II (1-qubit:
X/Y/Z each with p/3) and its 2-qubit analogue (the 15 non-identity two-qubit
Paulis each with p/15), attached after the gate it follows.
"""

from .circuits import (  # noqa: F401
    GATE_NAMES,
    MEASURE_KINDS,
    Circuit,
    brickwork,
    ising,
    bell_pair,
    batch_job_params,
    batch_jobs,
    serving_requests,
    random_small_circuit,
    syndrome_rounds,
)
