"""Pins of the oracle's walk over circuits with mid-circuit measurement
layers (non-invertible edges, Sec. III-B.2): the DFTT+Caching result for
every cache capacity equals a per-shot definition written here with NumPy
operators, closed forms, the density matrix (statistically), and the
operation counts of Eq. (3) obey their invariants."""

import math

import numpy as np
import pytest

import oracle
from oracle import dms
from workloads import Circuit, random_small_circuit, syndrome_rounds
from workloads.circuits import depol1, depol2


def _patterns(n, qubits):
    idx = np.arange(1 << n)
    pat = np.zeros(1 << n, dtype=np.int64)
    for b, q in enumerate(qubits):
        pat |= ((idx >> q) & 1) << b
    return pat


def _per_shot_definition(c, t, seed):
    """Average over every shot of |psi|^2, each shot simulated alone: its
    leaf's events before the gate of their slot, and at the k-th measurement
    layer its own outcome: u from stream 3 with counter (shot, leaf, k), the
    first o with u * T < P_0 + ... + P_o, projection, renormalisation and, for
    MR, the measured qubits returned to 0."""
    n, G, N = c.n, c.n_gates, 1 << c.n
    S = int(t.shots.sum())
    mats = {}
    for g in range(G):
        if c.kinds[g] not in ("M", "MR"):
            mats[g] = dms.gate_full(n, c.kinds[g], c.qubits[g], c.params[g])
    paulis = {}
    layer_of = {}
    for g in range(G):
        if c.kinds[g] in ("M", "MR"):
            layer_of[g] = len(layer_of)
    dist = np.zeros(N)
    for leaf in range(t.n_leaves):
        ev = t.events(leaf)
        for j in range(int(t.shots[leaf])):
            psi = np.zeros(N, dtype=np.complex128)
            psi[0] = 1.0
            e = 0
            for g in range(G + 1):
                while e < len(ev) and ev[e][0] == g:
                    key = (ev[e][1], ev[e][2])
                    if key not in paulis:
                        paulis[key] = dms.pauli_full(n, [key])
                    psi = paulis[key] @ psi
                    e += 1
                if g == G:
                    break
                if g in mats:
                    psi = mats[g] @ psi
                    continue
                qs = c.qubits[g]
                pat = _patterns(n, qs)
                P = np.bincount(pat, weights=np.abs(psi) ** 2, minlength=1 << len(qs))
                u = oracle.uniform53(seed, j, leaf, layer_of[g], 3, 0)
                cum = np.cumsum(P)
                o = int(np.argmax(u * cum[-1] < cum))
                new = np.where(pat == o, psi, 0.0) / math.sqrt(P[o])
                if c.kinds[g] == "MR":
                    flip = sum(1 << q for b, q in enumerate(qs) if (o >> b) & 1)
                    new = new[np.arange(N) ^ flip]
                psi = new
            dist += np.abs(psi) ** 2 / S
    return dist


def _mcm_random(seed):
    c = random_small_circuit(4, 12, seed, p1=0.04, p2=0.06)
    c.add_measure((1,), reset=False)
    for g in range(8):
        k = ("RX", "CX", "H", "RY")[g % 4]
        if k == "CX":
            c.add("CX", (g % 4, (g + 1) % 4), (), depol2(0.06))
        else:
            c.add(k, (g % 4,), (0.3 * g + 0.2,) if k != "H" else (), depol1(0.04))
    c.add_measure((0, 2), reset=True)
    c.add("U3", (3,), (0.4, 0.1, 0.9), depol1(0.04))
    c.add("CX", (3, 0), (), depol2(0.06))
    return c


@pytest.mark.parametrize("fam", ["syndrome", "random"])
@pytest.mark.parametrize("K", [0, 1, 2, 3])
def test_walk_equals_per_shot_definition(fam, K):
    c = syndrome_rounds(3, 3, 0.02, 0.05, theta=0.7) if fam == "syndrome" else _mcm_random(5)
    S, seed = 600, 17
    t = oracle.ecm(c, S, seed, prune=False)
    want = _per_shot_definition(c, t, seed)
    dist, samples, ct, held = oracle.run_mcm(c, t, seed, K)
    np.testing.assert_allclose(dist, want, atol=1e-12)
    assert held <= min(K, c.n_measure_layers)
    assert ct["draws"] == S and len(samples) == S
    if K == 0:
        assert ct["inv_gates"] + ct["inv_paulis"] == 0


def test_capacity_changes_work_not_results():
    c = syndrome_rounds(3, 4, 0.02, 0.05, theta=0.9)
    S, seed = 1500, 3
    t = oracle.ecm(c, S, seed, prune=False)
    M = c.n_measure_layers
    runs = [oracle.run_mcm(c, t, seed, K) for K in range(M + 2)]
    ref = runs[0]
    ops = [r[2]["paper_ops"] for r in runs]
    for d, smp, ct, held in runs[1:]:
        np.testing.assert_allclose(d, ref[0], atol=1e-12)
        assert np.array_equal(smp, ref[1])          # same walk order, same draws
        assert ct["leaves"] == ref[2]["leaves"]
        assert ct["checkpoint_restores"] >= ct["checkpoint_saves"]
    # Eq. (3): N_1 = ops with DFTT off (K = 0), N_2 = ops with every
    # pre-measurement node cached; alpha rises to 1 with K
    assert all(a >= b for a, b in zip(ops, ops[1:]))
    assert ops[M] == ops[M + 1] and ops[0] > ops[M]
    alpha = [(ops[0] - x) / (ops[0] - ops[M]) for x in ops]
    assert alpha[0] == 0.0 and alpha[M] == 1.0
    assert runs[0][2]["checkpoint_saves"] == 0
    assert runs[0][2]["resets"] == runs[0][2]["leaves"]


def test_deterministic_outcomes_keep_the_tree_and_count_naive_ops():
    """Without the RY the syndrome circuit is a stabiliser circuit: every
    outcome is fixed by the errors, so each tree leaf stays one final leaf
    and DFTT-off costs, per leaf, its 1-qubit tokens + 4 per CX + one per
    measurement edge."""
    c = syndrome_rounds(3, 3, 0.02, 0.05, theta=0.0)
    S, seed = 2000, 8
    t = oracle.ecm(c, S, seed, prune=False)
    _, _, ct, _ = oracle.run_mcm(c, t, seed, 0, want_samples=False)
    assert ct["leaves"] == t.n_leaves
    M = c.n_measure_layers
    n_cx = sum(1 for k in c.kinds if k == "CX")
    n_1q = sum(1 for k in c.kinds if k not in ("CX", "M", "MR"))
    want = sum(n_1q + 4 * n_cx + len(t.events(l)) + M for l in range(t.n_leaves))
    assert ct["paper_ops"] == want
    assert ct["mcm_edges"] == M * t.n_leaves


@pytest.mark.parametrize("reset", [False, True])
def test_bell_measurement_closed_form(reset):
    c = Circuit(2)
    c.add("H", (0,))
    c.add("CX", (0, 1))
    c.add_measure((0,), reset=reset)
    S = 4000
    t = oracle.ecm(c, S, 2, prune=False)
    assert t.n_leaves == 1
    dist, samples, ct, _ = oracle.run_mcm(c, t, 2, 1)
    one = 2 if reset else 3       # |1>_1 |0>_0 after a reset, else |11>
    assert ct["leaves"] == 2 and ct["mcm_edges"] == 2
    assert dist[0] + dist[one] == pytest.approx(1.0, abs=1e-14)
    assert all(dist[i] == 0.0 for i in range(4) if i not in (0, one))
    assert abs(dist[0] - 0.5) < 5 * math.sqrt(0.25 / S)
    # every sample is the outcome its branch fixed
    assert set(np.unique(samples)) <= {0, one}
    assert np.count_nonzero(samples == 0) == round(dist[0] * S)


def test_measurement_layers_match_density_matrix():
    c = syndrome_rounds(2, 3, 0.03, 0.06, theta=1.1)
    S = 40_000
    t = oracle.ecm(c, S, 11, prune=False)
    dist, _, _, _ = oracle.run_mcm(c, t, 11, 2, want_samples=False)
    rho = dms.density_matrix(c)
    p = np.real(np.diag(rho))
    sig = np.sqrt(p * (1 - p) / S) + 1e-12
    assert np.all(np.abs(dist - p) < 6 * sig + 1e-3)


def test_errors_stop_at_a_measurement_of_their_qubit():
    c = Circuit(3)
    c.add("H", (0,), (), (0.1, 0.1, 0.1))
    c.add_measure((0,), reset=True)
    c.add("RX", (0,), (0.4,))
    c.add("X", (1,), (), (0.1, 0.1, 0.1))
    c.add_measure((2,), reset=True)
    c.add("X", (1,))
    # an X after H on qubit 0 meets the measurement: reported just before it
    assert oracle.commute(c, [0], [1]) == [(1, 0, 1)]
    # a Z after X on qubit 1 passes the noiseless X (rule 2) and the
    # measurement of qubit 2 (another qubit): it ends after the last gate
    assert oracle.commute(c, [1], [3]) == [(6, 1, 3)]


def test_plain_traversals_refuse_measurement_layers():
    c = syndrome_rounds(2, 1, 0.01, 0.01)
    t = oracle.ecm(c, 100, 1, prune=False)
    with pytest.raises(ValueError):
        oracle.run(c, t, 1)
    tp = oracle.ecm(c, 100, 1, prune=True, alpha=(1, 2), beta=1)
    if any(tp.shots != tp.count):
        with pytest.raises(ValueError):
            oracle.run_mcm(c, tp, 1, 1)
