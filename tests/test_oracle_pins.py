"""Pins for the CPU oracle: each test checks it against something that does
not come from the oracle itself (published RNG vectors, the paper's worked
numbers and closed forms, density-matrix simulation, brute-force operator
identities, exact enumeration)."""

import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import dms
from workloads import Circuit, bell_pair, brickwork, random_small_circuit
from workloads.circuits import depol1, depol2

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


def _read_golden(golden_dir, name):
    rows = []
    with open(f"{golden_dir}/{name}") as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


# --------------------------------------------------------------------------
# Random numbers and channel thresholds

def test_philox_known_answer_vectors(golden_dir):
    rows = _read_golden(golden_dir, "philox4x32_10_kat.txt")
    assert len(rows) == 3
    for r in rows:
        vals = [int(x, 16) for x in r]
        assert oracle.philox(vals[0:4], vals[4:6]) == tuple(vals[6:10])


def test_thresholds_exact_and_identity():
    assert oracle.thresholds([0.0, 0.0, 0.0]) == [0, 0, 0]
    # 0.25 is exact in binary: C = 2^62 * k
    assert oracle.thresholds([0.25, 0.25, 0.25]) == [1 << 62, 2 << 62, 3 << 62]
    assert oracle.thresholds([0.5, 0.5]) == [1 << 63, 2**64 - 1]


def _single_channel_counts(p, shots, seed):
    c = Circuit(1)
    c.add("H", (0,), (), depol1(p))
    t = oracle.ecm(c, shots, seed, do_commute=False, prune=False)
    counts = {0: 0, 1: 0, 2: 0, 3: 0}
    for leaf in range(t.n_leaves):
        ev = t.events(leaf)
        counts[ev[0][2] if ev else 0] += int(t.count[leaf])
    return counts


def test_worked_sampling_example_frequencies(golden_dir):
    row = [r for r in _read_golden(golden_dir, "closed_forms.txt") if r[0] == "depol_example"][0]
    S = 200_000
    counts = _single_channel_counts(0.1, S, seed=11)
    exp = {0: 0.9, 1: 0.1 / 3, 2: 0.1 / 3, 3: 0.1 / 3}
    assert "I=0.9" in row
    for k, p in exp.items():
        sigma = math.sqrt(S * p * (1 - p))
        assert abs(counts[k] - S * p) < 5 * sigma, (k, counts[k], S * p)


def test_zero_noise_gives_single_noiseless_leaf():
    c = brickwork(4, 3, 0.0, 0.0, seed=1)
    c2 = Circuit(4)
    for k, q, p in zip(c.kinds, c.qubits, c.params):
        c2.add(k, q, p, depol1(0.0) if len(q) == 1 else depol2(0.0))
    t = oracle.ecm(c2, 1000, seed=5)
    assert t.n_leaves == 1 and t.events(0) == [] and int(t.count[0]) == 1000
    dist, _, _, _ = oracle.run(c2, t, seed=5, want_samples=False)
    psi = dms.circuit_unitary(c)[:, 0]
    np.testing.assert_allclose(dist, np.abs(psi) ** 2, atol=1e-13)


def test_hamming_weight_histogram_matches_binomial():
    # Fig. 2C set-up: ERs of length 20 at p = 1%.
    C, p, S = 20, 0.01, 100_000
    c = Circuit(20)
    for q in range(C):
        c.add("U3", (q,), (0.3, 0.2, 0.1), depol1(p))
    t = oracle.ecm(c, S, seed=3, do_commute=False, prune=False)
    shot, _, _ = t.raw_events()
    w = np.bincount(np.bincount(shot, minlength=S), minlength=8)
    for k in range(5):
        pk = math.comb(C, k) * p ** k * (1 - p) ** (C - k)
        sigma = math.sqrt(S * pk * (1 - pk)) + 1
        assert abs(w[k] - S * pk) < 5 * sigma, (k, w[k], S * pk)
    # the paper calls weight > 2 "zero"; the binomial value is ~1.0e-3
    tail = 1 - sum(math.comb(C, k) * p ** k * (1 - p) ** (C - k) for k in range(3))
    assert 0.9e-3 < tail < 1.1e-3
    assert abs(w[3:].sum() - S * tail) < 5 * math.sqrt(S * tail) + 1


def test_er_draws_are_per_shot_reproducible():
    c = brickwork(5, 4, 0.05, 0.1, seed=2)
    t = oracle.ecm(c, 300, seed=99, do_commute=False, prune=False)
    shot, chan, out = t.raw_events()
    for j in (0, 17, 299):
        ch, o = oracle.sample_shot(c, 99, j)
        np.testing.assert_array_equal(ch, chan[shot == j])
        np.testing.assert_array_equal(o, out[shot == j])


# --------------------------------------------------------------------------
# Commutation rules (Sec. III-A.2, rules 1-6), checked by matrix products

def _pauli_of(m2):
    """Identify a 4x4 matrix as phase * (P_a on qubit 0 (x) P_b on qubit 1)."""
    for a in range(4):
        for b in range(4):
            P = dms.pauli_full(2, [(0, a), (1, b)])
            if dms.equal_up_to_phase(m2, P):
                return a, b
    return None


def test_cx_conjugation_table_matches_matrix_products():
    CX = dms.cx_full(2, 0, 1)
    for a in range(4):
        for b in range(4):
            if a == 0 and b == 0:
                continue
            P = dms.pauli_full(2, [(0, a), (1, b)])
            want = _pauli_of(CX @ P @ CX.conj().T)
            assert want is not None
            # circuit: noisy U3 on q0 and q1, noiseless CX, then blocking U3s
            c = Circuit(2)
            c.add("U3", (0,), (0.1, 0.2, 0.3), depol1(0.1))
            c.add("U3", (1,), (0.4, 0.5, 0.6), depol1(0.1))
            c.add("CX", (0, 1))
            c.add("U3", (0,), (0.7, 0.8, 0.9))
            c.add("U3", (1,), (1.0, 1.1, 1.2))
            chan, outc = [], []
            if a:
                chan.append(0); outc.append(a)
            if b:
                chan.append(1); outc.append(b)
            ev = oracle.commute(c, chan, outc)
            got = {q: p for (_, q, p) in ev}
            assert (got.get(0, 0), got.get(1, 0)) == want, (a, b)
            for s, q, _ in ev:
                assert s == 3 + q  # blocked right before the U3 on its qubit


@pytest.mark.parametrize("rot", ["RX", "RY", "RZ"])
def test_axis_rules_and_blocking(rot):
    theta = 0.7
    R = dms.gate_2x2(rot, [theta])
    axis = {"RX": 1, "RY": 2, "RZ": 3}[rot]
    for p in (1, 2, 3):
        commutes = np.allclose(R @ dms.PAULIS[p] @ R.conj().T, dms.PAULIS[p])
        assert commutes == (p == axis)
        c = Circuit(1)
        c.add("H", (0,), (), depol1(0.1))
        c.add(rot, (0,), (theta,))
        c.add("H", (0,))
        ev = oracle.commute(c, [0], [p])
        assert ev == [(2 if commutes else 1, 0, p)]


def test_paulis_pass_noiseless_paulis_and_others_block():
    for g in ("X", "Y", "Z"):
        c = Circuit(1)
        c.add("U3", (0,), (0.1, 0.2, 0.3), depol1(0.1))
        c.add(g, (0,))
        for p in (1, 2, 3):
            assert oracle.commute(c, [0], [p]) == [(2, 0, p)]
    for g in ("U3", "H", "S", "SDG", "T", "TDG"):
        c = Circuit(1)
        c.add("H", (0,), (), depol1(0.1))
        c.add(g, (0,), (0.3, 0.2, 0.1))
        assert oracle.commute(c, [0], [1]) == [(1, 0, 1)]


def test_merge_rule_and_identity_vanishes():
    c = Circuit(1)
    c.add("U3", (0,), (0.1, 0.2, 0.3), depol1(0.1))
    c.add("X", (0,), (), depol1(0.1))
    c.add("Z", (0,), (), depol1(0.1))
    assert oracle.commute(c, [0, 1], [1, 3]) == [(3, 0, 2)]  # X then Z -> Y
    assert oracle.commute(c, [0, 1], [2, 2]) == []            # Y Y = I


def test_fig4b_example_merges():
    # H then CX, errors X after H versus XX after CX: same canonical ER.
    c = bell_pair(0.1, 0.1)
    e1 = oracle.commute(c, [0], [1])
    e2 = oracle.commute(c, [1], [4 * 1 + 1])
    assert e1 == e2 == [(2, 0, 1), (2, 1, 1)]


def test_fig4c_example_does_not_merge():
    # X through RZ(theta) would become RZ(-theta): the X must stay put.
    theta = 0.9
    RZ = dms.gate_2x2("RZ", [theta])
    RZm = dms.gate_2x2("RZ", [-theta])
    np.testing.assert_allclose(dms.PX @ RZ, RZm @ dms.PX, atol=1e-14)
    c = Circuit(1)
    c.add("H", (0,), (), depol1(0.1))
    c.add("RZ", (0,), (theta,), depol1(0.1))
    c.add("H", (0,))
    assert oracle.commute(c, [0], [1]) == [(1, 0, 1)]
    assert oracle.commute(c, [1], [1]) == [(2, 0, 1)]
    assert oracle.commute(c, [0, 1], [1, 1]) == [(1, 0, 1), (2, 0, 1)]


@pytest.mark.parametrize("seed", range(12))
def test_commuted_er_is_the_same_operator(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 5))
    kinds = ("U3", "RX", "RY", "RZ", "H", "S", "T", "X", "Y", "Z", "CX", "CX", "CX")
    c = random_small_circuit(n, int(rng.integers(4, 14)), seed, p1=0.4, p2=0.6, kinds=kinds)
    for shot in range(6):
        chan, outc = oracle.sample_shot(c, seed, shot)
        raw = oracle.commute(c, chan, outc, do_commute=False)
        can = oracle.commute(c, chan, outc, do_commute=True)
        assert dms.equal_up_to_phase(dms.circuit_unitary(c, raw), dms.circuit_unitary(c, can))
        assert len(set((s, q) for s, q, _ in can)) == len(can)
        assert can == sorted(can)


# --------------------------------------------------------------------------
# Statevector and the mixture: density-matrix equality, closed forms

def _small_noisy(seed, n):
    rng = np.random.default_rng(100 + seed)
    c = Circuit(n)
    n1 = 0
    n2 = 0
    for _ in range(7):
        if n >= 2 and rng.random() < 0.3 and n2 < 1:
            a, b = rng.choice(n, 2, replace=False)
            c.add("CX", (int(a), int(b)), (), depol2(0.2))
            n2 += 1
        else:
            k = ["U3", "RX", "RY", "RZ", "H", "S", "T", "SDG", "TDG"][int(rng.integers(9))]
            noisy = n1 < 4
            c.add(k, (int(rng.integers(n)),), rng.random(3) * 6.28,
                  depol1(0.3) if noisy else None)
            n1 += noisy
    return c


@pytest.mark.parametrize("seed", range(6))
def test_weighted_trajectories_equal_density_matrix(seed):
    n = 2 + seed % 3
    c = _small_noisy(seed, n)
    rho = dms.density_matrix(c)
    mix = np.zeros(1 << n)
    wsum = 0.0
    for p, ev in dms.enumerate_ers(c):
        psi = oracle.trajectory(c, ev)
        mix += p * np.abs(psi) ** 2
        wsum += p
        # the commuted ER gives the same distribution
        if p > 0 and ev:
            chan = []
            outc = []
            gch = {g: i for i, g in enumerate(g for g, x in enumerate(c.noise) if x is not None)}
            per_gate = {}
            for s, q, pa in ev:
                per_gate.setdefault(s - 1, {})[q] = pa
            for g, qp in sorted(per_gate.items()):
                qs = c.qubits[g]
                if len(qs) == 1:
                    k = qp[qs[0]]
                else:
                    k = 4 * qp.get(qs[0], 0) + qp.get(qs[1], 0)
                chan.append(gch[g]); outc.append(k)
            can = oracle.commute(c, chan, outc)
            np.testing.assert_allclose(np.abs(oracle.trajectory(c, can)) ** 2,
                                       np.abs(psi) ** 2, atol=1e-12)
    assert abs(wsum - 1.0) < 1e-12
    np.testing.assert_allclose(mix, np.real(np.diag(rho)), atol=1e-12)


def test_noiseless_trajectory_matches_kron_unitary():
    for seed in range(5):
        c = random_small_circuit(4, 25, seed, p1=0, p2=0)
        psi = oracle.trajectory(c, [])
        want = dms.circuit_unitary(c)[:, 0]
        np.testing.assert_allclose(psi, want, atol=1e-13)


@pytest.mark.parametrize("p", [0.0, 0.01, 0.3, 0.9])
def test_bell_closed_form(p, golden_dir):
    c = bell_pair(0.0, p) if p > 0 else bell_pair(0.0, 0.0)
    mix = np.zeros(4)
    for pr, ev in dms.enumerate_ers(c):
        mix += pr * np.abs(oracle.trajectory(c, ev)) ** 2
    want = np.array([(1 - 8 * p / 15) / 2, 4 * p / 15, 4 * p / 15, (1 - 8 * p / 15) / 2])
    np.testing.assert_allclose(mix, want, atol=1e-14)


@pytest.mark.parametrize("p", [0.05, 0.5])
def test_h_depolarizing_is_half_half(p):
    c = Circuit(1)
    c.add("H", (0,), (), depol1(p))
    mix = np.zeros(2)
    for pr, ev in dms.enumerate_ers(c):
        mix += pr * np.abs(oracle.trajectory(c, ev)) ** 2
    np.testing.assert_allclose(mix, [0.5, 0.5], atol=1e-15)
    # and through the whole pipeline with sampled ERs
    t = oracle.ecm(c, 5000, seed=1, prune=False)
    dist, _, _, _ = oracle.run(c, t, seed=1, want_samples=False)
    np.testing.assert_allclose(dist, [0.5, 0.5], atol=1e-14)


def test_norm_preserved_and_uncompute_returns():
    c = brickwork(6, 8, 0.05, 0.05, seed=4)
    t = oracle.ecm(c, 500, seed=4, prune=False)
    for leaf in range(0, t.n_leaves, max(1, t.n_leaves // 7)):
        ev = t.events(leaf)
        psi = oracle.trajectory(c, ev)
        assert abs(np.vdot(psi, psi).real - 1.0) < 1e-13
        for depth in (0, 5, 40, c.n_gates // 2, c.n_gates + len(ev)):
            assert oracle.roundtrip(c, ev, depth) <= 1e-12


# --------------------------------------------------------------------------
# The pipeline: lossless result equals the plain definition; modes agree

def _definition_distribution(c, S, seed):
    """(1/S) sum over shots of |U_{e_j}|0>|^2, each shot's raw ER placed
    right after its gate (no tallying, no commutation, no tree)."""
    t = oracle.ecm(c, S, seed, do_commute=False, prune=False)
    shot, chan, outc = t.raw_events()
    per = {}
    for j in range(S):
        m = shot == j
        key = tuple(zip(chan[m].tolist(), outc[m].tolist()))
        per[key] = per.get(key, 0) + 1
    acc = np.zeros(1 << c.n)
    for key, cnt in per.items():
        ev = oracle.commute(c, [k[0] for k in key], [k[1] for k in key], do_commute=False)
        acc += cnt * np.abs(oracle.trajectory(c, ev)) ** 2
    return acc / S


@pytest.mark.parametrize("fam", ["brick", "random"])
def test_lossless_pipeline_equals_definition(fam):
    if fam == "brick":
        c = brickwork(5, 6, 0.02, 0.05, seed=8)
    else:
        c = random_small_circuit(5, 40, 8, p1=0.03, p2=0.05)
    S, seed = 3000, 21
    want = _definition_distribution(c, S, seed)
    for commute in (False, True):
        t = oracle.ecm(c, S, seed, do_commute=commute, prune=False)
        assert int(t.count.sum()) == S
        for trav in ("dftt", "naive", "hybrid", "checkpoint"):
            dist, _, _, _ = oracle.run(c, t, seed, traversal=trav, want_samples=False)
            np.testing.assert_allclose(dist, want, atol=1e-12)
        for slots in (1, 2):
            dist, _, _, _ = oracle.run(c, t, seed, traversal="checkpoint", want_samples=False,
                                       checkpoint_slots=slots)
            np.testing.assert_allclose(dist, want, atol=1e-12)


def test_commutation_only_merges():
    c = random_small_circuit(5, 60, 3, p1=0.03, p2=0.05,
                             kinds=("RX", "RZ", "CX", "CX", "X", "H"))
    t0 = oracle.ecm(c, 4000, 5, do_commute=False, prune=False)
    t1 = oracle.ecm(c, 4000, 5, do_commute=True, prune=False)
    assert t1.n_leaves < t0.n_leaves
    assert t1.stats["raw_unique"] == t0.n_leaves


def test_convergence_to_density_matrix():
    c = brickwork(4, 3, 0.02, 0.06, seed=12)
    rho = np.real(np.diag(dms.density_matrix(c)))
    S = 40_000
    t = oracle.ecm(c, S, seed=77, prune=False)
    dist, _, _, _ = oracle.run(c, t, 77, want_samples=False)
    # each probability is a mean of S bounded per-shot values: within a few sigma/sqrt(S)
    assert np.max(np.abs(dist - rho)) < 5 * 0.5 / math.sqrt(S)


# --------------------------------------------------------------------------
# DFTT operation counts (Sec. III-B.1)

def test_full_bary_tree_counts(golden_dir):
    row = [r for r in _read_golden(golden_dir, "closed_forms.txt") if r[0] == "bary"][0]
    vals = dict(x.split("=") for x in row[1:])
    b, h = int(vals["b"]), int(vals["h"])
    c = Circuit(1)
    for _ in range(h):
        c.add("U3", (0,), (0.3, 0.5, 0.7), depol1(0.75))   # I, X, Y, Z each 1/4
    t = oracle.ecm(c, 20_000, seed=1, prune=False)
    assert t.n_leaves == b ** h == int(vals["Nl"])
    E = sum(b ** k for k in range(1, h + 1))
    assert E == int(vals["E"])
    assert h == round(math.log((b - 1) * E + b, b) - 1)
    assert b ** h == (1 - 1 / b) * E + 1
    _, _, ct, _ = oracle.run(c, t, 1, traversal="dftt", want_dist=False, want_samples=False)
    fwd = ct["fwd_gates"] + ct["fwd_paulis"]
    back = ct["inv_gates"] + ct["inv_paulis"] + ct["ret_gates"] + ct["ret_paulis"]
    # each (gate, outcome) edge is one gate or one Pauli token per sibling
    assert fwd == E and back == E and fwd + back == int(vals["Tdftt"])
    assert t.n_leaves * h == int(vals["Tnaive"])
    _, _, cn, _ = oracle.run(c, t, 1, traversal="naive", want_dist=False, want_samples=False)
    assert cn["resets"] == t.n_leaves and cn["inv_gates"] == 0


def _trie_nodes(c, t, lb=0, le=None):
    le = le or t.n_leaves
    nodes = set()
    for leaf in range(lb, le):
        ev = t.events(leaf)
        toks = []
        e = 0
        for s in range(c.n_gates + 1):
            while e < len(ev) and ev[e][0] == s:
                toks.append(("e",) + ev[e]); e += 1
            if s < c.n_gates:
                toks.append(("g", s))
        for d in range(1, len(toks) + 1):
            nodes.add(tuple(toks[:d]))
    return nodes


def test_dftt_forward_tokens_equal_trie_size():
    c = brickwork(5, 5, 0.03, 0.06, seed=9)
    t = oracle.ecm(c, 2000, seed=9, prune=False)
    nodes = _trie_nodes(c, t)
    _, _, ct, _ = oracle.run(c, t, 9, traversal="dftt", want_dist=False, want_samples=False)
    assert ct["fwd_gates"] + ct["fwd_paulis"] == len(nodes)
    assert ct["inv_gates"] + ct["inv_paulis"] + ct["ret_gates"] + ct["ret_paulis"] == len(nodes)
    _, _, cn, _ = oracle.run(c, t, 9, traversal="naive", want_dist=False, want_samples=False)
    lengths = sum(c.n_gates + len(t.events(l)) for l in range(t.n_leaves))
    assert cn["fwd_gates"] + cn["fwd_paulis"] == lengths
    _, _, chy, _ = oracle.run(c, t, 9, traversal="hybrid", want_dist=False, want_samples=False)
    tot = lambda x: x["fwd_gates"] + x["fwd_paulis"] + x["inv_gates"] + x["inv_paulis"]
    assert tot(chy) <= min(tot(ct), tot(cn))
    # branch checkpoints: the same forward trie walk with every undo replaced
    # by a restore, one save per branching node that still has siblings
    _, _, cc, _ = oracle.run(c, t, 9, traversal="checkpoint", want_dist=False, want_samples=False)
    assert cc["fwd_gates"] + cc["fwd_paulis"] == len(nodes)
    assert cc["inv_gates"] + cc["inv_paulis"] == 0
    assert cc["checkpoint_restores"] == t.n_leaves - 1
    assert 1 <= cc["checkpoint_saves"] <= t.n_leaves - 1


# --------------------------------------------------------------------------
# Pruning (Sec. III-A.4, Eq. (2))

@pytest.mark.parametrize("seed", [1, 2, 3])
def test_pruning_invariants(seed):
    c = brickwork(6, 10, 0.01, 0.03, seed=seed)
    S = 20_000
    tl = oracle.ecm(c, S, seed, prune=False)
    tp = oracle.ecm(c, S, seed, prune=True, alpha=(1, 100), beta=50)
    smax = int(tl.count.max())
    sig = int((100 * tl.count >= smax).sum())
    ins = tl.n_leaves - sig
    assert tp.stats["significant"] == sig and tp.stats["insignificant"] == ins
    assert tp.n_leaves == sig + min(50, ins)                       # Eq. (2)
    assert sum(Fraction(int(a), int(b)) for a, b in zip(tp.wnum, tp.wden)) == 1
    assert int(tp.shots.sum()) == S
    ins_mask = 100 * tp.count < smax
    w_ins = sum(Fraction(int(a), int(b)) for a, b, m in zip(tp.wnum, tp.wden, ins_mask) if m)
    assert w_ins == Fraction(tp.stats["s_insig"], S)
    # leaves kept are a subset of the lossless leaves, in the same order
    lossless = [tuple(tl.events(i)) for i in range(tl.n_leaves)]
    kept = [tuple(tp.events(i)) for i in range(tp.n_leaves)]
    pos = [lossless.index(k) for k in kept]
    assert pos == sorted(pos)
    # apportioned shots are floor or ceil of the exact share
    for a, b, s, m in zip(tp.wnum, tp.wden, tp.shots, ins_mask):
        if m:
            exact = Fraction(int(a), int(b)) * S
            assert math.floor(exact) <= int(s) <= math.ceil(exact)


def test_pruning_off_limits_are_lossless():
    c = brickwork(6, 10, 0.01, 0.03, seed=5)
    S = 5000
    tl = oracle.ecm(c, S, 5, prune=False)
    ta = oracle.ecm(c, S, 5, prune=True, alpha=(0, 100), beta=1)
    tb = oracle.ecm(c, S, 5, prune=True, alpha=(1, 100), beta=10 ** 6)
    assert tl.serialize() == ta.serialize() == tb.serialize()


def test_pruned_keeps_exactly_beta_insignificant():
    c = brickwork(4, 6, 0.02, 0.05, seed=2)
    for s in range(20):
        t = oracle.ecm(c, 3000, 1000 + s, prune=True, alpha=(1, 20), beta=5)
        n_ins = sum(1 for i in range(t.n_leaves) if 20 * int(t.count[i]) < t.stats["s_max"])
        assert n_ins == min(5, t.stats["insignificant"])


# The selection step: the paper asks for beta of the insignificant circuits
# "sampled at random"; read as uniform selection without replacement, every
# beta-subset of the |C_I| positions is equally likely.  These checks hold
# for that reading whatever generator drives it, so a biased shuffle, an
# off-by-one draw range, a repeated position or a modulo bias fails them.

def _chi2_bound(dof, tail=1e-6):
    from scipy.stats import chi2
    return float(chi2.ppf(1.0 - tail, dof))


@pytest.mark.parametrize("nins,beta", [(10, 3), (7, 6), (12, 1)])
def test_prune_selection_uniform_over_subsets(nins, beta):
    seeds = 6000
    subsets = {}
    for seed in range(seeds):
        sel = oracle.prune_select(seed, nins, beta)
        assert sel == sorted(sel) and len(set(sel)) == beta        # no position twice
        assert all(0 <= x < nins for x in sel)
        subsets[tuple(sel)] = subsets.get(tuple(sel), 0) + 1
    k = math.comb(nins, beta)
    assert len(subsets) == k                                        # every subset reachable
    e = seeds / k
    chi2 = sum((subsets.get(sub, 0) - e) ** 2 / e
               for sub in itertools.combinations(range(nins), beta))
    assert chi2 < _chi2_bound(k - 1), chi2
    # each position is kept with probability beta / nins
    p = beta / nins
    for pos in range(nins):
        x = sum(v for sub, v in subsets.items() if pos in sub)
        assert abs(x - seeds * p) < 5 * math.sqrt(seeds * p * (1 - p)), (pos, x)


@pytest.mark.parametrize("m", [3 << 62, (1 << 63) + 1, 7])
def test_bounded_draws_are_uniform(m):
    # m = 3 * 2^62: reducing a 64-bit draw modulo m without rejection puts the
    # values below 2^62 twice as often (probability 1/2 instead of 1/3);
    # m = 2^63 + 1: the lower half gets 3/4 instead of 1/2
    n = 6000
    r = [oracle.bounded(seed, t, m) for seed in range(n // 30) for t in range(30)]
    assert all(0 <= x < m for x in r)
    if m > 1 << 62:
        for cut, p in ((1 << 62, (1 << 62) / m), (m // 2, (m // 2) / m)):
            x = sum(1 for v in r if v < cut)
            assert abs(x - n * p) < 5 * math.sqrt(n * p * (1 - p)), (cut, x, n * p)
    else:
        e = n / m
        chi2 = sum((r.count(v) - e) ** 2 / e for v in range(m))
        assert chi2 < _chi2_bound(m - 1), chi2
    assert oracle.bounded(5, 0, 1) == 0


def test_pipeline_selection_matches_uniform_inclusion():
    # through the whole error characterisation: per seed, the insignificant
    # leaves of the lossless tree (in leaf order) and the ones the pruned
    # tree keeps; rank r of C_I is kept with probability beta / |C_I|
    c = brickwork(2, 2, 0.01, 0.03, seed=2)     # |C_I| of 12 .. 18 leaves
    beta, S = 4, 400
    X, E, V = {}, {}, {}
    runs = 0
    for s in range(2400):
        seed = 7000 + s
        tl = oracle.ecm(c, S, seed, prune=False)
        smax = int(tl.count.max())
        ins = [i for i in range(tl.n_leaves) if 20 * int(tl.count[i]) < smax]
        if len(ins) <= beta:
            continue
        tp = oracle.ecm(c, S, seed, prune=True, alpha=(1, 20), beta=beta)
        lossless = {tuple(tl.events(i)): i for i in range(tl.n_leaves)}
        kept = [lossless[tuple(tp.events(j))] for j in range(tp.n_leaves)]
        kept_ins = [i for i in kept if i in set(ins)]
        assert len(kept_ins) == beta == len(set(kept_ins))
        rank = {i: r for r, i in enumerate(ins)}
        p = beta / len(ins)
        for r in range(len(ins)):
            E[r] = E.get(r, 0.0) + p
            V[r] = V.get(r, 0.0) + p * (1 - p)
        for i in kept_ins:
            X[rank[i]] = X.get(rank[i], 0) + 1
        runs += 1
    assert runs >= 2000
    z2 = 0.0
    for r in E:
        if V[r] < 25:   # ranks seen too rarely for a normal bound
            continue
        z = (X.get(r, 0) - E[r]) / math.sqrt(V[r])
        assert abs(z) < 5, (r, X.get(r, 0), E[r])
        z2 += z * z
    dof = sum(1 for r in E if V[r] >= 25)
    assert z2 < _chi2_bound(dof), (z2, dof)


# The shots of the selected circuits: Eq. (2) shares the insignificant shots
# s_I in proportion to the selected counts; integers by the largest-remainder
# (Hamilton) method, ties to the earlier circuit.

# (s_I, selected counts, shots) worked by hand.  Quotas q_j = s_I s_j / D:
#  10, (1,1,1):  D=3, q = 10/3 each -> floors 3,3,3, one unit left, three equal
#                remainders 1/3 -> the first circuit: 4,3,3
#   8, (1,1,1):  q = 8/3 each -> floors 2,2,2, two left, equal remainders 2/3
#                -> the first two: 3,3,2
#  10, (1,2,4):  D=7, q = 10/7, 20/7, 40/7 -> floors 1,2,5, remainders 3/7,
#                6/7, 5/7, two left -> the second and third: 1,3,6
#  11, (3,2,2):  D=7, q = 33/7, 22/7, 22/7 -> floors 4,3,3, remainders 5/7,
#                1/7, 1/7, one left -> the first: 5,3,3
#   9, (2,1,2,1): D=6, q = 3, 1.5, 3, 1.5 -> floors 3,1,3,1, remainders 0,
#                1/2, 0, 1/2, one left, tie of the second and fourth -> the
#                second: 3,2,3,1
#   7, (2,1,3,1): D=7, quotas exact: 2,1,3,1
#   5, (1,1,1,1,1,1): q = 5/6 each, floors 0, five left -> 1,1,1,1,1,0
HAND_APPORTIONED = [
    (10, (1, 1, 1), (4, 3, 3)),
    (8, (1, 1, 1), (3, 3, 2)),
    (10, (1, 2, 4), (1, 3, 6)),
    (11, (3, 2, 2), (5, 3, 3)),
    (9, (2, 1, 2, 1), (3, 2, 3, 1)),
    (7, (2, 1, 3, 1), (2, 1, 3, 1)),
    (5, (1, 1, 1, 1, 1, 1), (1, 1, 1, 1, 1, 0)),
]


@pytest.mark.parametrize("s_insig,counts,want", HAND_APPORTIONED)
def test_apportionment_hand_worked(s_insig, counts, want):
    got = oracle.apportion(s_insig, counts)
    assert tuple(got) == want
    assert sum(got) == s_insig


def _closest_apportionment(s_insig, counts):
    """Brute force: among allocations a_j in {floor q_j, floor q_j + 1} with
    sum s_I, those closest to the quotas in squared distance (exact
    fractions); of several, the one giving the extra units to the earliest
    circuits (lexicographically largest)."""
    D = sum(counts)
    q = [Fraction(s_insig * c, D) for c in counts]
    fl = [math.floor(x) for x in q]
    left = s_insig - sum(fl)
    best, best_d = None, None
    for extra in itertools.combinations(range(len(counts)), left):
        a = [f + (1 if j in extra else 0) for j, f in enumerate(fl)]
        d = sum((Fraction(x) - y) ** 2 for x, y in zip(a, q))
        if best_d is None or d < best_d or (d == best_d and a > best):
            best, best_d = a, d
    return best


def test_apportionment_is_the_closest_to_the_quotas():
    rng = np.random.default_rng(11)
    for _ in range(400):
        k = int(rng.integers(1, 8))
        counts = [int(x) for x in rng.integers(1, 6, size=k)]
        s_insig = int(rng.integers(0, 40))
        assert oracle.apportion(s_insig, counts) == _closest_apportionment(s_insig, counts), \
            (s_insig, counts)


# --------------------------------------------------------------------------
# Shot sampling (leaf-level inverse CDF)

def test_samples_follow_leaf_distribution():
    c = brickwork(4, 4, 0.0, 0.0, seed=6)
    t = oracle.ecm(c, 200_000, seed=6)
    assert t.n_leaves == 1
    dist, samples, ct, norms = oracle.run(c, t, 6)
    assert ct["draws"] == 200_000 and len(samples) == 200_000
    h = np.bincount(samples.astype(np.int64), minlength=16) / 200_000
    sig = np.sqrt(dist * (1 - dist) / 200_000) + 1e-9
    assert np.all(np.abs(h - dist) < 5 * sig)
    assert abs(norms[0] - 1) < 1e-13


def test_sample_indices_and_margins_consistent():
    c = brickwork(5, 5, 0.02, 0.05, seed=7)
    t = oracle.ecm(c, 3000, seed=7)
    _, samples, _, _ = oracle.run(c, t, 7)
    off = 0
    for leaf in range(t.n_leaves):
        k = int(t.shots[leaf])
        psi = oracle.trajectory(c, t.events(leaf))
        idx, mar = oracle.leaf_margins(c, psi, 7, leaf, k)
        np.testing.assert_array_equal(idx, samples[off:off + k])
        probs = np.abs(psi[idx.astype(np.int64)]) ** 2
        assert np.all(probs > 0)
        off += k


# --------------------------------------------------------------------------
# Pauli-twirled thermal relaxation (Sec. VI-A, Eq. (4))

_PAULI = {"X": np.array([[0, 1], [1, 0]], complex), "Y": np.array([[0, -1j], [1j, 0]]),
          "Z": np.array([[1, 0], [0, -1]], complex)}
THERMAL_CASES = [(0.05, 1.0, 1.5), (0.3, 2.0, 0.7), (1.0, 1.0, 2.0), (2e-3, 100.0, 60.0),
                 (0.0, 1.0, 1.0), (5.0, 1.0, 0.1)]


def _relaxation_kraus(t, t1, t2):
    """Amplitude damping (gamma = 1 - e^{-t/T1}) followed by pure dephasing
    that brings the coherence decay to e^{-t/T2}."""
    g = 1.0 - math.exp(-t / t1)
    ad = [np.array([[1, 0], [0, math.sqrt(1 - g)]], complex),
          np.array([[0, math.sqrt(g)], [0, 0]], complex)]
    rest = math.exp(-t / t2) / math.sqrt(1 - g) if g < 1 else 1.0   # 1 - 2q
    q = (1.0 - rest) / 2.0
    pd = [math.sqrt(1 - q) * np.eye(2, dtype=complex), math.sqrt(q) * _PAULI["Z"]]
    return [b @ a for a in ad for b in pd]


@pytest.mark.parametrize("t,t1,t2", THERMAL_CASES)
def test_thermal_twirl_is_the_chi_diagonal_of_relaxation(t, t1, t2):
    """The Pauli twirl of a channel keeps the diagonal of its chi matrix,
    p_P = sum_K |Tr(P K)|^2 / 4: Eq. (4) must equal it for amplitude damping
    plus dephasing (computed here from Kraus operators)."""
    ks = _relaxation_kraus(t, t1, t2)
    assert np.allclose(sum(k.conj().T @ k for k in ks), np.eye(2), atol=1e-14)
    chi = [sum(abs(np.trace(_PAULI[P] @ k)) ** 2 for k in ks) / 4 for P in "XYZ"]
    np.testing.assert_allclose(oracle.thermal_probs(t, t1, t2), chi, atol=1e-15, rtol=0)


@pytest.mark.parametrize("t,t1,t2", THERMAL_CASES)
def test_thermal_twirl_decay_rates(t, t1, t2):
    """The twirled channel contracts <Z> by e^{-t/T1} and <X>, <Y> by e^{-t/T2}
    (density-matrix check on |+> and |1>)."""
    px, py, pz = oracle.thermal_probs(t, t1, t2)
    def apply(rho):
        return ((1 - px - py - pz) * rho + px * _PAULI["X"] @ rho @ _PAULI["X"]
                + py * _PAULI["Y"] @ rho @ _PAULI["Y"] + pz * _PAULI["Z"] @ rho @ _PAULI["Z"])
    plus = np.full((2, 2), 0.5, complex)
    one = np.array([[0, 0], [0, 1]], complex)
    assert abs(np.trace(_PAULI["X"] @ apply(plus)).real - math.exp(-t / t2)) < 1e-14
    assert abs(np.trace(_PAULI["Z"] @ apply(one)).real + math.exp(-t / t1)) < 1e-14


@pytest.mark.parametrize("p", [(0.1, 0.25, 0.05), (1.0, 0.0, 1.0), (0.0, 0.4, 0.0)])
def test_readout_flips_closed_form(p):
    """Read-out flips (Sec. IV-D) on the product state X|0>, H|0>, |0>: each
    qubit reads its bit flipped with its own probability, so the output is a
    product of Bernoulli marginals -- qubit 0 reads 1 with probability 1 - p0,
    qubit 1 with 1/2 whatever p1, qubit 2 with p2.  Exact over every error
    pattern and by the density matrix; through the sampled lossless pipeline
    within the binomial spread."""
    c = Circuit(3)
    c.add("X", (0,), ())
    c.add("H", (1,), ())
    for q in range(3):
        c.add_readout_noise(q, p[q])
    one = [1 - p[0], 0.5, p[2]]
    want = np.array([np.prod([one[q] if b >> q & 1 else 1 - one[q] for q in range(3)])
                     for b in range(8)])
    mix = np.zeros(8)
    for pr, ev in dms.enumerate_ers(c):
        mix += pr * np.abs(oracle.trajectory(c, ev)) ** 2
    np.testing.assert_allclose(mix, want, atol=1e-15)
    np.testing.assert_allclose(np.real(np.diag(dms.density_matrix(c))), want, atol=1e-14)
    S = 200_000
    t = oracle.ecm(c, S, seed=4, prune=False)
    dist, _, _, _ = oracle.run(c, t, seed=4, want_samples=False)
    assert np.max(np.abs(dist - want)) < 5 * np.sqrt(0.25 / S) + 1e-15


# --------------------------------------------------------------------------
# A caller's unitaries (UNITARY1 / UNITARY2)

def _haar(d, rng):
    z = rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))
    q, r = np.linalg.qr(z)
    return q * (np.diag(r) / np.abs(np.diag(r)))


def _prep(n, rng):
    c = Circuit(n)
    for q in range(n):
        c.add("U3", (q,), rng.random(3) * 6.28)
    return c


def test_unitary1_with_a_named_gates_matrix_is_that_gate():
    rng = np.random.default_rng(3)
    for kind, npar in (("U3", 3), ("RX", 1), ("H", 0), ("T", 0)):
        pr = tuple(rng.random(npar) * 6.28)
        a, b = _prep(3, rng), None
        b = Circuit(3, kinds=list(a.kinds), qubits=list(a.qubits), params=list(a.params),
                    noise=list(a.noise))
        a.add(kind, (1,), pr)
        b.add_unitary((1,), dms.gate_2x2(kind, pr))
        np.testing.assert_allclose(oracle.trajectory(b), oracle.trajectory(a), atol=1e-14)


def test_unitary2_orientation_and_products():
    """The 4x4's basis index is 2 * bit(first qubit) + bit(second): the CX
    matrix on (c, t) is CX(c, t) in both qubit orders, and kron(A, B) on
    (qa, qb) is A on qa then B on qb."""
    rng = np.random.default_rng(4)
    cxm = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]], complex)
    for ctl, tgt in ((0, 2), (2, 0), (1, 2)):
        a = _prep(3, rng)
        b = Circuit(3, kinds=list(a.kinds), qubits=list(a.qubits), params=list(a.params),
                    noise=list(a.noise))
        a.add("CX", (ctl, tgt))
        b.add_unitary((ctl, tgt), cxm)
        np.testing.assert_allclose(oracle.trajectory(b), oracle.trajectory(a), atol=1e-14)
    A, B = _haar(2, rng), _haar(2, rng)
    a = _prep(3, rng)
    b = Circuit(3, kinds=list(a.kinds), qubits=list(a.qubits), params=list(a.params),
                noise=list(a.noise))
    a.add_unitary((2, 0), np.kron(A, B))
    b.add_unitary((2,), A)
    b.add_unitary((0,), B)
    np.testing.assert_allclose(oracle.trajectory(a), oracle.trajectory(b), atol=1e-14)
    # and against the plain matrix product on the whole space
    np.testing.assert_allclose(oracle.trajectory(a), dms.circuit_unitary(a)[:, 0], atol=1e-13)


def test_user_unitaries_undo_to_the_start():
    """The undo of a UNITARY1 / UNITARY2 (its conjugate transpose) returns
    the state: forward to every depth and back gives |0...0>."""
    rng = np.random.default_rng(5)
    c = Circuit(3)
    for _ in range(3):
        c.add_unitary((int(rng.integers(3)),), _haar(2, rng), depol1(0.3))
        a, b = rng.choice(3, 2, replace=False)
        c.add_unitary((int(a), int(b)), _haar(4, rng), depol2(0.3))
    ev = [(2, 0, 1), (4, 1, 3), (5, 2, 2)]
    for depth in range(1, c.n_gates + len(ev) + 1):
        assert oracle.roundtrip(c, ev, depth) < 1e-13


def test_no_pauli_moves_through_a_user_unitary():
    """RX lets an X error through and CX maps X_c to X_c X_t; the same
    matrices given as UNITARY1 / UNITARY2 stop the error at their slot."""
    rx = dms.gate_2x2("RX", (0.7,))
    cxm = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]], complex)
    for named in (True, False):
        c = Circuit(2)
        c.add("X", (0,), (), (1.0, 0.0, 0.0))        # always an X error on qubit 0
        if named:
            c.add("RX", (0,), (0.7,))
            c.add("CX", (0, 1))
        else:
            c.add_unitary((0,), rx)
            c.add_unitary((0, 1), cxm)
        chan, outc = oracle.sample_shot(c, 1, 0)
        ev = oracle.commute(c, chan, outc)
        assert ev == ([(3, 0, 1), (3, 1, 1)] if named else [(1, 0, 1)])
        assert dms.equal_up_to_phase(dms.circuit_unitary(c, ev),
                                     dms.circuit_unitary(c, oracle.commute(
                                         c, chan, outc, do_commute=False)))


@pytest.mark.parametrize("seed", range(3))
def test_noisy_user_unitaries_equal_density_matrix(seed):
    rng = np.random.default_rng(40 + seed)
    c = Circuit(3)
    c.add_unitary((0,), _haar(2, rng), depol1(0.2))
    c.add_unitary((1, 2), _haar(4, rng), depol2(0.2))
    c.add("H", (2,), (), depol1(0.1))
    c.add_unitary((2, 0), _haar(4, rng), (0.01,) * 15)
    mix = np.zeros(8)
    for p, ev in dms.enumerate_ers(c):
        mix += p * np.abs(oracle.trajectory(c, ev)) ** 2
    np.testing.assert_allclose(mix, np.real(np.diag(dms.density_matrix(c))), atol=1e-12)


def test_add_unitary_refuses_bad_input():
    c = Circuit(3)
    for qs, m in (((0,), np.eye(4)), ((0, 1), np.eye(2)), ((0, 0), np.eye(4)),
                  ((0,), [[1, 1], [0, 1]]), ((3,), np.eye(2)), ((0,), [[np.nan, 0], [0, 1]])):
        with pytest.raises(ValueError):
            c.add_unitary(qs, m)
    with pytest.raises(ValueError):
        c.add_unitary((0,), np.eye(2), depol2(0.1))
    assert c.n_gates == 0


def test_thermal_twirl_on_cx_is_the_product_channel():
    p1 = oracle.thermal_probs(0.2, 1.3, 0.9)
    p2 = oracle.thermal_probs(0.2, 1.3, 0.9, two_qubit=True)
    q = [1 - sum(p1)] + p1
    for k in range(1, 16):
        assert p2[k - 1] == q[k >> 2] * q[k & 3]
    assert abs(sum(p2) + q[0] * q[0] - 1) < 1e-15
    for bad in ((-1.0, 1.0, 1.0), (1.0, 0.0, 1.0), (1.0, 1.0, 0.0), (1.0, 1.0, 2.5)):
        with pytest.raises(ValueError):
            oracle.thermal_probs(*bad)


def test_bounded_checkpoints_trade_undo_for_memory():
    """With at most K kept states the checkpoint walk saves at the same
    depths, restores where the state is still kept and undoes (as plain
    DFTT) where it was dropped: every transition is one or the other, undo
    work falls as K grows and vanishes without a bound."""
    c = brickwork(6, 8, 0.02, 0.05, seed=3)
    t = oracle.ecm(c, 3000, 4, prune=False)
    _, _, dftt, _ = oracle.run(c, t, 4, traversal="dftt", want_dist=False, want_samples=False)
    undo = lambda x: x["inv_gates"] + x["inv_paulis"]
    runs = [oracle.run(c, t, 4, traversal="checkpoint", want_dist=False, want_samples=False,
                       checkpoint_slots=k)[2] for k in (1, 2, 3, 0)]
    for r in runs:
        assert r["checkpoint_saves"] == runs[-1]["checkpoint_saves"]
        assert r["fwd_gates"] + r["fwd_paulis"] == dftt["fwd_gates"] + dftt["fwd_paulis"]
        assert undo(r) <= undo(dftt)
    assert undo(runs[-1]) == 0 and runs[-1]["checkpoint_restores"] == t.n_leaves - 1
    assert all(undo(a) >= undo(b) for a, b in zip(runs, runs[1:]))
    assert all(a["checkpoint_restores"] <= b["checkpoint_restores"] for a, b in zip(runs, runs[1:]))


def test_run_margins_equal_the_per_leaf_margins():
    # the walk's per-draw margins are those of each leaf's state recomputed
    # from the root (up to the rounding an undo leaves, ~5e-15 here), and
    # the samples are the plain run's
    c = brickwork(6, 6, 5e-3, 3e-2, seed=4)
    t = oracle.ecm(c, 3000, 9)
    d0, s0, _, _ = oracle.run(c, t, 9)
    d1, s1, m1, _, _ = oracle.run_with_margins(c, t, 9)
    assert np.array_equal(d0, d1) and np.array_equal(s0, s1)
    off = 0
    for leaf in range(t.n_leaves):
        k = int(t.shots[leaf])
        if not k:
            continue
        psi = oracle.trajectory(c, t.events(leaf))
        idx, mar = oracle.leaf_margins(c, psi, 9, leaf, k)
        assert np.array_equal(idx, s1[off:off + k])
        np.testing.assert_allclose(m1[off:off + k], mar, rtol=0, atol=1e-13)
        off += k
    assert off == len(s1)
