"""GPU edge cases through the C ABI: degenerate circuits and shot counts,
closed forms, tiles that span the whole state or leave a ragged set of
qubits, every traversal on a noise-only tree, and the complex64 path on the
smallest inputs.  Each case is checked against the oracle or an exact
answer."""

import sys

import numpy as np
import pytest

import oracle
import paper_2508_04880_amd as tq
from workloads import Circuit, bell_pair, brickwork, random_small_circuit
from workloads.circuits import depol1, depol2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = tq.Context(0)
    yield c
    c.close()


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _run(ctx, c, S, seed, **kw):
    ec = tq.Circuit(c)
    o = tq.tusq_opts_default(shots=S, seed=seed, **kw)
    t = tq.Tree(ec, o)
    return t, tq.tusq_run_tree(ctx, ec, t, o)


@pytest.mark.parametrize("precision", ["c128", "c64"])
def test_empty_circuit_is_the_zero_state(ctx, precision):
    _say(f"[gpu] empty circuit {precision}")
    c = Circuit(5)
    t, r = _run(ctx, c, 100, 1, precision=precision)
    d = r.distribution()
    assert d[0] == 1.0 and not d[1:].any()
    assert len(r.samples()) == 100 and not r.samples().any()


@pytest.mark.parametrize("S", [1, 2, 7])
def test_few_shots_single_qubit(ctx, S):
    _say(f"[gpu] one qubit S={S}")
    c = Circuit(1)
    c.add("H", (0,), (), depol1(0.3))
    c.add("T", (0,), (), depol1(0.2))
    seed = 11
    ot = oracle.ecm(c, S, seed)
    dist, _, _, _ = oracle.run(c, ot, seed, want_samples=False)
    t, r = _run(ctx, c, S, seed)
    assert t.serialize() == ot.serialize()
    np.testing.assert_allclose(r.distribution(), dist, atol=1e-12, rtol=0)
    assert len(r.samples()) == S


def test_bell_pair_closed_form_through_the_engine(ctx):
    """Lossless: every noisy instance is its own leaf, so the averaged
    distribution is the empirical mixture; with many shots it approaches the
    channel output P(00)=P(11)=(1-8p/15)/2, P(01)=P(10)=4p/15."""
    _say("[gpu] bell pair")
    p = 0.3
    c = bell_pair(0.0, p)
    S, seed = 400_000, 3
    ot = oracle.ecm(c, S, seed, prune=False)
    dist, _, _, _ = oracle.run(c, ot, seed, want_samples=False)
    t, r = _run(ctx, c, S, seed, prune=0)
    d = r.distribution()
    np.testing.assert_allclose(d, dist, atol=1e-12, rtol=0)
    exact = np.array([(1 - 8 * p / 15) / 2, 4 * p / 15, 4 * p / 15, (1 - 8 * p / 15) / 2])
    # binomial spread of the sampled error frequencies at S shots
    assert np.max(np.abs(d - exact)) < 5 * np.sqrt(0.25 / S)


@pytest.mark.parametrize("trav", ["dftt", "naive", "hybrid", "checkpoint"])
def test_noise_only_tree(ctx, trav):
    """Identity gates only (X twice) with strong noise: the tree is all
    error branches; every traversal equals the oracle."""
    _say(f"[gpu] noise-only tree {trav}")
    c = Circuit(3)
    for _ in range(4):
        for q in range(3):
            c.add("X", (q,), (), depol1(0.2))
        c.add("CX", (0, 2), (), depol2(0.2))
        c.add("CX", (0, 2), ())
    S, seed = 5000, 9
    ot = oracle.ecm(c, S, seed)
    dist, _, _, _ = oracle.run(c, ot, seed, traversal=trav, want_samples=False)
    t, r = _run(ctx, c, S, seed, traversal=trav)
    np.testing.assert_allclose(r.distribution(), dist, atol=1e-12, rtol=0)


@pytest.mark.parametrize("n,kmax", [(12, 12), (13, 12), (12, 16), (17, 12), (9, 4)])
@pytest.mark.parametrize("precision", ["c128", "c64"])
def test_tile_spans_state_or_leaves_ragged_qubits(ctx, n, kmax, precision):
    """Tiles of the whole state (k = n, one workgroup), one qubit more than a
    tile, tiles larger than the state, and tiles smaller than a wavefront's
    register block."""
    _say(f"[gpu] tiles n={n} k={kmax} {precision}")
    c = brickwork(n, 6, 2e-3, 2e-2, 40 + n)
    S, seed = 3000, 13
    ot = oracle.ecm(c, S, seed)
    dist, _, _, _ = oracle.run(c, ot, seed, want_samples=False)
    t, r = _run(ctx, c, S, seed, precision=precision, fusion_max_qubits=kmax,
                fusion_low_qubits=min(4, max(kmax - 2, 1)), drift_bound=1.0)
    tol = 1e-10 if precision == "c128" else 1e-4
    np.testing.assert_allclose(r.distribution(), dist, atol=tol, rtol=0)


def test_noiseless_circuit_is_one_leaf_with_all_shots(ctx):
    _say("[gpu] noiseless")
    c = random_small_circuit(6, 40, 3, p1=0.0, p2=0.0)
    S, seed = 1234, 5
    ot = oracle.ecm(c, S, seed)
    assert ot.n_leaves == 1
    dist, _, _, _ = oracle.run(c, ot, seed, want_samples=False)
    t, r = _run(ctx, c, S, seed)
    np.testing.assert_allclose(r.distribution(), dist, atol=1e-12, rtol=0)
    assert len(r.samples()) == S


@pytest.mark.parametrize("precision", ["c128", "c64"])
def test_thermal_relaxation_noise_matches_oracle(ctx, precision):
    """Brickwork with the Pauli-twirled thermal-relaxation channel (Eq. (4))
    after every gate, attached through tusq_circuit_thermal_noise, against the
    oracle run on oracle-computed probabilities."""
    _say(f"[gpu] thermal noise {precision}")
    base = brickwork(9, 10, 0.0, 0.0, 23)
    t_1q, t_2q, T1, T2 = 0.01, 0.05, 1.0, 0.7
    c = Circuit(9)
    ec = tq.Circuit(Circuit(9, kinds=list(base.kinds), qubits=list(base.qubits),
                            params=list(base.params), noise=[None] * base.n_gates))
    for g, (k, q, p) in enumerate(zip(base.kinds, base.qubits, base.params)):
        t = t_2q if k == "CX" else t_1q
        c.add(k, q, p, oracle.thermal_probs(t, T1, T2, two_qubit=(k == "CX")))
        ec.thermal_noise(g, t, T1, T2)
    S, seed = 20_000, 4
    ot = oracle.ecm(c, S, seed)
    dist, _, _, _ = oracle.run(c, ot, seed, want_samples=False)
    o = tq.tusq_opts_default(shots=S, seed=seed, precision=precision, drift_bound=1.0)
    t = tq.Tree(ec, o)
    assert t.serialize() == ot.serialize()
    r = tq.tusq_run_tree(ctx, ec, t, o)
    tol = 1e-10 if precision == "c128" else 1e-4
    np.testing.assert_allclose(r.distribution(), dist, atol=tol, rtol=0)


@pytest.mark.parametrize("precision", ["c128", "c64"])
@pytest.mark.parametrize("trav", ["dftt", "checkpoint"])
def test_user_unitaries_match_oracle(ctx, precision, trav):
    """A caller's UNITARY1 / UNITARY2 gates (Haar-random) mixed with U3 and
    CX, all noisy, on 13 qubits with tiles of 10: against the oracle."""
    from workloads.circuits import unitary_mix
    _say(f"[gpu] user unitaries {precision} {trav}")
    c = unitary_mix(13, 120, 17)
    S, seed = 5000, 8
    ot = oracle.ecm(c, S, seed)
    dist, _, oc, _ = oracle.run(c, ot, seed, traversal=trav, want_samples=False)
    t, r = _run(ctx, c, S, seed, precision=precision, traversal=trav, fusion_max_qubits=10,
                fusion_low_qubits=4, drift_bound=1.0)
    assert t.serialize() == ot.serialize()
    tol = 1e-10 if precision == "c128" else 1e-4
    np.testing.assert_allclose(r.distribution(), dist, atol=tol, rtol=0)
    ct = r.counters()
    for k in ("fwd_gates", "inv_gates", "fwd_paulis", "inv_paulis", "paper_ops"):
        assert ct[k] == oc[k], k


@pytest.mark.parametrize("precision", ["c128", "c64"])
def test_readout_noise_matches_oracle(ctx, precision):
    """Brickwork with the paper's depolarising noise plus a read-out flip on
    every qubit (tusq_circuit_readout_noise), against the oracle run on the
    same circuit built through the workload helper."""
    _say(f"[gpu] read-out noise {precision}")
    base = brickwork(9, 10, 1e-3, 1e-2, 23)
    c = Circuit(9, kinds=list(base.kinds), qubits=list(base.qubits),
                params=list(base.params), noise=list(base.noise))
    ec = tq.Circuit(Circuit(9, kinds=list(base.kinds), qubits=list(base.qubits),
                            params=list(base.params), noise=list(base.noise)))
    for q in range(9):
        p = 0.01 * (q + 1)
        c.add_readout_noise(q, p)
        ec.readout_noise(q, p)
    S, seed = 20_000, 6
    ot = oracle.ecm(c, S, seed)
    dist, _, _, _ = oracle.run(c, ot, seed, want_samples=False)
    o = tq.tusq_opts_default(shots=S, seed=seed, precision=precision, drift_bound=1.0)
    t = tq.Tree(ec, o)
    assert t.serialize() == ot.serialize()
    r = tq.tusq_run_tree(ctx, ec, t, o)
    tol = 1e-10 if precision == "c128" else 1e-4
    np.testing.assert_allclose(r.distribution(), dist, atol=tol, rtol=0)


@pytest.mark.parametrize("slots", [0, 2])
@pytest.mark.parametrize("precision", ["c128", "c64"])
@pytest.mark.parametrize("n,kmax", [(10, 6), (18, 12)])
def test_checkpoint_traversal_matches_oracle(ctx, precision, n, kmax, slots):
    """Branch checkpoints kept in device memory: the distribution equals the
    oracle's, no gate or Pauli is ever undone, and the save and restore
    counts equal the oracle's walk of the same tree."""
    _say(f"[gpu] checkpoint n={n} kmax={kmax} {precision} slots={slots}")
    c = brickwork(n, 8, 3e-3, 2e-2, 31)
    S, seed = 4000, 13
    ot = oracle.ecm(c, S, seed)
    dist, _, oc, _ = oracle.run(c, ot, seed, traversal="checkpoint", want_samples=False,
                                checkpoint_slots=slots)
    t, r = _run(ctx, c, S, seed, traversal="checkpoint", precision=precision,
                fusion_max_qubits=kmax, drift_bound=1.0, checkpoint_slots=slots)
    assert t.serialize() == ot.serialize()
    tol = 1e-10 if precision == "c128" else 1e-4
    np.testing.assert_allclose(r.distribution(), dist, atol=tol, rtol=0)
    ct = r.counters()
    for k in ("checkpoint_saves", "checkpoint_restores", "resets", "leaves", "inv_gates",
              "inv_paulis", "paper_ops"):
        assert ct[k] == oc[k], k
    if not slots:
        assert ct["inv_gates"] == 0 and ct["inv_paulis"] == 0
        assert ct["checkpoint_restores"] == ot.n_leaves - 1


def test_checkpoint_budget_is_enforced(ctx):
    """A budget that holds the state but not its checkpoints is refused
    before any device work, and the same run fits with plain DFTT."""
    _say("[gpu] checkpoint budget")
    c = brickwork(16, 6, 5e-3, 3e-2, 3)
    N, S = 1 << 16, 3000
    ot = oracle.ecm(c, S, 2)
    _, _, oc, _ = oracle.run(c, ot, 2, traversal="checkpoint", want_dist=False,
                             want_samples=False)
    assert oc["checkpoint_saves"] > 0
    # a job's device memory: state, FP64 accumulator, sampler chunk sums and
    # prefix, samples and a 64 MiB plan reserve; half a state more is too
    # little for one checkpoint slot
    job = N * 16 + N * 8 + 2 * (N >> 11) * 8 + S * 8 + (64 << 20)
    small = tq.Context(0, hbm_budget=job + N * 8)
    try:
        _run(small, c, S, 2)
        with pytest.raises(tq.TusqError) as e:
            _run(small, c, S, 2, traversal="checkpoint")
        assert e.value.code == -2 and "checkpoint" in str(e.value)
    finally:
        small.close()


def test_distribution_written_to_device_memory(ctx):
    """tusq_result_distribution_device fills device memory (allocated here
    through the HIP runtime) with the values the host copy returns, on a
    caller stream."""
    import ctypes as C
    _say("[gpu] distribution to device memory")
    c = brickwork(10, 6, 2e-3, 2e-2, 5)
    t, r = _run(ctx, c, 2000, 3)
    host = r.distribution()
    hip = C.CDLL("libamdhip64.so")
    nbytes = host.nbytes
    dptr, stream = C.c_void_p(), C.c_void_p()
    assert hip.hipMalloc(C.byref(dptr), C.c_size_t(nbytes)) == 0
    try:
        assert hip.hipStreamCreate(C.byref(stream)) == 0
        r.distribution_to_device(dptr.value, stream.value)
        back = np.full_like(host, -1.0)
        assert hip.hipMemcpy(back.ctypes.data_as(C.c_void_p), dptr, C.c_size_t(nbytes), 2) == 0
        assert np.array_equal(back, host)
    finally:
        if stream.value:
            hip.hipStreamDestroy(stream)
        hip.hipFree(dptr)
