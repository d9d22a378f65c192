"""GPU parity of DFTT+Caching over circuits with mid-circuit measurement
layers (Sec. III-B.2), through the C ABI: distributions, samples and every
operation counter against the oracle's walk for each cache capacity,
complex64 within its stated error, tiled sweeps, and the refusals."""

import sys

import numpy as np
import pytest

import oracle
import paper_2508_04880_amd as tq
from workloads import Circuit, syndrome_rounds
from workloads.circuits import depol1, depol2

pytestmark = pytest.mark.gpu

COUNTERS = ("fwd_gates", "inv_gates", "fwd_paulis", "inv_paulis", "resets", "leaves", "draws",
            "checkpoint_saves", "checkpoint_restores", "mcm_edges", "paper_ops")


@pytest.fixture(scope="module")
def ctx():
    c = tq.Context(0)
    yield c
    c.close()


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _mixed(seed):
    """Random gates, a 1-qubit measurement without reset, more gates, a
    2-qubit measure-and-reset layer, a tail."""
    rng = np.random.default_rng(seed)
    c = Circuit(5)
    for q in range(5):
        c.add("U3", (q,), rng.random(3) * 6.28, depol1(0.03))
    for q in range(4):
        c.add("CX", (q, q + 1), (), depol2(0.05))
    c.add_measure((2,), reset=False)
    for q in range(5):
        c.add("RY", (q,), (float(rng.random() * 3),), depol1(0.03))
    c.add("CX", (4, 0), (), depol2(0.05))
    c.add_measure((0, 3), reset=True)
    c.add("H", (0,), (), depol1(0.03))
    c.add("CX", (0, 1), (), depol2(0.05))
    return c


def _run(ctx, c, S, seed, K, precision="c128", **kw):
    ec = tq.Circuit(c)
    o = tq.tusq_opts_default(shots=S, seed=seed, prune=0, traversal="caching", cache_capacity=K,
                             precision=precision, **kw)
    t = tq.Tree(ec, o)
    return t, tq.tusq_run_tree(ctx, ec, t, o)


@pytest.mark.parametrize("fam", ["syndrome", "mixed"])
@pytest.mark.parametrize("K", [0, 1, 2, 3])
def test_caching_walk_matches_oracle(ctx, fam, K):
    _say(f"[gpu] mcm {fam} K={K}")
    c = syndrome_rounds(3, 3, 0.02, 0.05, theta=0.7) if fam == "syndrome" else _mixed(4)
    S, seed = 3000, 12
    ot = oracle.ecm(c, S, seed, prune=False)
    dist, samples, oc, held = oracle.run_mcm(c, ot, seed, K)
    t, r = _run(ctx, c, S, seed, K)
    assert t.serialize() == ot.serialize()
    np.testing.assert_allclose(r.distribution(), dist, atol=1e-10, rtol=0)
    ct = r.counters()
    for k in COUNTERS:
        assert ct[k] == oc[k], k
    got = r.samples()
    assert len(got) == S
    assert np.count_nonzero(got != samples) <= 2
    assert np.all(np.abs(r.norms(ct["leaves"]) - 1.0) < 1e-12)


@pytest.mark.parametrize("precision", ["c128", "c64"])
def test_tiled_sweeps_between_measurements(ctx, precision):
    """13 qubits (repetition code of distance 7, 6 ancillas per layer) with
    8-qubit sweep tiles: every stage runs through the tiled kernels."""
    _say(f"[gpu] mcm tiled {precision}")
    c = syndrome_rounds(7, 3, 0.01, 0.03, theta=0.5)
    S, seed = 2000, 21
    ot = oracle.ecm(c, S, seed, prune=False)
    dist, _, oc, _ = oracle.run_mcm(c, ot, seed, 2, want_samples=False)
    t, r = _run(ctx, c, S, seed, 2, precision=precision, fusion_max_qubits=8,
                fusion_low_qubits=4, want=1)
    tol = 1e-10 if precision == "c128" else 1e-4
    np.testing.assert_allclose(r.distribution(), dist, atol=tol, rtol=0)
    ct = r.counters()
    if precision == "c128":
        for k in COUNTERS:
            if k != "draws":
                assert ct[k] == oc[k], k
    assert ct["leaves"] > 0


def test_alpha_rises_with_the_cache(ctx):
    """Eq. (3) from the engine's own counts: alpha(0) = 0, alpha(M) = 1,
    non-decreasing in between, and the same distribution for every K."""
    _say("[gpu] mcm alpha")
    c = syndrome_rounds(3, 4, 0.02, 0.05, theta=0.9)
    M = c.n_measure_layers
    S, seed = 2500, 7
    runs = [_run(ctx, c, S, seed, K)[1] for K in range(M + 1)]
    ops = [r.counters()["paper_ops"] for r in runs]
    alpha = [(ops[0] - x) / (ops[0] - ops[M]) for x in ops]
    assert alpha[0] == 0.0 and alpha[M] == 1.0
    assert all(a <= b for a, b in zip(alpha, alpha[1:]))
    for r in runs[1:]:
        np.testing.assert_allclose(r.distribution(), runs[0].distribution(), atol=1e-12)


def test_refusals(ctx):
    _say("[gpu] mcm refusals")
    c = syndrome_rounds(3, 2, 0.02, 0.05, theta=0.7)
    ec = tq.Circuit(c)
    o = tq.tusq_opts_default(shots=500, seed=1, prune=0)
    t = tq.Tree(ec, o)
    with pytest.raises(tq.TusqError) as e:
        tq.tusq_run_tree(ctx, ec, t, o)           # plain DFTT cannot undo a measurement
    assert e.value.code == -3
    o2 = tq.tusq_opts_default(shots=500, seed=1, prune=1, traversal="caching")
    with pytest.raises(tq.TusqError) as e2:
        tq.tusq_run(ctx, ec, o2)
    assert e2.value.code == -3
    # a budget that holds the job but not its cached states
    N = 1 << c.n
    job = N * 16 + N * 8 + 2 * 8 + 500 * 8 + (64 << 20)
    small = tq.Context(0, hbm_budget=job + 1024)
    try:
        o3 = tq.tusq_opts_default(shots=500, seed=1, prune=0, traversal="caching",
                                  cache_capacity=2)
        with pytest.raises(tq.TusqError) as e3:
            tq.tusq_run_tree(small, ec, t, o3)
        assert e3.value.code == -2
    finally:
        small.close()


def test_leaf_range_and_no_outputs(ctx):
    """A depth-first slice of the tree starts from the root and draws its
    samples with the slice's own counters, as the oracle's walk over the same
    slice does; want = 0 runs the walk and returns only counters."""
    _say("[gpu] mcm leaf range")
    c = _mixed(9)
    S, seed = 2000, 5
    ot = oracle.ecm(c, S, seed, prune=False)
    lb, le = 3, max(4, ot.n_leaves - 5)
    dist, samples, oc, _ = oracle.run_mcm(c, ot, seed, 2, leaf_begin=lb, leaf_end=le)
    t, r = _run(ctx, c, S, seed, 2, leaf_begin=lb, leaf_end=le)
    np.testing.assert_allclose(r.distribution(), dist, atol=1e-10, rtol=0)
    assert np.count_nonzero(r.samples() != samples) <= 2
    ct = r.counters()
    for k in COUNTERS:
        assert ct[k] == oc[k], k
    t2, r2 = _run(ctx, c, S, seed, 2, want=0)
    _, _, oc2, _ = oracle.run_mcm(c, ot, seed, 2, want_dist=False, want_samples=False)
    assert r2.counters()["paper_ops"] == oc2["paper_ops"]
    assert len(r2.samples()) == 0
