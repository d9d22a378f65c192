"""GPU parity of the batched executor: many independent jobs in one
persistent, graph-captured launch; each job's distribution and samples
against the oracle run alone with the same seed, and against the
single-job engine path."""

import sys

import numpy as np
import pytest

import oracle
import paper_2508_04880_amd as tq
from conftest import same_bits
from workloads import brickwork, ising, random_small_circuit
from workloads.circuits import unitary_mix

pytestmark = pytest.mark.gpu

MARGIN = 1e-11


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = tq.Context(0)
    yield c
    c.close()


def _with_readout(c, p):
    for q in range(c.n):
        c.add_readout_noise(q, p)
    return c


JOBS = [
    lambda: brickwork(5, 6, 2e-3, 2e-2, 11),
    lambda: brickwork(10, 12, 1e-3, 1e-2, 12),
    lambda: ising(8, 5, 5e-3, 1e-2),
    lambda: random_small_circuit(9, 50, 13, p1=0.01, p2=0.02),
    lambda: brickwork(13, 10, 1e-3, 1e-2, 14),
    lambda: brickwork(14, 8, 1e-3, 1e-2, 15),
    lambda: brickwork(16, 6, 1e-3, 5e-3, 16),
    lambda: ising(15, 4, 1e-3, 5e-3),
    lambda: unitary_mix(11, 60, 21),
    lambda: _with_readout(brickwork(7, 8, 1e-3, 1e-2, 17), 0.03),
]


def _oracle_job(c, S, seed):
    ot = oracle.ecm(c, S, seed)
    dist, samples, _, _ = oracle.run(c, ot, seed)
    return ot, dist, samples


def _check_samples(c, ot, seed, got):
    off = 0
    for leaf in range(ot.n_leaves):
        k = int(ot.shots[leaf])
        if not k:
            continue
        psi = oracle.trajectory(c, ot.events(leaf))
        idx, mar = oracle.leaf_margins(c, psi, seed, leaf, k)
        g = got[off:off + k]
        bad = g != idx
        if bad.any():
            assert np.all(mar[bad] < MARGIN), (leaf, g[bad][:4], idx[bad][:4])
        off += k
    assert off == len(got)


@pytest.mark.parametrize("trav", ["dftt", "hybrid"])
def test_batch_matches_oracle_per_job(ctx, trav):
    _say(f"[gpu] batch parity trav={trav}")
    circs = [f() for f in JOBS]
    S, base = 3000, 500
    ecs = [tq.Circuit(c) for c in circs]
    o = tq.tusq_opts_default(shots=S, seed=base, traversal=trav)
    res = tq.tusq_run_batch(ctx, ecs, o)
    for j, (c, r) in enumerate(zip(circs, res)):
        ot, dist, samples = _oracle_job(c, S, base + j)
        np.testing.assert_allclose(r.distribution(), dist, atol=1e-10, rtol=0)
        _check_samples(c, ot, base + j, r.samples())


def test_batch_equals_single_job_path(ctx):
    """complex128: the batched walk applies the same matrices in the same
    order as the single-job path, with another kernel (LDS op lists instead
    of register programs) and so another rounding order: distributions
    agree to 1e-12, samples up to draws at a CDF boundary."""
    _say("[gpu] batch vs alone")
    circs = [f() for f in JOBS[:6]]
    S, base = 2000, 900
    ecs = [tq.Circuit(c) for c in circs]
    res = tq.tusq_run_batch(ctx, ecs, tq.tusq_opts_default(shots=S, seed=base))
    for j, (ec, r) in enumerate(zip(ecs, res)):
        o = tq.tusq_opts_default(shots=S, seed=base + j)
        alone = tq.tusq_run(ctx, ec, o)
        np.testing.assert_allclose(r.distribution(), alone.distribution(), atol=1e-12, rtol=0)
        a, b = r.samples(), alone.samples()
        assert len(a) == len(b) and (a != b).sum() <= 2


@pytest.mark.parametrize("precision", ["c128", "c64"])
def test_batch_autotuned_shapes_match_oracle(ctx, precision):
    """The batch autotuner picks a launch shape per qubit count (threads per
    workgroup; tile qubits, low qubits and ops per sweep for states in
    global memory); batches run with the tuned shapes match the oracle job
    by job: complex128 to 1e-10, complex64 with its error against the
    oracle stated and bounded and its norm drift reported."""
    _say(f"[gpu] batch autotune {precision}")
    circs = [f() for f in JOBS]
    S, base = 3000, 2100
    ecs = [tq.Circuit(c) for c in circs]
    o = tq.tusq_opts_default(shots=S, seed=base, precision=precision)
    tq.tusq_batch_autotune(ctx, ecs, o, 2)
    kl = 14 if precision == "c64" else 13
    for c in circs:
        (th, tile, low, ops, reg), tuned = tq.tusq_batch_shape(ctx, c.n, precision)
        assert tuned and th in (256, 512, 1024)
        if c.n <= kl:
            assert tile == c.n and low == 0 and reg == 0
        elif reg:
            assert tile in (12, 13) and th == 1 << (tile - 4) and low in (4, 5) and ops in (0, 16)
        else:
            assert tile in (kl - 2, kl - 1, kl) and low in (4, 5) and ops in (0, 16, 32)
        _say(f"[gpu]   n={c.n}: threads {th}, tile {tile}, low {low}, ops {ops}, "
             f"register programs {reg}")
    res = tq.tusq_run_batch(ctx, ecs, o)
    worst, worst_tv, drift = 0.0, 0.0, 0.0
    for j, (c, r) in enumerate(zip(circs, res)):
        ot, dist, samples = _oracle_job(c, S, base + j)
        d = r.distribution()
        err = float(np.max(np.abs(d - dist)))
        worst = max(worst, err)
        worst_tv = max(worst_tv, 0.5 * float(np.abs(d - dist).sum()))
        drift = max(drift, r.counters()["max_norm_drift"])
        if precision == "c128":
            assert err <= 1e-10, (j, err)
            _check_samples(c, ot, base + j, r.samples())
    _say(f"[gpu]   {precision} against the oracle: max |dP| {worst:.3e}, total variation "
         f"{worst_tv:.3e}, max norm drift {drift:.3e}")
    if precision == "c64":
        assert worst < 1e-5 and worst_tv < 1e-4 and drift < 1e-4


def test_batch_graph_is_replayed(ctx):
    """A second and third call with the same launch shapes replay the graph
    the first one captured (eager single-job work runs in between) and give
    the first call's results bit for bit; a smaller batch of the same qubit
    counts (half the jobs) replays it too and still matches the oracle."""
    _say("[gpu] batch graph replay")
    circs = [f() for f in JOBS]
    ecs = [tq.Circuit(c) for c in circs]
    S, base = 2000, 3300
    o = tq.tusq_opts_default(shots=S, seed=base)
    twice = ecs + ecs            # every qubit count twice
    first = tq.tusq_run_batch(ctx, twice, o)
    ref = [(r.distribution(), r.samples()) for r in first]
    for rep in range(2):
        tq.tusq_run(ctx, tq.Circuit(brickwork(9, 6, 1e-3, 1e-2, 50 + rep)),
                    tq.tusq_opts_default(shots=500, seed=rep))
        again = tq.tusq_run_batch(ctx, twice, o)
        assert all(r.counters()["batch_graph_reused"] == 1 for r in again)
        for (d0, s0), r in zip(ref, again):
            assert same_bits(r.distribution(), d0)
            assert same_bits(r.samples(), s0)
    # the first half alone: the same qubit counts, buffers that already fit
    fewer = tq.tusq_run_batch(ctx, ecs, o)
    assert all(r.counters()["batch_graph_reused"] == 1 for r in fewer)
    for j, r in enumerate(fewer):
        assert same_bits(r.distribution(), ref[j][0])
        ot, dist, _ = _oracle_job(circs[j], S, base + j)
        np.testing.assert_allclose(r.distribution(), dist, atol=1e-10, rtol=0)


def test_batch_is_deterministic_and_c64_error_bounded(ctx):
    _say("[gpu] batch determinism and c64")
    circs = [f() for f in JOBS]
    ecs = [tq.Circuit(c) for c in circs]
    o = tq.tusq_opts_default(shots=2500, seed=77)
    r1 = tq.tusq_run_batch(ctx, ecs, o)
    r2 = tq.tusq_run_batch(ctx, ecs, o)
    for a, b in zip(r1, r2):
        assert same_bits(a.distribution(), b.distribution())
        assert same_bits(a.samples(), b.samples())
    o64 = tq.tusq_opts_default(shots=2500, seed=77, precision="c64")
    r3 = tq.tusq_run_batch(ctx, ecs, o64)
    worst = max(float(np.max(np.abs(a.distribution() - b.distribution()))) for a, b in zip(r1, r3))
    drift = max(r.counters()["max_norm_drift"] for r in r3)
    _say(f"[gpu] batch c64 max-abs error vs c128: {worst:.3e}, max norm drift {drift:.3e}")
    assert worst < 1e-5
    assert 0 < drift < 1e-4
