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
    _say(f"[gpu] batch c64 max-abs error vs c128: {worst:.3e}")
    assert worst < 1e-5
