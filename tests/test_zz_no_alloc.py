"""The no-allocation run (tusq_run_tree_noalloc) against tusq_run_tree on the
same circuit, tree and options: same kernels in the same order, so the
distribution and the samples must agree bit for bit.  Two calls in a row,
the second on a smaller state, so that the reused static scratch is shown
to start clean; both precisions; oversized jobs and short buffers refused
before any device work."""

import sys

import numpy as np
import pytest
import torch

import paper_2508_04880_amd as tq
from conftest import same_bits
from workloads import brickwork

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = tq.Context(0)
    yield c
    c.close()


def _pair(ctx, n, layers, S, seed, precision, traversal="dftt"):
    c = brickwork(n, layers, 1e-3, 1e-2, 40 + n)
    ec = tq.Circuit(c)
    o = tq.tusq_opts_default(shots=S, seed=seed, precision=precision, traversal=traversal,
                             want=tq.WANT_DIST | tq.WANT_SAMPLES)
    t = tq.Tree(ec, o)
    ref = tq.tusq_run_tree(ctx, ec, t, o)
    want_dist, want_samples = ref.distribution(), ref.samples()
    dev = torch.device("cuda:0")
    # poisoned outputs: every value must be written by the run
    dist = torch.full((1 << n,), float("nan"), dtype=torch.float64, device=dev)
    samples = torch.full((len(want_samples),), -1, dtype=torch.int64, device=dev)
    torch.cuda.synchronize()
    ct = tq.tusq_run_tree_noalloc(ctx, ec, t, o, dist.data_ptr(), samples.data_ptr(),
                                  len(want_samples))
    got_dist = dist.cpu().numpy()
    got_samples = samples.cpu().numpy().view(np.uint64)
    return want_dist, want_samples, got_dist, got_samples, ct, ref.counters()


@pytest.mark.parametrize("precision", ["c128", "c64"])
def test_noalloc_equals_run_tree_twice(ctx, precision):
    for (n, layers, S, seed, trav) in ((16, 12, 3000, 5, "dftt"), (11, 8, 2000, 6, "checkpoint")):
        _say(f"[gpu] noalloc {precision} n={n} L={layers} S={S} {trav}")
        wd, ws, gd, gs, ct, rct = _pair(ctx, n, layers, S, seed, precision, trav)
        assert same_bits(gd, wd), float(np.nanmax(np.abs(gd - wd)))
        assert same_bits(gs, ws)
        for k in ("fwd_gates", "inv_gates", "fwd_paulis", "passes_fwd", "passes_inv", "leaves",
                  "recomputes", "checkpoint_saves", "checkpoint_restores"):
            assert ct[k] == rct[k], k
        assert abs(gd.sum() - 1.0) < 1e-6


def test_noalloc_refuses_what_does_not_fit(ctx):
    _say("[gpu] noalloc refusals")
    dev = torch.device("cuda:0")
    # 22 qubits complex128: a 64 MiB state alone fills the scratch
    c = brickwork(22, 2, 1e-3, 1e-2, 3)
    ec = tq.Circuit(c)
    o = tq.tusq_opts_default(shots=100, seed=1, want=tq.WANT_DIST)
    t = tq.Tree(ec, o)
    dist = torch.zeros(1 << 22, dtype=torch.float64, device=dev)
    with pytest.raises(tq.TusqError) as e:
        tq.tusq_run_tree_noalloc(ctx, ec, t, o, dist.data_ptr(), 0, 0)
    assert e.value.code == -2  # TUSQ_ENOMEM
    # a samples buffer shorter than the shots
    c = brickwork(8, 4, 1e-3, 1e-2, 3)
    ec = tq.Circuit(c)
    o = tq.tusq_opts_default(shots=100, seed=1, want=tq.WANT_SAMPLES)
    t = tq.Tree(ec, o)
    s = torch.zeros(50, dtype=torch.int64, device=dev)
    with pytest.raises(tq.TusqError) as e:
        tq.tusq_run_tree_noalloc(ctx, ec, t, o, 0, s.data_ptr(), 50)
    assert e.value.code == -1  # TUSQ_EINVAL
    # a distribution asked for without a buffer
    o = tq.tusq_opts_default(shots=100, seed=1, want=tq.WANT_DIST)
    with pytest.raises(tq.TusqError) as e:
        tq.tusq_run_tree_noalloc(ctx, ec, t, o, 0, 0, 0)
    assert e.value.code == -1
