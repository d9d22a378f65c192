"""Host-side parity of the engine (no GPU needed): the C ABI loads and
exports what include/tusq.h declares; the engine's error characterisation
(ER sampling, tallying, commutation, pruning, leaf order) reproduces the
oracle's tree and raw-ER stream bit for bit; its depth-first schedule makes
the oracle's gate/Pauli application counts; and its fused sweeps, applied
with NumPy, give the oracle's distribution."""

import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_2508_04880_amd as tq
from workloads import brickwork, ising, random_small_circuit, Circuit, bell_pair
from workloads.circuits import depol1, depol2

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    with open(os.path.join(ROOT, "include", "tusq.h")) as f:
        src = f.read()
    names = set(re.findall(r"\b(tusq_[a-z0-9_]+)\s*\(", src))
    assert len(names) >= 30
    lib = ctypes.CDLL(tq.LIB_PATH)
    missing = [n for n in sorted(names) if not hasattr(lib, n)]
    assert not missing, missing
    assert tq.lib.tusq_abi_version() == tq.ABI_VERSION == 10


def test_product_binding_has_no_oracle_dependency():
    pkg = os.path.join(ROOT, "paper_2508_04880_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".cpp", ".hip", ".hpp", ".h")):
                with open(os.path.join(dirpath, fn)) as f:
                    text = f.read()
                assert "import oracle" not in text and "from oracle" not in text, fn
                assert "tusq_oracle" not in text and "liboracle" not in text, fn


CASES = [
    ("brick8", lambda: brickwork(8, 20, 1e-3, 1e-2, 1), 10_000),
    ("brick6_noisy", lambda: brickwork(6, 12, 0.02, 0.05, 3), 5_000),
    ("ising8", lambda: ising(8, 6, 5e-3, 2e-2), 8_000),
    ("soup5", lambda: random_small_circuit(5, 60, 4, p1=0.03, p2=0.06), 6_000),
    ("soup4_axis", lambda: random_small_circuit(
        4, 80, 9, p1=0.05, p2=0.05, kinds=("RX", "RY", "RZ", "CX", "X", "Y", "Z", "H")), 6_000),
    ("bell", lambda: bell_pair(0.1, 0.2), 3_000),
]


@pytest.mark.slow
@pytest.mark.parametrize("name,make", [
    ("brickwork26_L100", lambda: brickwork(26, 100, 1e-3, 1e-2, 1)),
    ("ising30_T20", lambda: ising(30, 20, 5e-4, 5e-3))])
def test_full_size_tree_bit_exact_against_oracle(name, make):
    """The two HBM-scale workloads at their full 10^6 shots: the engine's
    tree (all significant leaves at 26 qubits; 101 pruned leaves at 30)
    and its raw-ER stream equal the oracle's byte for byte."""
    c = make()
    S, seed = 1_000_000, 2
    threads = min(os.cpu_count() or 1, 16)
    oracle.set_threads(threads)
    try:
        ot = oracle.ecm(c, S, seed)
    finally:
        oracle.set_threads(1)
    ec = tq.Circuit(c)
    et = tq.Tree(ec, tq.tusq_opts_default(shots=S, seed=seed, host_threads=threads))
    assert et.info()["n_leaves"] == ot.n_leaves
    a, b = et.serialize(), ot.serialize()
    assert len(a) == len(b) and a == b
    del a, b
    import hashlib
    assert et.raw_er_hash() == hashlib.sha256(_raw_bytes(*ot.raw_events())).digest()


@pytest.mark.parametrize("name,make,S", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("commute,prune,alpha,beta", [
    (True, True, (1, 100), 100), (True, False, (1, 100), 100), (False, True, (1, 100), 100),
    (True, True, (1, 20), 7), (False, False, (1, 100), 100)])
def test_tree_bit_exact_against_oracle(name, make, S, commute, prune, alpha, beta):
    c = make()
    seed = 1234 + S
    ot = oracle.ecm(c, S, seed, do_commute=commute, prune=prune, alpha=alpha, beta=beta)
    ec = tq.Circuit(c)
    o = tq.tusq_opts_default(shots=S, seed=seed, commute=int(commute), prune=int(prune),
                             alpha=alpha, beta=beta, host_threads=3)
    et = tq.Tree(ec, o)
    assert et.serialize() == ot.serialize()
    for a, b in zip(ot.raw_events(), et.raw_events()):
        np.testing.assert_array_equal(a, b)
    info = et.info()
    for k in ("raw_unique", "canonical_unique", "significant", "insignificant", "s_max"):
        assert info[k] == ot.stats[k], k


def test_tree_independent_of_host_thread_count():
    c = brickwork(10, 15, 2e-3, 2e-2, 5)
    outs = []
    for th in (1, 2, 7):
        o = tq.tusq_opts_default(shots=20_000, seed=9, host_threads=th)
        outs.append(tq.Tree(tq.Circuit(c), o).serialize())
    assert outs[0] == outs[1] == outs[2]


@pytest.mark.parametrize("trav", ["dftt", "naive", "hybrid", "checkpoint"])
@pytest.mark.parametrize("name,make,S", CASES[:4], ids=[c[0] for c in CASES[:4]])
def test_schedule_counts_match_oracle(trav, name, make, S):
    c = make()
    ot = oracle.ecm(c, S, 5, prune=False)
    ec = tq.Circuit(c)
    o = tq.tusq_opts_default(shots=S, seed=5, prune=0, traversal=trav)
    et = tq.Tree(ec, o)
    pc = tq.tusq_plan_counters(ec, et, o)
    _, _, oc, _ = oracle.run(c, ot, 5, traversal=trav, want_dist=False, want_samples=False)
    for k in ("fwd_gates", "inv_gates", "fwd_paulis", "inv_paulis", "resets", "leaves",
              "ret_gates", "ret_paulis", "checkpoint_saves", "checkpoint_restores", "paper_ops"):
        assert pc[k] == oc[k], k
    if trav == "checkpoint":
        for slots in (1, 2, 3):
            o3 = tq.tusq_opts_default(shots=S, seed=5, prune=0, traversal=trav,
                                      checkpoint_slots=slots)
            pc3 = tq.tusq_plan_counters(ec, et, o3)
            _, _, oc3, _ = oracle.run(c, ot, 5, traversal=trav, want_dist=False,
                                      want_samples=False, checkpoint_slots=slots)
            for k in ("fwd_gates", "inv_gates", "fwd_paulis", "inv_paulis", "resets",
                      "checkpoint_saves", "checkpoint_restores", "paper_ops"):
                assert pc3[k] == oc3[k], (slots, k)
    # a leaf range starts from the root
    nl = et.info()["n_leaves"]
    if nl > 6:
        o2 = tq.tusq_opts_default(shots=S, seed=5, prune=0, traversal=trav, leaf_begin=2,
                                  leaf_end=nl - 3)
        pc2 = tq.tusq_plan_counters(ec, et, o2)
        _, _, oc2, _ = oracle.run(c, ot, 5, traversal=trav, leaf_begin=2, leaf_end=nl - 3,
                                  want_dist=False, want_samples=False)
        for k in ("fwd_gates", "inv_gates", "fwd_paulis", "inv_paulis", "resets", "leaves",
                  "checkpoint_saves", "checkpoint_restores"):
            assert pc2[k] == oc2[k], k


# --------------------------------------------------------------------------
# The fused sweeps, executed with NumPy on the full state

def _apply_local(psi, n, qubits, op, M, inverse):
    a, b = int(op[0]), int(op[1])
    st = psi.reshape([2] * n)  # axis n-1-q is qubit q
    if b == 0xFF:
        m = M.reshape(2, 2)
        if inverse:
            m = m.conj().T
        ax = n - 1 - int(qubits[a])
        st = np.moveaxis(np.tensordot(m, st, axes=([1], [ax])), 0, ax)
    else:
        m = M.reshape(4, 4)
        if inverse:
            m = m.conj().T
        qa, qb = int(qubits[a]), int(qubits[b])
        axa, axb = n - 1 - qa, n - 1 - qb
        m4 = m.reshape(2, 2, 2, 2)  # (ra, rb, ca, cb)
        st = np.tensordot(m4, st, axes=([2, 3], [axa, axb]))
        st = np.moveaxis(st, [0, 1], [axa, axb])
    return st.reshape(-1)


def _run_plan_numpy(c, dump, weights, lb):
    n = c.n
    psi = np.zeros(1 << n, complex)
    acc = np.zeros(1 << n)
    slots = {}
    for kind, ident in dump["steps"]:
        if kind == 4:            # checkpoint save
            slots[ident] = psi.copy()
            continue
        if kind == 5:            # checkpoint restore
            psi = slots[ident].copy()
            continue
        if kind == 0:
            psi[:] = 0
            psi[0] = 1
        elif kind in (1, 2):
            inv = kind == 2
            q = dump["qubits"][ident]
            b0, cnt = dump["op_range"][ident]
            rng = range(b0, b0 + cnt)
            for i in (reversed(rng) if inv else rng):
                op = dump["ops"][i]
                size = 4 if op[1] == 0xFF else 16
                M = dump["mats"][op[2]: op[2] + size]
                psi = _apply_local(psi, n, q, op, M, inv)
        else:
            acc += weights[ident] * np.abs(psi) ** 2
    return acc


@pytest.mark.parametrize("search", [1, 2])
@pytest.mark.parametrize("trav", ["dftt", "naive", "hybrid", "checkpoint"])
@pytest.mark.parametrize("kmax,low,maxops", [(3, 1, 2), (4, 2, 5), (5, 3, 12), (16, 5, 12)])
def test_fused_plan_reproduces_oracle_distribution(trav, kmax, low, maxops, search):
    c = brickwork(7, 8, 0.02, 0.05, 11)
    S = 3000
    ot = oracle.ecm(c, S, 3, prune=True, alpha=(1, 50), beta=20)
    dist, _, _, _ = oracle.run(c, ot, 3, traversal=trav, want_samples=False)
    ec = tq.Circuit(c)
    o = tq.tusq_opts_default(shots=S, seed=3, alpha=(1, 50), beta=20, traversal=trav,
                             fusion_max_qubits=kmax, fusion_low_qubits=low,
                             fusion_max_ops=maxops, fusion_search=search)
    et = tq.Tree(ec, o)
    dump = tq.tusq_plan_dump(ec, et, o)
    if kmax < c.n:
        assert all((q[:kmax] != 0xFFFFFFFF).all() for q in dump["qubits"])
    acc = _run_plan_numpy(c, dump, ot.weights(), 0)
    np.testing.assert_allclose(acc, dist, atol=1e-12)


THR_ASC = 0xFFFFFFFF


def _layout(k, r, reg_word, thr_word):
    """(register positions, thread positions) of a layout's two words."""
    reg = [(reg_word >> (5 * i)) & 31 for i in range(r)]
    if thr_word == THR_ASC:
        thr = [p for p in range(k) if p not in reg]
    else:   # a 9th thread bit's position sits in bits 20..23 of the register word
        thr = [(thr_word >> (4 * b)) & 15 if b < 8 else (reg_word >> 20) & 15
               for b in range(k - r)]
    assert sorted(reg + thr) == list(range(k)), (reg, thr)
    return reg, thr


def _run_programs_numpy(c, dump, progs, weights):
    """Replay the register-blocked programs: a re-layout or lane exchange
    only changes which local qubits the register bits name; ops act on
    those qubits.  Also checks the program form the kernels rely on."""
    n = c.n
    R = progs["reg_qubits"]
    psi = np.zeros(1 << n, complex)
    acc = np.zeros(1 << n)
    slots = {}
    for kind, ident in dump["steps"]:
        if kind == 4:
            slots[ident] = psi.copy()
            continue
        if kind == 5:
            psi = slots[ident].copy()
            continue
        if kind == 0:
            psi[:] = 0
            psi[0] = 1
            continue
        if kind == 3:
            acc += weights[ident] * np.abs(psi) ** 2
            continue
        q = dump["qubits"][ident]
        k = int((q != 0xFFFFFFFF).sum())
        r = min(R, k)
        low = 0
        while low < k and q[low] == low:
            low += 1
        rg = progs["ranges"][ident]
        inv = kind == 2
        b, e = (rg[2], rg[3]) if inv else (rg[0], rg[1])
        lay = rg[8:12] if inv else rg[4:8]
        reg, thr = _layout(k, r, int(lay[0]), int(lay[1]))
        end_reg, end_thr = _layout(k, r, int(lay[2]), int(lay[3]))
        # loads and stores move contiguous runs: the lowest local positions
        # sit at the lowest thread bits
        lowc = min(low, 4, k - r)
        for lay_thr in (thr, end_thr):
            assert lay_thr[:lowc] == list(range(lowc))
        assert (e - b) % 2 == 0      # instructions run in pairs
        # the kernel reads slot s from register array s % 2 and writes the
        # other; every instruction is one of the four forms below
        for w0, mat in progs["instr"][b:e]:
            typ, arg = int(w0) & 3, int(w0) >> 2
            swaps = []
            if typ == 0:
                reg, thr = _layout(k, r, arg, int(mat))
            elif typ == 1:
                assert (arg & 7) < r and ((arg >> 3) & 7) == 0
                M = dump["mats"][mat: mat + 4]
                psi = _apply_local(psi, n, q, (reg[arg & 7], 0xFF), M, False)
            elif typ == 2:
                assert r > (arg & 7) > ((arg >> 3) & 7)
                M = dump["mats"][mat: mat + 16]
                psi = _apply_local(psi, n, q, (reg[arg & 7], reg[(arg >> 3) & 7]), M, False)
            else:
                assert arg >> 6 == 0
                swaps = [arg & 63]
            if typ in (1, 2):
                assert arg >> 6 == 0
            for xa in swaps:
                # lane exchange: thread bits 0 .. 5 are the lane bits of full wavefronts
                assert k - r >= 6
                ri, h = xa & 7, xa >> 3
                assert ri < r and h < 6
                reg[ri], thr[h] = thr[h], reg[ri]
        assert (reg, thr) == (end_reg, end_thr)
    return acc


@pytest.mark.parametrize("kernel", [0, 1, 5])
@pytest.mark.parametrize("precision", ["c128", "c64"])
@pytest.mark.parametrize("trav", ["dftt", "hybrid", "checkpoint"])
@pytest.mark.parametrize("n,kmax,low,maxops", [(8, 6, 2, 4), (8, 7, 3, 12), (8, 16, 5, 12),
                                               (12, 10, 4, 16), (13, 12, 4, 24), (14, 13, 4, 32)])
def test_register_programs_reproduce_oracle(kernel, precision, trav, n, kmax, low, maxops):
    c = brickwork(n, 6, 0.02, 0.05, 12)
    S = 3000
    ot = oracle.ecm(c, S, 4, prune=True, alpha=(1, 50), beta=20)
    dist, _, _, _ = oracle.run(c, ot, 4, traversal=trav, want_samples=False)
    ec = tq.Circuit(c)
    o = tq.tusq_opts_default(shots=S, seed=4, alpha=(1, 50), beta=20, traversal=trav,
                             precision=precision, fusion_max_qubits=kmax,
                             fusion_low_qubits=low, fusion_max_ops=maxops, sweep_kernel=kernel)
    et = tq.Tree(ec, o)
    dump = tq.tusq_plan_dump(ec, et, o)
    progs = tq.tusq_plan_dump_programs(ec, et, o)
    assert progs["reg_qubits"] == (3 if kernel in (3, 5) else 4)
    acc = _run_programs_numpy(c, dump, progs, ot.weights())
    np.testing.assert_allclose(acc, dist, atol=1e-12)
    if kernel in (1, 2, 3):     # one-tile kernels: start and end in the top R qubits
        assert all(int(r[5]) == 0xFFFFFFFF and int(r[9]) == 0xFFFFFFFF
                   for r in progs["ranges"])
        assert not any(int(w) & 3 == 3 for w, _ in progs["instr"])


def test_fused_plan_ising_and_soup():
    for c in (ising(6, 4, 1e-2, 3e-2), random_small_circuit(6, 70, 2, p1=0.03, p2=0.05)):
        ot = oracle.ecm(c, 4000, 8, prune=False)
        dist, _, _, _ = oracle.run(c, ot, 8, want_samples=False)
        ec = tq.Circuit(c)
        o = tq.tusq_opts_default(shots=4000, seed=8, prune=0, fusion_max_qubits=4,
                                 fusion_low_qubits=2, fusion_max_ops=3)
        et = tq.Tree(ec, o)
        acc = _run_plan_numpy(c, tq.tusq_plan_dump(ec, et, o), ot.weights(), 0)
        np.testing.assert_allclose(acc, dist, atol=1e-12)


# --------------------------------------------------------------------------
# Validation at the boundary

def test_invalid_inputs_are_rejected():
    lib = tq.lib
    h = ctypes.c_void_p()
    assert lib.tusq_circuit_create(0, ctypes.byref(h)) == -1
    assert lib.tusq_circuit_create(3, ctypes.byref(h)) == 0
    q = (ctypes.c_uint32 * 2)(3, 0)
    assert lib.tusq_circuit_gate(h, 0, q, None, None) == -1
    assert b"range" in lib.tusq_last_error()
    q = (ctypes.c_uint32 * 2)(1, 1)
    assert lib.tusq_circuit_gate(h, 12, q, None, None) == -1      # CX with equal qubits
    assert lib.tusq_circuit_gate(h, 99, q, None, None) == -1      # unknown kind
    q = (ctypes.c_uint32 * 2)(0, 1)
    gi = ctypes.c_uint32()
    assert lib.tusq_circuit_gate(h, 12, q, None, ctypes.byref(gi)) == 0
    p3 = (ctypes.c_double * 3)(0.1, 0.1, 0.1)
    assert lib.tusq_circuit_pauli_noise(h, gi, p3, 3) == -1       # CX needs 15
    bad = (ctypes.c_double * 15)(*([0.1] * 15))
    assert lib.tusq_circuit_pauli_noise(h, gi, bad, 15) == -1     # sums above 1
    neg = (ctypes.c_double * 15)(*([-0.01] + [0.0] * 14))
    assert lib.tusq_circuit_pauli_noise(h, gi, neg, 15) == -1
    ok = (ctypes.c_double * 15)(*([0.01] * 15))
    assert lib.tusq_circuit_pauli_noise(h, gi, ok, 15) == 0
    assert lib.tusq_circuit_pauli_noise(h, gi, ok, 15) == -1      # one channel per gate
    o = tq.tusq_opts_default(shots=0)
    t = ctypes.c_void_p()
    assert lib.tusq_ecm_build(h, ctypes.byref(o), ctypes.byref(t)) == -1
    for bad_opt in (dict(traversal=5), dict(fusion_search=3), dict(precision=2)):
        o = tq.tusq_opts_default(shots=10, **bad_opt)
        assert lib.tusq_ecm_build(h, ctypes.byref(o), ctypes.byref(t)) == -1, bad_opt
    assert lib.tusq_circuit_destroy(h) == 0
    assert lib.tusq_circuit_destroy(None) == 0
    assert lib.tusq_result_destroy(None) == 0


# --------------------------------------------------------------------------
# Twirled thermal relaxation at the boundary (Eq. (4))

def test_thermal_probs_match_oracle_and_reject_bad_times():
    rng = np.random.default_rng(5)
    for _ in range(200):
        t1 = float(rng.uniform(0.1, 10))
        t2 = float(rng.uniform(0.05, 2 * t1))
        t = float(rng.uniform(0, 3))
        got = tq.tusq_thermal_pauli_probs(t, t1, t2)
        assert list(got) == oracle.thermal_probs(t, t1, t2)
    for bad in ((-1.0, 1.0, 1.0), (1.0, 0.0, 1.0), (1.0, 1.0, -1.0), (1.0, 1.0, 2.5),
                (float("nan"), 1.0, 1.0)):
        with pytest.raises(tq.TusqError) as e:
            tq.tusq_thermal_pauli_probs(*bad)
        assert e.value.code == -1


def test_thermal_noise_attached_by_the_library_gives_the_oracle_tree():
    """A brickwork circuit with the twirled channel after every gate: built
    through tusq_circuit_thermal_noise it yields the same tree, byte for byte,
    as the oracle's own circuit with oracle-computed probabilities."""
    base = brickwork(6, 6, 0.0, 0.0, 21)
    t_1q, t_2q, T1, T2 = 0.02, 0.1, 1.0, 0.8
    c = Circuit(6)
    for k, q, p in zip(base.kinds, base.qubits, base.params):
        c.add(k, q, p, oracle.thermal_probs(t_2q if k == "CX" else t_1q, T1, T2,
                                            two_qubit=(k == "CX")))
    ec = tq.Circuit(Circuit(6, kinds=list(base.kinds), qubits=list(base.qubits),
                            params=list(base.params), noise=[None] * base.n_gates))
    for g, k in enumerate(base.kinds):
        ec.thermal_noise(g, t_2q if k == "CX" else t_1q, T1, T2)
    S, seed = 4000, 3
    ot = oracle.ecm(c, S, seed)
    o = tq.tusq_opts_default(shots=S, seed=seed)
    assert tq.Tree(ec, o).serialize() == ot.serialize()
    with pytest.raises(tq.TusqError):
        ec.thermal_noise(0, 0.1, 1.0, 1.0)       # the gate already has a channel


@pytest.mark.parametrize("commute,prune", [(True, True), (True, False), (False, True)])
def test_user_unitary_trees_equal_the_oracle(commute, prune):
    """Circuits mixing named gates with a caller's UNITARY1 / UNITARY2
    (tusq_circuit_gate copies the matrix): the library's tree equals the
    oracle's byte for byte."""
    from workloads.circuits import unitary_mix
    for seed in range(3):
        c = unitary_mix(6, 40, seed)
        ot = oracle.ecm(c, 3000, 5 + seed, do_commute=commute, prune=prune)
        o = tq.tusq_opts_default(shots=3000, seed=5 + seed, commute=int(commute),
                                 prune=int(prune))
        assert tq.Tree(tq.Circuit(c), o).serialize() == ot.serialize()


@pytest.mark.parametrize("kernel", [0, 4])
def test_user_unitary_programs_reproduce_oracle(kernel):
    """The fused register programs of a circuit with a caller's unitaries,
    replayed on the CPU, give the oracle's distribution."""
    from workloads.circuits import unitary_mix
    c = unitary_mix(10, 60, 7)
    S = 3000
    ot = oracle.ecm(c, S, 4)
    dist, _, _, _ = oracle.run(c, ot, 4, want_samples=False)
    ec = tq.Circuit(c)
    o = tq.tusq_opts_default(shots=S, seed=4, fusion_max_qubits=8, fusion_low_qubits=2,
                             fusion_max_ops=12, sweep_kernel=kernel)
    et = tq.Tree(ec, o)
    acc = _run_programs_numpy(c, tq.tusq_plan_dump(ec, et, o),
                              tq.tusq_plan_dump_programs(ec, et, o), ot.weights())
    np.testing.assert_allclose(acc, dist, atol=1e-12)


def test_unitary_gate_arguments_are_checked():
    import ctypes as C
    h = C.c_void_p()
    assert tq.lib.tusq_circuit_create(C.c_uint32(3), C.byref(h)) == 0
    try:
        q = (C.c_uint32 * 2)(0, 1)
        same = (C.c_uint32 * 2)(1, 1)
        eye2 = (C.c_double * 8)(1, 0, 0, 0, 0, 0, 1, 0)
        eye4 = (C.c_double * 32)(*[float(i % 10 == 0 and i % 2 == 0) for i in range(32)])
        bad = (C.c_double * 8)(1, 0, 1, 0, 0, 0, 1, 0)          # [[1, 1], [0, 1]]
        nan = (C.c_double * 8)(float("nan"), 0, 0, 0, 0, 0, 1, 0)
        g = C.c_uint32()
        assert tq.lib.tusq_circuit_gate(h, 15, q, eye2, C.byref(g)) == 0 and g.value == 0
        assert tq.lib.tusq_circuit_gate(h, 16, q, eye4, C.byref(g)) == 0 and g.value == 1
        for kind, qs, m in ((15, q, bad), (15, q, nan), (15, q, None), (16, same, eye4),
                            (17, q, eye2)):
            assert tq.lib.tusq_circuit_gate(h, kind, qs, m, C.byref(g)) == -1
        p3 = (C.c_double * 3)(0.1, 0, 0)
        p15 = (C.c_double * 15)(*([0.01] * 15))
        assert tq.lib.tusq_circuit_pauli_noise(h, 1, p3, 3) == -1
        assert tq.lib.tusq_circuit_pauli_noise(h, 1, p15, 15) == 0
        assert tq.lib.tusq_circuit_pauli_noise(h, 0, p3, 3) == 0
        assert tq.lib.tusq_circuit_gate(h, 0, q, None, C.byref(g)) == 0 and g.value == 2
    finally:
        tq.lib.tusq_circuit_destroy(h)


def _raw_bytes(shot, chan, out):
    rec = np.zeros(len(shot), dtype=[("s", "<u4"), ("c", "<u4"), ("o", "u1")])
    rec["s"], rec["c"], rec["o"] = shot, chan, out
    return rec.tobytes()


def test_raw_er_hash_is_sha256_of_the_oracles_raw_events():
    """tusq_raw_er_hash equals hashlib's SHA-256 of the oracle's raw events
    (9 bytes each: u32 shot, u32 channel, u8 outcome): no events (the
    standard's digest of the empty message), lists whose byte length falls
    on either side of the padding boundaries (55 / 56 / 64 bytes mod 64),
    and a large list."""
    import hashlib
    c0 = random_small_circuit(4, 10, 1, p1=0.0, p2=0.0)
    et = tq.Tree(tq.Circuit(c0), tq.tusq_opts_default(shots=50, seed=1))
    assert et.raw_er_hash() == hashlib.sha256(b"").digest()
    assert et.raw_er_hash().hex().startswith("e3b0c442")
    seen = set()
    cases = [(S, 0.5) for S in range(1, 41)] + [(20000, 0.05)]
    for S, p in cases:
        c = random_small_circuit(5, 30, 2, p1=p, p2=p)
        ot = oracle.ecm(c, S, 9)
        et = tq.Tree(tq.Circuit(c), tq.tusq_opts_default(shots=S, seed=9))
        msg = _raw_bytes(*ot.raw_events())
        seen.add(len(msg) % 64)
        assert et.raw_er_hash() == hashlib.sha256(msg).digest(), (S, len(msg))
    # a residue that still fits the length in the last block, and one that
    # pushes it into an extra block
    assert seen & set(range(48, 56)) and seen & set(range(56, 64)), sorted(seen)


def test_readout_noise_through_the_library_gives_the_oracle_tree():
    """Read-out flips (Sec. IV-D) appended through tusq_circuit_readout_noise
    give the same tree, byte for byte, as the oracle's circuit with the same
    flips written as RZ(0) gates carrying an X channel; bad arguments are
    refused and append nothing."""
    base = brickwork(6, 6, 1e-3, 1e-2, 21)
    flips = [0.01, 0.02, 0.0, 0.05, 0.3, 1.0]
    c = Circuit(6, kinds=list(base.kinds), qubits=list(base.qubits),
                params=list(base.params), noise=list(base.noise))
    ec = tq.Circuit(Circuit(6, kinds=list(base.kinds), qubits=list(base.qubits),
                            params=list(base.params), noise=list(base.noise)))
    for q, p in enumerate(flips):
        assert ec.readout_noise(q, p) == c.add_readout_noise(q, p)
    S, seed = 4000, 3
    ot = oracle.ecm(c, S, seed)
    o = tq.tusq_opts_default(shots=S, seed=seed)
    assert tq.Tree(ec, o).serialize() == ot.serialize()
    for q, p in ((0, -0.1), (0, 1.5), (0, float("nan")), (6, 0.1)):
        with pytest.raises(tq.TusqError) as e:
            ec.readout_noise(q, p)
        assert e.value.code == -1
    # nothing was appended by the refused calls
    assert ec.readout_noise(0, 0.1) == base.n_gates + len(flips)


# --------------------------------------------------------------------------
# Measurement layers (Sec. III-B.2): host side

def test_measurement_tree_bit_exact_against_oracle():
    from workloads import syndrome_rounds
    for theta, commute in ((0.0, True), (0.7, True), (0.7, False)):
        c = syndrome_rounds(3, 3, 0.02, 0.05, theta=theta)
        ot = oracle.ecm(c, 3000, 9, do_commute=commute, prune=False)
        o = tq.tusq_opts_default(shots=3000, seed=9, prune=0, commute=int(commute))
        et = tq.Tree(tq.Circuit(c), o)
        assert et.serialize() == ot.serialize()


def test_measurement_layer_arguments_are_checked():
    import ctypes as C
    h = C.c_void_p()
    assert tq.lib.tusq_circuit_create(C.c_uint32(4), C.byref(h)) == 0
    try:
        q = (C.c_uint32 * 9)(0, 1, 2, 3, 0, 1, 2, 3, 0)
        assert tq.lib.tusq_circuit_measure(h, q, C.c_uint32(9), 1, None) == tq._lib.TUSQ_EINVAL
        assert tq.lib.tusq_circuit_measure(h, q, C.c_uint32(0), 1, None) == tq._lib.TUSQ_EINVAL
        rep = (C.c_uint32 * 2)(1, 1)
        assert tq.lib.tusq_circuit_measure(h, rep, C.c_uint32(2), 0, None) == tq._lib.TUSQ_EINVAL
        bad = (C.c_uint32 * 1)(4)
        assert tq.lib.tusq_circuit_measure(h, bad, C.c_uint32(1), 0, None) == tq._lib.TUSQ_EINVAL
        gi = C.c_uint32()
        ok = (C.c_uint32 * 2)(3, 1)
        assert tq.lib.tusq_circuit_measure(h, ok, C.c_uint32(2), 1, C.byref(gi)) == 0
        probs = (C.c_double * 3)(0.1, 0.1, 0.1)
        assert tq.lib.tusq_circuit_pauli_noise(h, gi, probs, C.c_uint32(3)) == tq._lib.TUSQ_EINVAL
    finally:
        tq.lib.tusq_circuit_destroy(h)


def test_measurement_circuits_refuse_other_traversals_and_pruning():
    from workloads import syndrome_rounds
    c = syndrome_rounds(2, 2, 0.01, 0.01)
    ec = tq.Circuit(c)
    o = tq.tusq_opts_default(shots=100, seed=1, prune=0)
    t = tq.Tree(ec, o)
    with pytest.raises(tq.TusqError) as e:
        tq.tusq_plan_counters(ec, t, o)
    assert e.value.code == tq._lib.TUSQ_EUNSUPPORTED


def test_window_search_fuses_brickwork_into_fewer_sweeps():
    """Tiles chosen as the low qubits plus the best window of consecutive
    qubits take more tokens per sweep than the tokens-in-order tile on a
    nearest-neighbour brickwork, at the same dense-op work."""
    c = brickwork(16, 30, 1e-3, 1e-2, 2)
    ec = tq.Circuit(c)
    o = tq.tusq_opts_default(shots=2000, seed=1, leaf_begin=0, leaf_end=4)
    t = tq.Tree(ec, o)
    got = {}
    for search in (1, 2):
        o = tq.tusq_opts_default(shots=2000, seed=1, leaf_begin=0, leaf_end=4,
                                 fusion_max_qubits=8, fusion_max_ops=32, fusion_search=search)
        got[search] = tq.tusq_plan_counters(ec, t, o)
    assert got[2]["passes_fwd"] < 0.8 * got[1]["passes_fwd"]
    assert got[2]["fwd_gates"] == got[1]["fwd_gates"]
