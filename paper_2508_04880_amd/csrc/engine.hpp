// engine.hpp -- internal data structures of the noisy statevector engine.
#pragma once

#include <complex>
#include <cstdint>
#include <string>
#include <unordered_map>
#include <vector>

#include "tusq.h"

namespace tusq {

using cd = std::complex<double>;

// ---------------------------------------------------------------------------
// Status handling: internal code throws Error; the C ABI converts it.
struct Error {
    int code;
    std::string msg;
};
[[noreturn]] void fail(int code, const std::string &msg);

// ---------------------------------------------------------------------------
// Circuit
struct Gate {
    uint8_t kind;
    uint32_t q[2];  // measurement layers: the measured-qubit mask, low word in q[0]
    double p[3];
    int32_t chan;   // channel index or -1
    uint32_t umat;  // UNITARY1 / UNITARY2: offset of the matrix in Circuit::umats
};

struct Channel {
    uint32_t gate;
    uint8_t m;           // 3 (1-qubit) or 15 (CX)
    uint64_t thr[15];    // integer cumulative thresholds
    double prob[15];
};

struct Circuit {
    uint32_t n = 0;
    std::vector<Gate> gates;
    std::vector<Channel> chans;  // rebuilt in gate order by finalize()
    std::vector<cd> umats;       // matrices of the caller's unitaries, row-major
    bool dirty = true;
    void finalize();
};

bool is_cx(uint8_t kind);
bool is_two_qubit(uint8_t kind);  // CX or UNITARY2
bool is_measure(uint8_t kind);
inline uint64_t measure_mask(const Gate &g) { return uint64_t(g.q[0]) | (uint64_t(g.q[1]) << 32); }
bool has_measure(const Circuit &c);
void gate_matrix(const Circuit &c, const Gate &g, cd m[4]);  // 2x2 of a 1-qubit gate

// ---------------------------------------------------------------------------
// Error events and the tree of circuits to simulate
struct Ev {
    uint32_t slot;   // applied just before gate `slot` (slot == G: after the last gate)
    uint32_t qubit;
    uint8_t pauli;   // 1 X, 2 Y, 3 Z
};
inline bool ev_less(const Ev &a, const Ev &b) {
    if (a.slot != b.slot) return a.slot < b.slot;
    if (a.qubit != b.qubit) return a.qubit < b.qubit;
    return a.pauli < b.pauli;
}
inline bool ev_eq(const Ev &a, const Ev &b) {
    return a.slot == b.slot && a.qubit == b.qubit && a.pauli == b.pauli;
}

struct Tree {
    uint32_t n = 0, G = 0;
    uint64_t S = 0;
    std::vector<uint64_t> off;   // leaf l's events: ev[off[l] .. off[l+1])
    std::vector<Ev> ev;
    std::vector<uint64_t> count, shots, wnum, wden;
    tusq_tree_info info{};
    std::vector<uint32_t> raw_shot, raw_chan;
    std::vector<uint8_t> raw_out;

    uint64_t leaves() const { return count.size(); }
    uint64_t nev(uint64_t l) const { return off[l + 1] - off[l]; }
    const Ev *evs(uint64_t l) const { return ev.data() + off[l]; }
};

Tree build_tree(const Circuit &c, const tusq_opts &o);
std::vector<uint8_t> serialize_tree(const Tree &t);

// ---------------------------------------------------------------------------
// Plan: the depth-first schedule with its fused sweeps.
//
// A sweep ("pass") touches every amplitude once: the state is cut into tiles
// of 2^k amplitudes whose local index bits are the pass's qubits; each tile
// is staged in LDS, the pass's dense 1- and 2-qubit ops are applied there,
// and the tile is written back.
constexpr int KMAX = 16;  // most qubits a tile may span

struct Op {
    uint8_t a;      // local index of the (first) qubit
    uint8_t b;      // local index of the second qubit, or 0xFF for a 1-qubit op
    uint32_t mat;   // offset (complex numbers) into the matrix pool
    uint32_t adj;   // offset of its adjoint
};

struct Pass {
    uint32_t k = 0;
    uint32_t q[KMAX];
    uint32_t op_begin = 0, op_end = 0;
    uint32_t n_gates = 0, n_paulis = 0;  // tokens fused into it
    // register-blocked programs (forward and undo), see Instr
    uint32_t fwd_begin = 0, fwd_end = 0, inv_begin = 0, inv_end = 0;
    // per direction: layouts the program starts (load) and ends (store) in,
    // as (register word, thread word) pairs, see Instr
    uint32_t lay[2][4] = {};
};

// One instruction of a register-blocked sweep program.  Each thread holds
// 2^R amplitudes of its tile whose local index bits at the R "register
// qubits" vary; the others come from the thread index.  A layout is a
// register word (bits 5i.. of register bit i's local position) and a thread
// word (bits 4b.. of thread-index bit b's local position, or THR_ASC: the
// positions outside the register set in ascending order).
//   IN_RELAYOUT: move the tile through LDS into the layout (arg, mat);
//   IN_OP1:      2x2 matrix on register bit (arg & 7);
//   IN_OP2:      4x4 matrix on register bits a = arg & 7 (high bit of the
//                4x4 index) and b = (arg >> 3) & 7, with a > b;
//   IN_EXCH:     swap register bit r = arg & 7 with thread-index bit
//                h = (arg >> 3) & 7 < 6 (a lane exchange inside the wavefront).
// mat is an offset (complex numbers) into the matrix pool for ops; undo
// programs reference the adjoint matrices, in reverse op order.  Every
// program has even length (padded with a 2x2 identity).
enum : uint32_t { IN_RELAYOUT = 0, IN_OP1 = 1, IN_OP2 = 2, IN_EXCH = 3 };
constexpr uint32_t THR_ASC = 0xFFFFFFFFu;
struct Instr {
    uint32_t w0;  // type | arg << 2
    uint32_t mat;
};

// ST_SAVE / ST_RESTORE (checkpoint traversal): copy the state into / out of
// checkpoint slot `id`
enum StepKind : int64_t { ST_RESET = 0, ST_FWD = 1, ST_INV = 2, ST_LEAF = 3, ST_SAVE = 4,
                          ST_RESTORE = 5 };
struct Step {
    StepKind kind;
    uint64_t id;  // pass index (FWD/INV) or leaf index (LEAF)
};

struct FusionParams {
    uint32_t max_qubits;  // tile qubits
    uint32_t max_ops;     // dense ops per sweep
    uint32_t low_qubits;  // lowest qubits every tile contains (coalescing)
    bool window_search;   // also try the low qubits plus a window of
                          // consecutive qubits as a sweep's tile
};

struct Plan {
    uint32_t n = 0;
    std::vector<Pass> passes;
    std::vector<Op> ops;
    std::vector<cd> mats;
    std::vector<std::pair<uint32_t, uint32_t>> mat_blocks;  // (offset, dim) of each matrix in mats
    std::vector<Step> steps;
    std::vector<Instr> prog;
    uint32_t reg_qubits = 4;  // R of the register-blocked programs
    bool general_layouts = false;  // programs for the persistent kernel (see build_programs)
    std::unordered_map<uint32_t, uint32_t> swapped;  // 4x4 offset -> same op, qubits swapped
    // matrix pool entries by content (bitwise), so that repeated fused ops
    // share one copy: hash -> offset of the matrix (its adjoint follows it)
    std::unordered_multimap<uint64_t, std::pair<uint32_t, int>> mat_index;  // -> (offset, dim)
    uint32_t identity2 = UINT32_MAX;  // pool offset of the 2x2 identity (program padding)
    uint64_t checkpoint_slots = 0;    // states the checkpoint traversal keeps at once
    // per leaf in the range: the passes forming its path from the root, used
    // to recompute a leaf exactly (c64 drift control)
    std::vector<uint64_t> path_off;
    std::vector<uint32_t> path;
    tusq_counters counters{};
};

FusionParams fusion_defaults(uint32_t n, uint32_t precision, const tusq_opts &o);
// programs = false skips the register-blocked programs (callers that run the
// op lists only, or count)
Plan build_plan(const Circuit &c, const Tree &t, const tusq_opts &o, bool keep_paths,
                bool programs = true);
// The plan's matrices for complex64 sweeps, as (re, im) floats: each matrix
// rounded so that its squared Frobenius norm stays the FP64 one (see
// host_plan.cpp).
void mats_to_c64(const Plan &p, std::vector<float> &out);

// ---------------------------------------------------------------------------
// Circuits with mid-circuit measurement layers (DFTT+Caching).  The tokens
// of a leaf split at its measurement gates into stages (stage s: between
// layers s-1 and s).  Every distinct stage token sequence is a McmPath whose
// tokens are fused once, in segments cut at every depth where another path
// of the same stage branches off, so any DFTT transition between two paths
// of a stage moves along whole segments.
struct McmSeg {
    uint32_t p0, p1;        // pass range
    uint32_t gates, paulis;
    uint64_t ops;           // operation count: 1 per 1-qubit token, 4 per CX
};
struct McmPath {
    std::vector<uint64_t> code;  // token codes (gate: 1 << 63 | g; event: its key)
    std::vector<uint64_t> cut;   // 0 = cut[0] < ... < cut.back() = tokens
    std::vector<McmSeg> seg;     // seg[i]: tokens [cut[i], cut[i + 1])
};
struct McmLayer {
    uint32_t gate;
    uint32_t m;                  // measured qubits
    uint32_t q[TUSQ_MAX_MEASURED];
    bool reset;
};
struct McmPlan {
    Plan plan;                   // passes, ops, matrices and programs of every segment
    uint64_t lb = 0, le = 0;
    uint32_t M = 0, K = 0;       // layers, effective cache capacity (<= M)
    std::vector<McmLayer> layers;
    std::vector<McmPath> paths;
    std::vector<uint32_t> leaf_path;  // (l - lb) * (M + 1) + s -> path of leaf l in stage s
};
McmPlan build_mcm_plan(const Circuit &c, const Tree &t, const tusq_opts &o, bool programs = true);
// real floating-point operations of one launch of a pass (see sweep_flops)
uint64_t plan_pass_flops(const Plan &plan, uint32_t pass);

double now_seconds();
unsigned host_threads(const tusq_opts &o);

}  // namespace tusq

struct tusq_circuit {
    tusq::Circuit c;
};
struct tusq_tree {
    tusq::Tree t;
};
