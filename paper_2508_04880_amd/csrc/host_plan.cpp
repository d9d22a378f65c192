// host_plan.cpp -- the depth-first traversal schedule (TUSQ Sec. III-B) and
// the fusion of its gate/error tokens into HBM sweeps.
//
// A leaf's path from |0...0> is its token list: for slot s = 0..G, the
// leaf's errors at slot s (qubit order), then gate s.  Consecutive leaves in
// depth-first order share a prefix; the plan undoes the previous leaf back
// to the deepest shared node with inverse sweeps and goes down to the next
// leaf (plain DFTT), or restarts from |0...0> (naive), or takes the cheaper
// of the two (hybrid).  Every point where some later transition stops its
// undo is a cut: tokens between cuts form a segment, and a segment is fused
// into sweeps that are undone as a unit (their inverses, in reverse order).
#include <algorithm>
#include <map>
#include <array>
#include <cmath>
#include <cstring>
#include <thread>

#include "engine.hpp"

namespace tusq {

namespace {

struct Tok {
    bool is_gate;
    uint32_t idx;  // gate index, or event index within the leaf
};

// Token at position p of a leaf, given the leaf's events.  Position p counts
// gates and events interleaved by slot.
void leaf_tokens(uint32_t G, const Ev *ev, uint64_t ne, std::vector<Tok> &out) {
    out.clear();
    uint64_t e = 0;
    for (uint32_t s = 0; s <= G; ++s) {
        while (e < ne && ev[e].slot == s) out.push_back(Tok{false, static_cast<uint32_t>(e++)});
        if (s < G) out.push_back(Tok{true, s});
    }
}

// Shared depth of two leaves: first differing event j, branch slot b (the
// smaller slot of the two events there); the common prefix is gates [0, b)
// and events [0, j): b + j tokens.
uint64_t shared_depth(uint32_t G, const Ev *a, uint64_t na, const Ev *b, uint64_t nb) {
    uint64_t j = 0;
    while (j < na && j < nb && ev_eq(a[j], b[j])) ++j;
    const uint64_t sa = j < na ? a[j].slot : uint64_t(G) + 1;
    const uint64_t sb = j < nb ? b[j].slot : uint64_t(G) + 1;
    return std::min<uint64_t>(std::min(sa, sb), G) + j;
}

using M2 = std::array<cd, 4>;
using M4 = std::array<cd, 16>;

// complex product written out: the same two products and sum as the
// library's operator for finite operands, without its NaN/infinity recovery
// call (the matrices here are finite)
inline cd cm(const cd &a, const cd &b) {
    return cd(a.real() * b.real() - a.imag() * b.imag(), a.real() * b.imag() + a.imag() * b.real());
}

M4 kron(const M2 &a, const M2 &b) {
    M4 r;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int k = 0; k < 2; ++k)
                for (int l = 0; l < 2; ++l) r[(2 * i + k) * 4 + (2 * j + l)] = cm(a[2 * i + j], b[2 * k + l]);
    return r;
}
M4 mul4(const M4 &a, const M4 &b) {
    M4 r;
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            cd s = 0.0;
            for (int k = 0; k < 4; ++k) s += cm(a[4 * i + k], b[4 * k + j]);
            r[4 * i + j] = s;
        }
    return r;
}
M2 mul2(const M2 &a, const M2 &b) {
    return M2{cm(a[0], b[0]) + cm(a[1], b[2]), cm(a[0], b[1]) + cm(a[1], b[3]),
              cm(a[2], b[0]) + cm(a[3], b[2]), cm(a[2], b[1]) + cm(a[3], b[3])};
}
const M2 I2m{1.0, 0.0, 0.0, 1.0};

// Products with a Kronecker factor, the terms of mul4 that are not zero
// (same operands, same order of summation): (A (x) I) M, (I (x) A) M and
// G (A (x) B).  Basis index 2 * high + low; the first Kronecker factor acts
// on the high bit.
M4 mul_hi(const M2 &a, const M4 &m) {  // (A (x) I) M
    M4 r;
    for (int i = 0; i < 2; ++i)
        for (int s = 0; s < 2; ++s)
            for (int c = 0; c < 4; ++c)
                r[4 * (2 * i + s) + c] = cm(a[2 * i], m[4 * s + c]) + cm(a[2 * i + 1], m[4 * (2 + s) + c]);
    return r;
}
M4 mul_lo(const M2 &a, const M4 &m) {  // (I (x) A) M
    M4 r;
    for (int h = 0; h < 2; ++h)
        for (int i = 0; i < 2; ++i)
            for (int c = 0; c < 4; ++c)
                r[4 * (2 * h + i) + c] = cm(a[2 * i], m[4 * (2 * h) + c]) + cm(a[2 * i + 1], m[4 * (2 * h + 1) + c]);
    return r;
}
bool is_identity(const M2 &a) { return a[0] == 1.0 && a[1] == 0.0 && a[2] == 0.0 && a[3] == 1.0; }
M4 mul_kron(const M4 &g, const M2 &a, const M2 &b) {  // G (A (x) B)
    if (is_identity(a) && is_identity(b)) return g;
    return mul4(g, kron(a, b));
}
M4 cx_matrix() {  // basis index 2 * control + target
    M4 r{};
    r[0 * 4 + 0] = 1.0;
    r[1 * 4 + 1] = 1.0;
    r[2 * 4 + 3] = 1.0;
    r[3 * 4 + 2] = 1.0;
    return r;
}
const M4 CX_MATRIX = cx_matrix();
M4 swap_halves(const M4 &m) {  // same operator written for the qubit pair in the other order
    static const int p[4] = {0, 2, 1, 3};
    M4 r;
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) r[4 * p[i] + p[j]] = m[4 * i + j];
    return r;
}
M2 pauli_matrix(uint8_t p) {
    const cd i(0.0, 1.0);
    if (p == 1) return M2{0.0, 1.0, 1.0, 0.0};
    if (p == 2) return M2{0.0, -i, i, 0.0};
    return M2{1.0, 0.0, 0.0, -1.0};
}

// Register layout of a tile: register bit i holds local position reg[i],
// thread-index bit b holds thr[b] (asc: the positions outside the register
// set, ascending).
struct Layout {
    uint32_t R = 0, T = 0;
    uint32_t reg[4] = {0, 0, 0, 0};
    uint32_t thr[16] = {};
    bool asc = true;
    uint32_t set() const {
        uint32_t m = 0;
        for (uint32_t i = 0; i < R; ++i) m |= 1u << reg[i];
        return m;
    }
    int reg_index(uint32_t pos) const {
        for (uint32_t i = 0; i < R; ++i)
            if (reg[i] == pos) return static_cast<int>(i);
        return -1;
    }
    // register word; an explicit layout with 9 thread bits keeps thread bit
    // 8's position in bits 20..23 of it
    uint32_t reg_word() const {
        uint32_t w = 0;
        for (uint32_t i = 0; i < R; ++i) w |= reg[i] << (5 * i);
        if (!asc && T > 8) w |= thr[8] << 20;
        return w;
    }
    uint32_t thr_word() const {
        if (asc) return THR_ASC;
        uint32_t w = 0;
        for (uint32_t b = 0; b < T && b < 8; ++b) w |= thr[b] << (4 * b);
        return w;
    }
};

uint32_t op_mask(const Op &op) { return (1u << op.a) | (op.b == 0xFF ? 0u : 1u << op.b); }

// The ops of one program still to emit, in order: `done` marks emitted
// ones, `head` is the first not emitted.  Scans stop as soon as their answer
// is fixed, so building a program stays close to linear in its ops.
struct Pending {
    std::vector<uint32_t> ops;  // op indices in program order
    std::vector<uint8_t> done;
    size_t head = 0;
    bool empty() const { return head == ops.size(); }
    void advance() {
        while (head < ops.size() && done[head]) ++head;
    }
};

// Next register set: the qubits of the next applicable ops (in order, while
// R qubits suffice), topped up with `fill` positions (lowest first) and then
// any others outside `avoid`.
uint32_t greedy_set(const Plan &plan, const Pending &pd, uint32_t R, uint32_t k, uint32_t fill,
                    uint32_t avoid) {
    const uint32_t all = (1u << k) - 1u;
    uint32_t nw = 0, blocked = 0;
    for (size_t i = pd.head; i < pd.ops.size(); ++i) {
        if (pd.done[i]) continue;
        const uint32_t qm = op_mask(plan.ops[pd.ops[i]]);
        if ((qm & blocked) || (qm & avoid)) blocked |= qm;
        else if (static_cast<uint32_t>(__builtin_popcount(nw | qm)) <= R) nw |= qm;
        else blocked |= qm;
        if (static_cast<uint32_t>(__builtin_popcount(nw)) == R || ((blocked | avoid) & all) == all) break;
    }
    for (uint32_t q = 0; q < k && static_cast<uint32_t>(__builtin_popcount(nw)) < R; ++q)
        if ((fill >> q & 1u) && !(avoid >> q & 1u)) nw |= 1u << q;
    for (uint32_t q = k; q-- > 0 && static_cast<uint32_t>(__builtin_popcount(nw)) < R;)
        if (!(avoid >> q & 1u)) nw |= 1u << q;
    return nw;
}

// Register-blocked programs of one sweep (see Instr): apply every op whose
// qubits are register qubits, in dependency order; when none is left, pick
// the next register set from the qubits of the next applicable ops and move
// there.
//
// For the persistent kernel (general layouts) a program starts and ends in
// layouts of its own choosing whose thread bits 0 .. lowc-1 hold the local
// positions 0 .. lowc-1 (the lowest global qubits, so loads and stores move
// contiguous runs); a move whose new register qubits all sit on lane bits
// (thread bits 0 .. 5) is a sequence of lane exchanges inside the wavefront
// (no LDS), and every LDS re-layout puts the qubits needed last on the wave
// bits (thread bits 6 and up).  Otherwise (other kernels) programs start and end in the
// initial layout (the top R local qubits) and every move is an LDS
// re-layout to an ascending register set.
void build_programs(Plan &plan, Pass &p) {
    const uint32_t k = p.k;
    const uint32_t R = std::min(plan.reg_qubits, k);
    const uint32_t T = k - R;
    uint32_t low = 0;
    while (low < k && p.q[low] == low) ++low;
    // positions kept at the lowest thread bits in load and store layouts
    // (at most 4, and leaving R positions for the registers)
    const uint32_t lowc = std::min<uint32_t>(std::min<uint32_t>(low, 4), T);
    const uint32_t lowmask = (1u << lowc) - 1u;
    const bool general = plan.general_layouts && T <= 9;
    const bool exch_ok = general && T >= 6;

    auto identity2 = [&]() {
        if (plan.identity2 == UINT32_MAX) {
            plan.identity2 = static_cast<uint32_t>(plan.mats.size());
            plan.mat_blocks.emplace_back(plan.identity2, 2u);
            plan.mats.insert(plan.mats.end(), {cd(1.0), cd(0.0), cd(0.0), cd(1.0)});
        }
        return plan.identity2;
    };
    // the op's matrix written for its two qubits in the other order
    auto swapped = [&](uint32_t mat) {
        auto it = plan.swapped.find(mat);
        if (it != plan.swapped.end()) return it->second;
        M4 m;
        for (int i = 0; i < 16; ++i) m[i] = plan.mats[mat + i];
        const M4 w = swap_halves(m);
        const uint32_t off = static_cast<uint32_t>(plan.mats.size());
        plan.mat_blocks.emplace_back(off, 4u);
        plan.mats.insert(plan.mats.end(), w.begin(), w.end());
        plan.swapped.emplace(mat, off);
        return off;
    };
    auto sorted_layout = [&](uint32_t set) {
        Layout L;
        L.R = R;
        L.T = T;
        uint32_t i = 0, b = 0;
        for (uint32_t q = 0; q < k; ++q) {
            if (set >> q & 1u) L.reg[i++] = q;
            else L.thr[b++] = q;
        }
        L.asc = true;
        return L;
    };
    // explicit layout with register set `set`: positions 0 .. lowc-1 stay at
    // their thread bits; the wave bits (thread bits 6 and up, which only an
    // LDS re-layout can reach) take the positions the remaining ops `rem`
    // need last; the other lane bits take the rest in ascending order
    auto make_layout = [&](uint32_t set, const Pending *rem) {
        Layout L = sorted_layout(set);
        L.asc = false;
        bool used[16] = {};
        bool placed[16] = {};
        for (uint32_t q = 0; q < lowc; ++q)
            if (!(set >> q & 1u)) { L.thr[q] = q; used[q] = placed[q] = true; }
        if (T > 6) {
            uint32_t first[16];
            for (uint32_t q = 0; q < k; ++q) first[q] = UINT32_MAX;
            if (rem) {
                const uint32_t want = ((1u << k) - 1u) & ~set;
                uint32_t seen = 0;
                for (size_t i = rem->head; i < rem->ops.size() && (seen & want) != want; ++i) {
                    if (rem->done[i]) continue;
                    const Op &op = plan.ops[rem->ops[i]];
                    if (first[op.a] == UINT32_MAX) first[op.a] = static_cast<uint32_t>(i);
                    if (op.b != 0xFF && first[op.b] == UINT32_MAX) first[op.b] = static_cast<uint32_t>(i);
                    seen |= op_mask(op);
                }
            }
            for (uint32_t b = 6; b < T; ++b) {
                int pick = -1;
                for (uint32_t q = 0; q < k; ++q) {
                    if ((set >> q & 1u) || placed[q]) continue;
                    if (pick < 0 || first[q] >= first[pick]) pick = static_cast<int>(q);
                }
                L.thr[b] = static_cast<uint32_t>(pick);
                used[b] = placed[pick] = true;
            }
        }
        uint32_t b = 0;
        for (uint32_t q = 0; q < k; ++q) {
            if ((set >> q & 1u) || placed[q]) continue;
            while (used[b]) ++b;
            L.thr[b] = q;
            used[b] = placed[q] = true;
        }
        return L;
    };
    // thread bit holding position q (-1: a register)
    auto thread_bit = [&](const Layout &L, uint32_t q) {
        for (uint32_t b = 0; b < T; ++b)
            if (L.thr[b] == q) return static_cast<int>(b);
        return -1;
    };
    auto exchange = [&](Layout &L, uint32_t r, uint32_t h) {
        plan.prog.push_back(Instr{IN_EXCH | ((r | (h << 3)) << 2), 0});
        std::swap(L.reg[r], L.thr[h]);
    };
    auto emit_relayout = [&](const Layout &L) {
        plan.prog.push_back(Instr{IN_RELAYOUT | (L.reg_word() << 2), L.thr_word()});
    };

    for (int pass_dir = 0; pass_dir < 2; ++pass_dir) {
        const bool inverse = pass_dir == 1;
        Pending rem;
        for (uint32_t i = p.op_begin; i < p.op_end; ++i) rem.ops.push_back(i);
        if (inverse) std::reverse(rem.ops.begin(), rem.ops.end());
        rem.done.assign(rem.ops.size(), 0);
        const uint32_t begin = static_cast<uint32_t>(plan.prog.size());
        const uint32_t init_set = ((1u << R) - 1u) << (k - R);
        Layout cur;
        if (general) {
            // start: registers from the first ops that avoid the coalesced positions
            const uint32_t s0 = greedy_set(plan, rem, R, k, init_set, lowmask);
            cur = make_layout(s0, &rem);
        } else {
            cur = sorted_layout(init_set);
        }
        const Layout start = cur;
        while (!rem.empty()) {
            // apply what the registers cover (no later op can once every
            // register qubit is held by an op left behind)
            const uint32_t set = cur.set();
            uint32_t blocked = 0;
            for (size_t i = rem.head; i < rem.ops.size(); ++i) {
                if (rem.done[i]) continue;
                const Op &op = plan.ops[rem.ops[i]];
                const uint32_t qm = op_mask(op);
                if ((qm & blocked) || (qm & set) != qm) {
                    blocked |= qm;
                    if ((blocked & set) == set) break;
                    continue;
                }
                rem.done[i] = 1;
                uint32_t mat = inverse ? op.adj : op.mat;
                const uint32_t A = static_cast<uint32_t>(cur.reg_index(op.a));
                if (op.b == 0xFF) {
                    plan.prog.push_back(Instr{IN_OP1 | (A << 2), mat});
                } else {
                    uint32_t B = static_cast<uint32_t>(cur.reg_index(op.b));
                    uint32_t hi = A, lo = B;
                    if (A < B) { hi = B; lo = A; mat = swapped(mat); }
                    plan.prog.push_back(Instr{IN_OP2 | ((hi | (lo << 3)) << 2), mat});
                }
            }
            rem.advance();
            if (rem.empty()) break;
            // move to the next register set: lane exchanges when every new
            // register qubit sits on a lane bit, else an LDS re-layout
            const uint32_t nw = greedy_set(plan, rem, R, k, set, 0);
            const uint32_t missing = nw & ~set;
            bool by_exchange = exch_ok;
            for (uint32_t q = 0; q < k && by_exchange; ++q)
                if ((missing >> q & 1u) && thread_bit(cur, q) >= 6) by_exchange = false;
            if (by_exchange) {
                for (uint32_t q = 0; q < k; ++q) {
                    if (!(missing >> q & 1u)) continue;
                    uint32_t r = 0;
                    while (nw >> cur.reg[r] & 1u) ++r;  // a register qubit the new set drops
                    exchange(cur, r, static_cast<uint32_t>(thread_bit(cur, q)));
                }
            } else {
                cur = general ? make_layout(nw, &rem) : sorted_layout(nw);
                emit_relayout(cur);
            }
        }
        // end: a layout the store moves coalesced (positions 0 .. lowc-1 on
        // thread bits 0 .. lowc-1), by lane exchanges where they reach
        if (general && exch_ok) {
            for (uint32_t q = 0; q < lowc; ++q) {
                if (cur.thr[q] == q) continue;
                const int b = thread_bit(cur, q);
                if (b >= 6) break;  // on a wave bit: LDS re-layout below
                if (b >= 0) exchange(cur, 0, static_cast<uint32_t>(b));  // into register 0
                exchange(cur, static_cast<uint32_t>(cur.reg_index(q)), q);
            }
        }
        bool ok_end = true;
        if (general) {
            for (uint32_t b = 0; b < lowc; ++b) ok_end = ok_end && cur.thr[b] == b;
        } else {
            ok_end = cur.set() == init_set;
        }
        if (!ok_end) {
            if (general) {
                uint32_t keepset = cur.set() & ~lowmask;
                for (uint32_t q = k; q-- > lowc && static_cast<uint32_t>(__builtin_popcount(keepset)) < R;)
                    keepset |= 1u << q;
                cur = make_layout(keepset, nullptr);
            } else {
                cur = sorted_layout(init_set);
            }
            emit_relayout(cur);
        }
        // even length (the ping-pong kernel runs instructions in pairs):
        // pad with the identity on register bit 0
        if ((plan.prog.size() - begin) & 1u) plan.prog.push_back(Instr{IN_OP1, identity2()});
        const uint32_t end = static_cast<uint32_t>(plan.prog.size());
        uint32_t *lay = p.lay[pass_dir];
        lay[0] = start.reg_word();
        lay[1] = start.thr_word();
        lay[2] = cur.reg_word();
        lay[3] = cur.thr_word();
        if (inverse) { p.inv_begin = begin; p.inv_end = end; }
        else { p.fwd_begin = begin; p.fwd_end = end; }
    }
}

struct BuildOp {
    uint32_t qa, qb;  // global qubits; qb = NONE for 1-qubit ops
    bool live;
    M2 m2;
    M4 m4;
};
constexpr uint32_t NONE = 0xFFFFFFFFu;

struct Fuser {
    const Circuit &c;
    const FusionParams fp;
    Plan &plan;
    bool programs;

    // pool offset of a d x d matrix followed by its adjoint, shared with an
    // earlier op of identical (bitwise) matrix
    uint32_t pool(const cd *m, int d) {
        const size_t nb = sizeof(cd) * d * d;
        // hash of 8 of the 64-bit words, spread over entries and real and
        // imaginary parts (equal matrices are told apart from colliding
        // ones by comparing all the bytes)
        static const uint8_t pick4[8] = {0, 5, 10, 15, 16, 21, 26, 31};
        uint64_t h = 0x9E3779B97F4A7C15ull * static_cast<uint64_t>(d);
        for (size_t i = 0; i < 8; ++i) {
            uint64_t w;
            std::memcpy(&w, reinterpret_cast<const unsigned char *>(m) + 8 * (d == 4 ? pick4[i] : i), 8);
            h = (h ^ w) * 0xff51afd7ed558ccdull;
            h ^= h >> 29;
        }
        auto range = plan.mat_index.equal_range(h);
        for (auto it = range.first; it != range.second; ++it)
            if (it->second.second == d && std::memcmp(plan.mats.data() + it->second.first, m, nb) == 0)
                return it->second.first;
        const uint32_t off = static_cast<uint32_t>(plan.mats.size());
        plan.mat_blocks.emplace_back(off, static_cast<uint32_t>(d));
        plan.mat_blocks.emplace_back(off + static_cast<uint32_t>(d * d), static_cast<uint32_t>(d));
        plan.mats.insert(plan.mats.end(), m, m + d * d);
        for (int r = 0; r < d; ++r)
            for (int cc = 0; cc < d; ++cc) plan.mats.push_back(std::conj(m[cc * d + r]));
        plan.mat_index.emplace(h, std::make_pair(off, d));
        return off;
    }

    struct Item {
        uint32_t qa, qb;  // qubits
        bool two;
        bool is_gate;
        M2 m2;            // 1-qubit matrix (gate or Pauli)
        const cd *m4;     // 2-qubit gate's 16 entries, row-major, basis index
                          // 2 * bit(qa) + bit(qb): the circuit's or CX_MATRIX
    };

    // Tokens one sweep would take from `rest` if its tile started as the
    // qubits of `init` (nq of them): the sweep's admission rule (a token is
    // taken unless one of its qubits is blocked, it would grow the tile past
    // max_qubits or the sweep holds max_ops dense ops; a token not taken
    // blocks its qubits), without building matrices.  Stops early once
    // nothing more can be taken.
    // scratch of fuse and dry_run, reused from call to call
    std::vector<BuildOp> f_ops;
    std::vector<uint32_t> f_keep;
    std::vector<uint8_t> dr_one;
    uint32_t dry_run(const std::vector<Item> &items, const std::vector<uint32_t> &rest,
                     const std::vector<uint8_t> &init, uint32_t nq0) {
        const uint32_t n = c.n;
        // the tile's and the blocked qubits as bit masks (n <= 34)
        uint64_t inm = 0, blm = 0;
        for (uint32_t q = 0; q < n; ++q)
            if (init[q]) inm |= 1ull << q;
        int last[64];
        std::fill(last, last + n, -1);
        std::vector<uint8_t> &one = dr_one;  // per live-or-dead op: 1-qubit?
        one.clear();
        uint32_t nq = nq0, live = 0, taken = 0;
        for (uint32_t idx : rest) {
            const Item &it = items[idx];
            const uint64_t m = (1ull << it.qa) | (it.two ? 1ull << it.qb : 0ull);
            const uint32_t need = nq + static_cast<uint32_t>(__builtin_popcountll(m & ~inm));
            if ((blm & m) || need > fp.max_qubits) {
                blm |= m;
                // a full tile whose qubits are all blocked takes nothing more
                if (nq == fp.max_qubits && static_cast<uint32_t>(__builtin_popcountll(blm & inm)) == nq) break;
                continue;
            }
            inm |= m;
            nq = need;
            ++taken;
            if (!it.two) {
                if (last[it.qa] < 0) {
                    one.push_back(1);
                    last[it.qa] = static_cast<int>(one.size()) - 1;
                    ++live;
                }
            } else {
                const int la = last[it.qa], lb = last[it.qb];
                if (!(la >= 0 && la == lb)) {
                    if (la >= 0 && one[la]) --live;
                    if (lb >= 0 && one[lb]) --live;
                    one.push_back(0);
                    last[it.qa] = last[it.qb] = static_cast<int>(one.size()) - 1;
                    ++live;
                }
            }
            if (live >= fp.max_ops) break;
        }
        return taken;
    }

    // Fuse one segment; appends passes to the plan, returns their range.
    std::pair<uint32_t, uint32_t> fuse(const std::vector<Item> &items) {
        const uint32_t first = static_cast<uint32_t>(plan.passes.size());
        const uint32_t n = c.n;
        std::vector<uint32_t> rest(items.size());
        for (uint32_t i = 0; i < items.size(); ++i) rest[i] = i;
        const bool whole = n <= fp.max_qubits;
        const uint32_t low = std::min(fp.low_qubits, n);
        std::vector<int> last(n, -1);
        std::vector<uint8_t> inq(n, 0), blocked(n, 0), cand(n, 0);
        std::vector<BuildOp> &ops = f_ops;
        std::vector<uint32_t> &keep = f_keep;
        while (!rest.empty()) {
            ops.clear();
            std::fill(last.begin(), last.end(), -1);
            std::fill(inq.begin(), inq.end(), 0);
            std::fill(blocked.begin(), blocked.end(), 0);
            uint32_t nq = 0;
            auto addq = [&](uint32_t q) { if (!inq[q]) { inq[q] = 1; ++nq; } };
            if (whole) {
                for (uint32_t q = 0; q < n; ++q) addq(q);
            } else {
                for (uint32_t q = 0; q < low; ++q) addq(q);
                if (fp.window_search && fp.max_qubits > low) {
                    // the tile the tokens claim in order (the start above), or
                    // the low qubits plus a window of consecutive qubits:
                    // whichever takes the most tokens this sweep
                    const uint32_t w = fp.max_qubits - low;
                    uint32_t best_take = dry_run(items, rest, inq, nq), best_a = 0;
                    bool window = false;
                    for (uint32_t a = low; a + w <= n; ++a) {
                        std::fill(cand.begin(), cand.end(), 0);
                        for (uint32_t q = 0; q < low; ++q) cand[q] = 1;
                        for (uint32_t q = a; q < a + w; ++q) cand[q] = 1;
                        const uint32_t tk = dry_run(items, rest, cand, low + w);
                        if (tk > best_take) {
                            best_take = tk;
                            best_a = a;
                            window = true;
                        }
                    }
                    if (window)
                        for (uint32_t q = best_a; q < best_a + w; ++q) addq(q);
                }
            }
            uint32_t live = 0, gates = 0, paulis = 0;
            keep.clear();
            bool full = false;
            const uint32_t cap = whole ? n : fp.max_qubits;
            uint32_t nblk_in = 0;  // tile qubits blocked so far
            auto block = [&](uint32_t q) {
                if (!blocked[q]) {
                    blocked[q] = 1;
                    if (inq[q]) ++nblk_in;
                }
            };
            for (size_t r = 0; r < rest.size(); ++r) {
                // nothing later can be taken once the sweep holds its op limit
                // or its tile is full with every tile qubit blocked: the rest
                // waits for the next sweep as it is
                if (full || (nq == cap && nblk_in == nq)) {
                    keep.insert(keep.end(), rest.begin() + static_cast<std::ptrdiff_t>(r), rest.end());
                    break;
                }
                const uint32_t idx = rest[r];
                const Item &it = items[idx];
                const bool blk = blocked[it.qa] || (it.two && blocked[it.qb]);
                bool take = false;
                if (!blk) {
                    uint32_t need = nq + (inq[it.qa] ? 0 : 1) + (it.two && !inq[it.qb] ? 1 : 0);
                    if (need <= cap) take = true;
                }
                if (!take) {
                    block(it.qa);
                    if (it.two) block(it.qb);
                    keep.push_back(idx);
                    continue;
                }
                addq(it.qa);
                if (it.two) addq(it.qb);
                if (it.is_gate) ++gates; else ++paulis;
                if (!it.two) {
                    const int l = last[it.qa];
                    if (l >= 0) {
                        BuildOp &o = ops[l];
                        if (o.qb == NONE) o.m2 = mul2(it.m2, o.m2);
                        else if (o.qa == it.qa) o.m4 = mul_hi(it.m2, o.m4);
                        else o.m4 = mul_lo(it.m2, o.m4);
                    } else {
                        ops.push_back(BuildOp{it.qa, NONE, true, it.m2, {}});
                        last[it.qa] = static_cast<int>(ops.size()) - 1;
                        ++live;
                    }
                } else {
                    const int la = last[it.qa], lb = last[it.qb];
                    M4 g;
                    std::copy(it.m4, it.m4 + 16, g.begin());
                    if (la >= 0 && la == lb) {
                        BuildOp &o = ops[la];
                        o.m4 = mul4(o.qa == it.qa ? g : swap_halves(g), o.m4);
                    } else {
                        M2 a = I2m, b = I2m;
                        if (la >= 0 && ops[la].qb == NONE) { a = ops[la].m2; ops[la].live = false; --live; }
                        if (lb >= 0 && ops[lb].qb == NONE) { b = ops[lb].m2; ops[lb].live = false; --live; }
                        ops.push_back(BuildOp{it.qa, it.qb, true, {}, mul_kron(g, a, b)});
                        last[it.qa] = last[it.qb] = static_cast<int>(ops.size()) - 1;
                        ++live;
                    }
                }
                if (!whole && live >= fp.max_ops) full = true;
            }
            rest.swap(keep);
            // fill the tile up with the lowest unused qubits: every sweep
            // then has tiles of the same size and a longer contiguous run
            for (uint32_t q = 0; q < n && nq < (whole ? n : fp.max_qubits); ++q) addq(q);
            // local qubit order: ascending global index
            Pass p;
            p.k = 0;
            int loc[64];
            for (uint32_t q = 0; q < n; ++q)
                if (inq[q]) { loc[q] = static_cast<int>(p.k); p.q[p.k++] = q; }
            p.op_begin = static_cast<uint32_t>(plan.ops.size());
            for (const BuildOp &o : ops) {
                if (!o.live) continue;
                Op op;
                op.a = static_cast<uint8_t>(loc[o.qa]);
                op.b = o.qb == NONE ? 0xFF : static_cast<uint8_t>(loc[o.qb]);
                // 2-qubit ops keep the higher local qubit as the high bit of
                // the 4x4 index (the kernels' canonical order)
                M4 m4 = o.m4;
                if (o.qb != NONE && op.a < op.b) {
                    std::swap(op.a, op.b);
                    m4 = swap_halves(m4);
                }
                const int d = o.qb == NONE ? 2 : 4;
                op.mat = pool(o.qb == NONE ? o.m2.data() : m4.data(), d);
                op.adj = op.mat + static_cast<uint32_t>(d * d);
                plan.ops.push_back(op);
            }
            p.op_end = static_cast<uint32_t>(plan.ops.size());
            p.n_gates = gates;
            p.n_paulis = paulis;
            if (programs) build_programs(plan, p);
            plan.passes.push_back(p);
        }
        return {first, static_cast<uint32_t>(plan.passes.size())};
    }
};

// Fuser items of tokens [a, b) of a leaf (toks from leaf_tokens); counts
// gates, Paulis and the operation count (1 per 1-qubit token, 4 per 2-qubit gate).
void token_items(const Circuit &c, const Ev *ev, const std::vector<Tok> &toks, uint64_t a,
                 uint64_t b, std::vector<Fuser::Item> &items, uint64_t &ng, uint64_t &np,
                 uint64_t &ops) {
    items.clear();
    ng = np = ops = 0;
    for (uint64_t i = a; i < b; ++i) {
        const Tok &tk = toks[i];
        Fuser::Item it{};
        if (tk.is_gate) {
            const Gate &g = c.gates[tk.idx];
            it.is_gate = true;
            it.qa = g.q[0];
            if (is_two_qubit(g.kind)) {
                it.two = true;
                it.qb = g.q[1];
                it.m4 = g.kind == TUSQ_UNITARY2 ? c.umats.data() + g.umat : CX_MATRIX.data();
                ops += 4;
            } else {
                it.two = false;
                it.qb = NONE;
                cd m[4];
                gate_matrix(c, g, m);
                it.m2 = M2{m[0], m[1], m[2], m[3]};
                ops += 1;
            }
            ++ng;
        } else {
            const Ev &e = ev[tk.idx];
            it.is_gate = false;
            it.two = false;
            it.qa = e.qubit;
            it.qb = NONE;
            it.m2 = pauli_matrix(e.pauli);
            ++np;
            ops += 1;
        }
        items.push_back(it);
    }
}

uint64_t pass_flops_per_amp(const Plan &plan, const Pass &p) {
    uint64_t f = 0;
    for (uint32_t i = p.op_begin; i < p.op_end; ++i) f += plan.ops[i].b == 0xFF ? 16 : 32;
    return f;
}

}  // namespace

// Complex64 copies of the matrices.  Rounding each entry to its nearest
// float leaves U^H U = I + E with tr E of the size of the rounding (~1e-7):
// an op scales the squared norm of a spread-out state by about
// 1 + tr(E)/d, with the same sign on every amplitude, and the same fused
// matrices recur many times in a walk, so this adds up to the norm drift
// that triggers complex128 recomputes.  Each matrix is rounded instead so
// that its squared Frobenius norm -- the trace of U^H U -- stays the FP64
// one: entries start at the nearest float, then, one at a time, an entry
// moves to its other float neighbour, always the move that brings sum |f|^2
// closest to the target, while a move improves it.  Every entry stays
// within one float spacing of its FP64 value.
void mats_to_c64(const Plan &p, std::vector<float> &out) {
    out.assign(2 * p.mats.size(), 0.0f);
    for (size_t i = 0; i < p.mats.size(); ++i) {
        out[2 * i] = static_cast<float>(p.mats[i].real());
        out[2 * i + 1] = static_cast<float>(p.mats[i].imag());
    }
    // blocks are independent: large plans split them over host threads
    const size_t nb = p.mat_blocks.size();
    const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    const unsigned nt = nb >= (size_t(1) << 16) ? hw : 1u;
    auto work = [&](size_t b0, size_t b1) {
    for (size_t bi = b0; bi < b1; ++bi) {
        const auto &blk = p.mat_blocks[bi];
        const uint32_t off = blk.first, nc = 2 * blk.second * blk.second;  // real components
        float *f = out.data() + 2 * static_cast<size_t>(off);
        double target = 0.0, sum = 0.0;
        float alt[32];
        bool moved[32] = {};
        for (uint32_t k = 0; k < nc; ++k) {
            const cd &z = p.mats[off + k / 2];
            const double x = (k & 1) ? z.imag() : z.real();
            target += x * x;
            alt[k] = x > f[k] ? std::nextafter(f[k], HUGE_VALF)
                   : x < f[k] ? std::nextafter(f[k], -HUGE_VALF) : f[k];
            sum += double(f[k]) * f[k];
        }
        double err = sum - target;
        for (;;) {
            int best = -1;
            double best_abs = std::fabs(err);
            for (uint32_t k = 0; k < nc; ++k) {
                if (moved[k] || alt[k] == f[k]) continue;
                const double e2 = err - double(f[k]) * f[k] + double(alt[k]) * alt[k];
                if (std::fabs(e2) < best_abs) {
                    best = static_cast<int>(k);
                    best_abs = std::fabs(e2);
                }
            }
            if (best < 0) break;
            err += double(alt[best]) * alt[best] - double(f[best]) * f[best];
            std::swap(f[best], alt[best]);
            moved[best] = true;
        }
    }
    };
    if (nt == 1) {
        work(0, nb);
        return;
    }
    std::vector<std::thread> th;
    for (unsigned t = 0; t < nt; ++t) th.emplace_back(work, nb * t / nt, nb * (t + 1) / nt);
    for (auto &x : th) x.join();
}

FusionParams fusion_defaults(uint32_t n, uint32_t precision, const tusq_opts &o) {
    FusionParams fp;
    // tiles of 2^12 amplitudes (64 KiB complex128, 32 KiB complex64) with the
    // 4 lowest qubits always in the tile (256-byte / 128-byte runs), up to 32
    // dense ops per sweep and the window search for the tile qubits: the
    // fastest shape measured on the 26-qubit brickwork slice
    fp.max_qubits = o.fusion_max_qubits ? o.fusion_max_qubits : 12;
    fp.max_ops = o.fusion_max_ops ? o.fusion_max_ops : 32;
    fp.low_qubits = o.fusion_low_qubits ? o.fusion_low_qubits : 4;
    fp.window_search = o.fusion_search != 1;
    if (fp.max_qubits > KMAX) fp.max_qubits = KMAX;
    if (fp.low_qubits > fp.max_qubits - 2) fp.low_qubits = fp.max_qubits - 2;
    (void)n;
    return fp;
}

Plan build_plan(const Circuit &c, const Tree &t, const tusq_opts &o, bool keep_paths,
                bool programs) {
    if (has_measure(c))
        fail(TUSQ_EUNSUPPORTED, "the circuit has measurement layers: run it with TUSQ_CACHING");
    Plan plan;
    plan.n = c.n;
    // register qubits per thread: 4 (16 amplitudes) unless an 8-amplitude
    // variant is asked for
    plan.reg_qubits = (o.sweep_kernel == 3 || o.sweep_kernel == 5) ? 3 : 4;
    plan.general_layouts = o.sweep_kernel == 0 || o.sweep_kernel == 4 || o.sweep_kernel == 5;
    const uint32_t G = t.G;
    uint64_t lb = o.leaf_begin, le = o.leaf_end;
    if (lb == 0 && le == 0) le = t.leaves();
    if (lb > le || le > t.leaves()) fail(TUSQ_EINVAL, "leaf range out of bounds");
    const FusionParams fp = fusion_defaults(c.n, o.precision, o);
    if (fp.max_qubits < 2 || fp.max_ops < 1) fail(TUSQ_EINVAL, "bad fusion parameters");

    // Pass 1: transitions and cut points.
    struct Comp {
        uint64_t leaf;
        bool reset;
        uint64_t from, len;
        std::vector<uint64_t> cuts;
    };
    std::vector<Comp> comps;
    struct Range {
        size_t comp;
        uint64_t start, end;
    };
    std::vector<Range> stack;
    for (uint64_t l = lb; l < le; ++l) {
        Comp cp{l, true, 0, G + t.nev(l), {}};
        if (l > lb && o.traversal != TUSQ_NAIVE) {
            const uint64_t p = l - 1;
            const uint64_t d = shared_depth(G, t.evs(p), t.nev(p), t.evs(l), t.nev(l));
            const uint64_t lp = G + t.nev(p);
            if (o.traversal == TUSQ_DFTT || o.traversal == TUSQ_CHECKPOINT ||
                o.traversal == TUSQ_CACHING ||
                (lp - d) + (cp.len - d) < cp.len) {
                cp.reset = false;
                cp.from = d;
            }
        }
        if (cp.reset) {
            stack.clear();
        } else {
            while (!stack.empty() && stack.back().start >= cp.from) stack.pop_back();
            if (!stack.empty() && stack.back().end > cp.from) {
                comps[stack.back().comp].cuts.push_back(cp.from);
                stack.back().end = cp.from;
            }
        }
        comps.push_back(cp);
        stack.push_back(Range{comps.size() - 1, cp.from, cp.len});
    }

    // Pass 2: segments, fused sweeps and the step list.
    Fuser fu{c, fp, plan, programs};
    struct Seg {
        uint32_t p0, p1;
        uint64_t start;
        uint64_t gates, paulis, ops;
    };
    std::vector<Seg> applied;
    std::vector<Tok> toks;
    std::vector<Fuser::Item> items;
    auto &ct = plan.counters;
    // checkpoint traversal: the states kept at cut depths of the current
    // path, innermost last, each in a device slot; with a slot limit a full
    // stack drops its bottom (the state farthest from the leaves)
    const bool ckpt = o.traversal == TUSQ_CHECKPOINT;
    const uint64_t slot_limit = o.checkpoint_slots;
    struct Kept {
        uint64_t depth;
        uint64_t slot;
    };
    std::vector<Kept> saved;
    std::vector<uint64_t> free_slots;
    uint64_t next_slot = 0;
    auto release = [&](const Kept &k) { free_slots.push_back(k.slot); };
    if (keep_paths) plan.path_off.push_back(0);
    for (const Comp &cp : comps) {
        if (cp.reset) {
            plan.steps.push_back(Step{ST_RESET, 0});
            ct.resets++;
            applied.clear();
            for (const Kept &k : saved) release(k);
            saved.clear();
        } else if (ckpt) {
            while (!saved.empty() && saved.back().depth > cp.from) {
                release(saved.back());
                saved.pop_back();
            }
            if (cp.from == 0) {
                plan.steps.push_back(Step{ST_RESET, 0});
                ct.resets++;
                applied.clear();
                for (const Kept &k : saved) release(k);
                saved.clear();
            } else if (!saved.empty() && saved.back().depth == cp.from) {
                // the branch depth's state was kept on the way down
                while (!applied.empty() && applied.back().start >= cp.from) applied.pop_back();
                plan.steps.push_back(Step{ST_RESTORE, saved.back().slot});
                ct.checkpoint_restores++;
            } else {
                // dropped for the slot limit: undo as plain DFTT does
                if (!slot_limit) fail(TUSQ_EINVAL, "internal: no checkpoint at a branch depth");
                while (!applied.empty() && applied.back().start >= cp.from) {
                    const Seg &s = applied.back();
                    for (uint32_t p = s.p1; p > s.p0; --p) plan.steps.push_back(Step{ST_INV, p - 1});
                    ct.passes_inv += s.p1 - s.p0;
                    ct.inv_gates += s.gates;
                    ct.inv_paulis += s.paulis;
                    ct.paper_ops += s.ops;
                    applied.pop_back();
                }
            }
        } else {
            while (!applied.empty() && applied.back().start >= cp.from) {
                const Seg &s = applied.back();
                for (uint32_t p = s.p1; p > s.p0; --p) plan.steps.push_back(Step{ST_INV, p - 1});
                ct.passes_inv += s.p1 - s.p0;
                ct.inv_gates += s.gates;
                ct.inv_paulis += s.paulis;
                ct.paper_ops += s.ops;
                applied.pop_back();
            }
        }
        const Ev *ev = t.evs(cp.leaf);
        leaf_tokens(G, ev, t.nev(cp.leaf), toks);
        std::vector<uint64_t> cuts = cp.cuts;
        std::sort(cuts.begin(), cuts.end());
        cuts.erase(std::unique(cuts.begin(), cuts.end()), cuts.end());
        uint64_t a = cp.from;
        for (size_t ci = 0; ci <= cuts.size(); ++ci) {
            const uint64_t b = ci < cuts.size() ? cuts[ci] : cp.len;
            if (b <= a) continue;
            uint64_t ng = 0, np = 0, nops = 0;
            token_items(c, ev, toks, a, b, items, ng, np, nops);
            const auto pr = fu.fuse(items);
            for (uint32_t p = pr.first; p < pr.second; ++p) plan.steps.push_back(Step{ST_FWD, p});
            ct.passes_fwd += pr.second - pr.first;
            ct.fwd_gates += ng;
            ct.fwd_paulis += np;
            ct.paper_ops += nops;
            applied.push_back(Seg{pr.first, pr.second, a, ng, np, nops});
            if (ckpt && b < cp.len) {  // a later leaf branches here
                if (slot_limit && saved.size() == slot_limit) {
                    release(saved.front());
                    saved.erase(saved.begin());
                }
                uint64_t slot;
                if (!free_slots.empty()) {
                    slot = free_slots.back();
                    free_slots.pop_back();
                } else {
                    slot = next_slot++;
                }
                plan.steps.push_back(Step{ST_SAVE, slot});
                saved.push_back(Kept{b, slot});
                ct.checkpoint_saves++;
                plan.checkpoint_slots = next_slot;
            }
            a = b;
        }
        plan.steps.push_back(Step{ST_LEAF, cp.leaf});
        ct.leaves++;
        ct.leaf_sweeps++;
        ct.draws += t.shots[cp.leaf];
        if (keep_paths) {
            for (const Seg &s : applied)
                for (uint32_t p = s.p0; p < s.p1; ++p) plan.path.push_back(p);
            plan.path_off.push_back(plan.path.size());
        }
    }
    if (!comps.empty()) {
        ct.ret_gates = G;
        ct.ret_paulis = t.nev(comps.back().leaf);
    }
    const uint64_t bytes_per_amp = o.precision == TUSQ_C64 ? 8 : 16;
    ct.sweep_bytes = (ct.passes_fwd + ct.passes_inv) * 2ull * (1ull << c.n) * bytes_per_amp;
    // dense-op work: per amplitude, a 2x2 is 2 complex multiply-adds and a
    // 4x4 is 4 (8 real operations each)
    uint64_t per_amp = 0;
    for (const Step &sp : plan.steps) {
        if (sp.kind != ST_FWD && sp.kind != ST_INV) continue;
        per_amp += pass_flops_per_amp(plan, plan.passes[sp.id]);
    }
    ct.sweep_flops = per_amp << c.n;
    return plan;
}

uint64_t plan_pass_flops(const Plan &plan, uint32_t pass) {
    return pass_flops_per_amp(plan, plan.passes[pass]) << plan.n;
}

McmPlan build_mcm_plan(const Circuit &c, const Tree &t, const tusq_opts &o, bool programs) {
    McmPlan mp;
    Plan &plan = mp.plan;
    plan.n = c.n;
    plan.reg_qubits = (o.sweep_kernel == 3 || o.sweep_kernel == 5) ? 3 : 4;
    plan.general_layouts = o.sweep_kernel == 0 || o.sweep_kernel == 4 || o.sweep_kernel == 5;
    const uint32_t G = t.G;
    uint64_t lb = o.leaf_begin, le = o.leaf_end;
    if (lb == 0 && le == 0) le = t.leaves();
    if (lb > le || le > t.leaves()) fail(TUSQ_EINVAL, "leaf range out of bounds");
    for (uint64_t l = lb; l < le; ++l)
        if (t.shots[l] != t.count[l] || t.wnum[l] != t.count[l] || t.wden[l] != t.S)
            fail(TUSQ_EUNSUPPORTED, "measurement layers need a tree built without pruning");
    mp.lb = lb;
    mp.le = le;
    for (uint32_t g = 0; g < G; ++g) {
        const Gate &gt = c.gates[g];
        if (!is_measure(gt.kind)) continue;
        McmLayer ly{};
        ly.gate = g;
        ly.reset = gt.kind == TUSQ_MEASURE_RESET;
        const uint64_t mk = measure_mask(gt);
        for (uint32_t q = 0; q < c.n; ++q)
            if ((mk >> q) & 1) ly.q[ly.m++] = q;
        mp.layers.push_back(ly);
    }
    mp.M = static_cast<uint32_t>(mp.layers.size());
    mp.K = std::min<uint32_t>(o.cache_capacity, mp.M);
    const FusionParams fp = fusion_defaults(c.n, o.precision, o);
    if (fp.max_qubits < 2 || fp.max_ops < 1) fail(TUSQ_EINVAL, "bad fusion parameters");
    const uint32_t S1 = mp.M + 1;

    // 1. the distinct stage token sequences (codes) and each leaf's path ids
    std::vector<Tok> toks;
    std::vector<std::map<std::vector<uint64_t>, uint32_t>> index(S1);
    std::vector<std::vector<uint32_t>> by_stage(S1);
    struct Src {
        uint64_t leaf, a, b;  // a leaf and token range the path was first seen in
    };
    std::vector<Src> src;
    mp.leaf_path.resize((le - lb) * S1);
    for (uint64_t l = lb; l < le; ++l) {
        const Ev *ev = t.evs(l);
        leaf_tokens(G, ev, t.nev(l), toks);
        uint64_t a = 0;
        uint32_t s = 0;
        for (uint64_t i = 0; i <= toks.size(); ++i) {
            const bool end = i == toks.size();
            if (!end && !(toks[i].is_gate && is_measure(c.gates[toks[i].idx].kind))) continue;
            std::vector<uint64_t> code;
            code.reserve(i - a);
            for (uint64_t k = a; k < i; ++k) {
                const Tok &tk = toks[k];
                if (tk.is_gate) {
                    code.push_back((1ull << 63) | tk.idx);
                } else {
                    const Ev &e = ev[tk.idx];
                    code.push_back((uint64_t(e.slot) << 32) | (uint64_t(e.qubit) << 8) | e.pauli);
                }
            }
            auto it = index[s].find(code);
            uint32_t id;
            if (it == index[s].end()) {
                id = static_cast<uint32_t>(mp.paths.size());
                McmPath path;
                path.code = code;
                mp.paths.push_back(std::move(path));
                src.push_back(Src{l, a, i});
                index[s].emplace(std::move(code), id);
                by_stage[s].push_back(id);
            } else {
                id = it->second;
            }
            mp.leaf_path[(l - lb) * S1 + s] = id;
            a = i + 1;
            ++s;
        }
        if (s != S1) fail(TUSQ_EINVAL, "internal: stage count of a leaf");
    }

    // 2. cuts: every depth where another path of the same stage branches off
    //    (in lexicographic order the depths shared with all others are the
    //    running minima of neighbour prefixes, walking out both ways)
    auto lcp = [&](uint32_t x, uint32_t y) {
        const auto &u = mp.paths[x].code, &v = mp.paths[y].code;
        uint64_t d = 0;
        while (d < u.size() && d < v.size() && u[d] == v[d]) ++d;
        return d;
    };
    for (uint32_t s = 0; s < S1; ++s) {
        std::vector<uint32_t> ids;
        for (const auto &kv : index[s]) ids.push_back(kv.second);  // map order = lexicographic
        std::vector<uint64_t> nb(ids.size() > 0 ? ids.size() - 1 : 0);
        for (size_t i = 0; i + 1 < ids.size(); ++i) nb[i] = lcp(ids[i], ids[i + 1]);
        for (size_t i = 0; i < ids.size(); ++i) {
            McmPath &p = mp.paths[ids[i]];
            std::vector<uint64_t> cut{0, p.code.size()};
            uint64_t run = UINT64_MAX;
            for (size_t j = i; j > 0; --j) {
                run = std::min(run, nb[j - 1]);
                cut.push_back(run);
                if (run == 0) break;
            }
            run = UINT64_MAX;
            for (size_t j = i; j + 1 < ids.size(); ++j) {
                run = std::min(run, nb[j]);
                cut.push_back(run);
                if (run == 0) break;
            }
            std::sort(cut.begin(), cut.end());
            cut.erase(std::unique(cut.begin(), cut.end()), cut.end());
            p.cut = std::move(cut);
        }
    }

    // 3. fuse every segment of every path once
    Fuser fu{c, fp, plan, programs};
    std::vector<Fuser::Item> items;
    for (uint32_t id = 0; id < mp.paths.size(); ++id) {
        McmPath &p = mp.paths[id];
        const Src &sr = src[id];
        const Ev *ev = t.evs(sr.leaf);
        leaf_tokens(G, ev, t.nev(sr.leaf), toks);
        for (size_t i = 0; i + 1 < p.cut.size(); ++i) {
            uint64_t ng, np, nops;
            token_items(c, ev, toks, sr.a + p.cut[i], sr.a + p.cut[i + 1], items, ng, np, nops);
            const auto pr = fu.fuse(items);
            p.seg.push_back(McmSeg{pr.first, pr.second, static_cast<uint32_t>(ng),
                                   static_cast<uint32_t>(np), nops});
        }
    }
    plan.checkpoint_slots = mp.K;
    return mp;
}

}  // namespace tusq
