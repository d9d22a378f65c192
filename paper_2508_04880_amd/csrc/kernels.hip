// kernels.hip -- gfx950 kernels of the noisy statevector engine.
//
//  k_sweep     one fused HBM sweep (TUSQ Eq. (1), many gates per pass): the
//              state is cut into tiles of 2^k amplitudes whose local index
//              bits are the sweep's qubits; a workgroup stages one tile in
//              LDS, applies the sweep's dense 1- and 2-qubit ops (in reverse
//              order and conjugate-transposed when undoing a sweep, Sec.
//              III-B), and writes the tile back.  The sweep's qubit set
//              always holds the lowest qubits, so every wavefront moves
//              contiguous runs of amplitudes.
//              This op-list form serves tiles smaller than a register block.
//  k_sweep_pp  the default sweep: the same tiles held in registers (16 or 8
//              amplitudes per thread), a host-compiled program of register
//              ops, in-wave lane exchanges and LDS re-layouts, a persistent
//              grid that prefetches the next tile while one computes.
//  k_sweep_reg, k_sweep_pipe   one tile per workgroup, and LDS double
//              buffering with global_load_lds (selectable variants).
//  k_leaf      acc += w |psi|^2 in FP64 and per-chunk FP64 probability sums
//              (fixed reduction order: results are bitwise reproducible).
//  k_scan      inclusive prefix of the chunk sums and the leaf norm (one
//              workgroup, fixed order).
//  k_sample    inverse-CDF shot sampling: one wavefront per draw, binary
//              search over chunk prefixes, then a wave scan inside the chunk.
//  k_reset, k_to_c64, k_fill   state initialisation and conversion.
//  k_mcm_probs / k_mcm_sum     outcome weights of a measurement layer (FP64,
//              fixed summation order); k_mcm_apply projects onto one outcome,
//              renormalises and resets, one coset of the measured bits per
//              thread (so it may run in place).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdint>

#include "kernels.hpp"
#include "regops.hpp"
#include "rng.hpp"

namespace tusq {

template <typename V>
__global__ void __launch_bounds__(256) k_sweep(V *__restrict__ psi, SweepArgs a,
                                               const DOp *__restrict__ ops,
                                               const V *__restrict__ mats) {
    extern __shared__ unsigned char smem_raw[];
    V *tile = reinterpret_cast<V *>(smem_raw);
    const uint32_t T = 1u << a.k;
    const uint32_t tid = threadIdx.x;
    const QMap qm = qmap(a);
    const uint64_t base = tile_base(blockIdx.x, qm, a.k);
    for (uint32_t l = tid; l < T; l += blockDim.x) tile[l] = psi[base + scatter(l, qm, a.low, a.k)];
    __syncthreads();
    for (uint32_t i = 0; i < a.nops; ++i) {
        const DOp op = ops[a.op_begin + (a.inverse ? a.nops - 1 - i : i)];
        const uint32_t qa = op.ab & 0xFFu, qb = (op.ab >> 8) & 0xFFu;
        const V *m = mats + op.mat;
        if (qb == 0xFFu) {
            V m00 = m[0], m01 = m[1], m10 = m[2], m11 = m[3];
            if (a.inverse) {
                const V t01 = m01;
                m00 = cconj(m00); m11 = cconj(m11);
                m01 = cconj(m10); m10 = cconj(t01);
            }
            const uint32_t bit = 1u << qa;
            for (uint32_t p = tid; p < (T >> 1); p += blockDim.x) {
                const uint32_t i0 = insert0(p, qa), i1 = i0 | bit;
                const V v0 = tile[i0], v1 = tile[i1];
                V r0{0, 0}, r1{0, 0};
                r0 = cfma(cfma(r0, m00, v0), m01, v1);
                r1 = cfma(cfma(r1, m10, v0), m11, v1);
                tile[i0] = r0;
                tile[i1] = r1;
            }
        } else {
            V mm[16];
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    mm[4 * r + c] = a.inverse ? cconj(m[4 * c + r]) : m[4 * r + c];
            const uint32_t lo = qa < qb ? qa : qb, hi = qa < qb ? qb : qa;
            const uint32_t A = 1u << qa, B = 1u << qb;
            for (uint32_t p = tid; p < (T >> 2); p += blockDim.x) {
                const uint32_t i0 = insert0(insert0(p, lo), hi);
                const uint32_t idx[4] = {i0, i0 | B, i0 | A, i0 | A | B};
                V v[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) v[r] = tile[idx[r]];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    V acc{0, 0};
#pragma unroll
                    for (int c = 0; c < 4; ++c) acc = cfma(acc, mm[4 * r + c], v[c]);
                    tile[idx[r]] = acc;
                }
            }
        }
        __syncthreads();
    }
    for (uint32_t l = tid; l < T; l += blockDim.x) psi[base + scatter(l, qm, a.low, a.k)] = tile[l];
}

// Register-blocked sweep, one tile per workgroup (the tile layout, ops and
// re-layouts are in regops.hpp).
template <typename V, int R>
__global__ void __launch_bounds__(256) k_sweep_reg(V *__restrict__ psi, SweepArgs a,
                                                   const Instr2 *__restrict__ prog,
                                                   const V *__restrict__ mats) {
    extern __shared__ unsigned char smem_raw[];
    V *lds = reinterpret_cast<V *>(smem_raw);
    const uint32_t k = a.k;
    const uint32_t tid = threadIdx.x;
    const QMap qm = qmap(a);
    const uint64_t base = tile_base(blockIdx.x, qm, k);
    // initial layout: register qubits are the top R local qubits
    const uint64_t toff = scatter(tid, qm, a.low, k);
    uint64_t roff[R];
#pragma unroll
    for (int i = 0; i < R; ++i) roff[i] = 1ull << qat(qm, k - R + i);
    V v[1 << R];
#pragma unroll
    for (int j = 0; j < (1 << R); ++j) {
        uint64_t o = base | toff;
#pragma unroll
        for (int i = 0; i < R; ++i)
            if (j >> i & 1) o |= roff[i];
        v[j] = psi[o];
    }
    run_program<V, R>(v, lds, tid, k, prog, a.inverse ? a.inv_begin : a.fwd_begin,
                      a.inverse ? a.inv_end : a.fwd_end, mats, false);
#pragma unroll
    for (int j = 0; j < (1 << R); ++j) {
        uint64_t o = base | toff;
#pragma unroll
        for (int i = 0; i < R; ++i)
            if (j >> i & 1) o |= roff[i];
        psi[o] = v[j];
    }
}

// ---------------------------------------------------------------------------
// Persistent ping-pong sweep.  Same programs and tile layout as k_sweep_reg,
// with three changes that take per-instruction overhead off the vector ALU
// and overlap HBM traffic with FP64 work:
//  * two register arrays alternate as source and destination: every
//    instruction writes its results straight into the other array, so the
//    interpreter loop carries no register copies (programs have even length,
//    padded with a copy instruction);
//  * relayout addresses are one XOR per element: the swizzle is linear, so the
//    thread part of an LDS address is the XOR of one wave-uniform column per
//    set thread-index bit, and the register parts are wave-uniform;
//  * each workgroup walks tiles blockIdx.x, +gridDim.x, ... and loads the
//    next tile into a third register array while the current one computes.

// workgroups of up to 2^PP_TBITS threads
constexpr int PP_TBITS = 9;

// thread word of a layout whose thread-index bits take the positions outside
// the register set in ascending order (an explicit layout with 9 thread bits
// keeps thread bit 8's position in bits 20..23 of the register word)
constexpr uint32_t PP_THR_ASC = 0xFFFFFFFFu;

// LDS byte offset of this thread's part of a layout: the XOR over set
// thread-index bits b of the swizzled column of the local position that bit
// b holds (explicit thread word: 4 bits per thread bit; ascending: the
// positions outside the register set, walked with a wave-uniform counter).
template <typename V, int R>
__device__ __forceinline__ uint32_t lds_thread_part(uint32_t tid, uint32_t k, uint32_t reg,
                                                    uint32_t thr) {
    uint32_t pd = 0;
    if (thr != PP_THR_ASC) {
#pragma unroll
        for (uint32_t b = 0; b < static_cast<uint32_t>(PP_TBITS); ++b) {
            if (b + R < k) {
                const uint32_t p = b < 8 ? (thr >> (4 * b)) & 15u : (reg >> 20) & 15u;
                pd ^= (0u - ((tid >> b) & 1u)) &
                      (Swz<V>::phys(1u << p) * static_cast<uint32_t>(sizeof(V)));
            }
        }
    } else {
        uint32_t set = 0;
#pragma unroll
        for (int i = 0; i < R; ++i) set |= 1u << ((reg >> (5 * i)) & 31u);
        uint32_t b = 0;
#pragma unroll
        for (uint32_t p = 0; p < 16; ++p) {
            if (p < k && !((set >> p) & 1u)) {
                pd ^= (0u - ((tid >> b) & 1u)) &
                      (Swz<V>::phys(1u << p) * static_cast<uint32_t>(sizeof(V)));
                ++b;
            }
        }
    }
    return pd;
}

// Global element offset of this thread's part of a layout (the thread-index
// bits placed at the tile qubits their local positions name).
template <int R>
__device__ __forceinline__ uint64_t layout_thread_offset(uint32_t tid, const QMap &qm, uint32_t k,
                                                         uint32_t reg, uint32_t thr) {
    uint64_t off = 0;
    if (thr != PP_THR_ASC) {
#pragma unroll
        for (uint32_t b = 0; b < static_cast<uint32_t>(PP_TBITS); ++b)
            if (b + R < k)
                off |= static_cast<uint64_t>((tid >> b) & 1u)
                       << qat(qm, b < 8 ? (thr >> (4 * b)) & 15u : (reg >> 20) & 15u);
    } else {
        uint32_t set = 0;
#pragma unroll
        for (int i = 0; i < R; ++i) set |= 1u << ((reg >> (5 * i)) & 31u);
        uint32_t b = 0;
#pragma unroll
        for (uint32_t p = 0; p < 16; ++p) {
            if (p < k && !((set >> p) & 1u)) {
                off |= static_cast<uint64_t>((tid >> b) & 1u) << qm.q[p];
                ++b;
            }
        }
    }
    return off;
}

// the register qubits of a layout as global qubit indices, one byte each
template <int R>
__device__ __forceinline__ uint32_t layout_reg_qubits(const QMap &qm, uint32_t reg) {
    uint32_t rq = 0;
#pragma unroll
    for (int i = 0; i < R; ++i) rq |= qat(qm, (reg >> (5 * i)) & 31u) << (8 * i);
    return rq;
}

// LDS byte offsets of the register parts of a layout (wave-uniform).
template <typename V, int R>
__device__ __forceinline__ void lds_reg_part(uint32_t packed, uint32_t (&pr)[1 << R]) {
    uint32_t bit[R];
#pragma unroll
    for (int i = 0; i < R; ++i) bit[i] = 1u << ((packed >> (5 * i)) & 31u);
#pragma unroll
    for (int j = 0; j < (1 << R); ++j) {
        uint32_t l = 0;
#pragma unroll
        for (int i = 0; i < R; ++i)
            if (j >> i & 1) l |= bit[i];
        pr[j] = Swz<V>::phys(l) * static_cast<uint32_t>(sizeof(V));
    }
}

template <typename V, int R, int B>
__device__ __forceinline__ void pp_op1(const V (&x)[1 << R], V (&y)[1 << R],
                                       const V *__restrict__ m) {
    const V m0 = m[0], m1 = m[1], m2 = m[2], m3 = m[3];
#pragma unroll
    for (int j = 0; j < (1 << R); ++j) {
        if (j & (1 << B)) continue;
        y[j] = cfma(cmul(m0, x[j]), m1, x[j | (1 << B)]);
        y[j | (1 << B)] = cfma(cmul(m2, x[j]), m3, x[j | (1 << B)]);
    }
}

// 4x4 matrix with row/column index 2 * bit(A) + bit(B); programs give A > B
template <typename V, int R, int A, int B>
__device__ __forceinline__ void pp_op2(const V (&x)[1 << R], V (&y)[1 << R],
                                       const V *__restrict__ m) {
#pragma unroll
    for (int j = 0; j < (1 << R); ++j) {
        if (j & ((1 << A) | (1 << B))) continue;
        const int i[4] = {j, j | (1 << B), j | (1 << A), j | (1 << A) | (1 << B)};
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            V acc = cmul(m[4 * r], x[i[0]]);
#pragma unroll
            for (int c = 1; c < 4; ++c) acc = cfma(acc, m[4 * r + c], x[i[c]]);
            y[i[r]] = acc;
        }
    }
}

// Swap register bit B with lane bit H: for each pair a = x[j], b = x[j | 1 << B]
// the lanes with bit H set take a's place in b and the others b's place in
// a, i.e. element (lane L, bit B = c) moves to (lane L with bit H = c, bit
// B = bit H of L).  Lane bits 4 and 5 use the row / half swaps
// (permlane16/32_swap); lane bits 2 and 3 a rotation inside the 16-lane row
// written under a bank mask; lane bits 0 and 1 fetch the partner lane with
// a quad permutation and select by the lane's bit.
template <int H>
__device__ __forceinline__ void lane_exchange(uint32_t a, uint32_t b, uint32_t &na, uint32_t &nb) {
    if constexpr (H == 5) {
        const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
        na = r[0];
        nb = r[1];
    } else if constexpr (H == 4) {
        const auto r = __builtin_amdgcn_permlane16_swap(a, b, false, false);
        na = r[0];
        nb = r[1];
    } else if constexpr (H >= 2) {
        // lane bits 2 and 3 are the bank bits of a 16-lane row: the DPP bank
        // mask writes only the lanes with bit H set (or clear), the others
        // keep the old value -- one row rotation per output word (by 4 / 12
        // for bit 2, by 8 for bit 3)
        constexpr int up = H == 2 ? 0x124 : 0x128;
        constexpr int dn = H == 2 ? 0x12C : 0x128;
        constexpr int hi_banks = H == 2 ? 0xA : 0xC;
        constexpr int lo_banks = H == 2 ? 0x5 : 0x3;
        na = static_cast<uint32_t>(__builtin_amdgcn_update_dpp(static_cast<int>(a), static_cast<int>(b), up,
                                                               0xF, hi_banks, false));
        nb = static_cast<uint32_t>(__builtin_amdgcn_update_dpp(static_cast<int>(b), static_cast<int>(a), dn,
                                                               0xF, lo_banks, false));
    } else {
        // partner of lane L is L ^ (1 << H): quad_perm [1,0,3,2] / [2,3,0,1]
        constexpr int up = H == 0 ? 0xB1 : 0x4E;
        constexpr int dn = up;
        const bool hi = (__lane_id() >> H) & 1u;
        const uint32_t fb = static_cast<uint32_t>(
            __builtin_amdgcn_mov_dpp(static_cast<int>(b), up, 0xF, 0xF, false));
        const uint32_t fa = static_cast<uint32_t>(
            __builtin_amdgcn_mov_dpp(static_cast<int>(a), dn, 0xF, 0xF, false));
        na = hi ? fb : a;
        nb = hi ? b : fa;
    }
}

template <typename V, int R, int B, int H>
__device__ __forceinline__ void pp_exch(const V (&x)[1 << R], V (&y)[1 << R]) {
    constexpr int W = sizeof(V) / 4;
    struct Words {
        uint32_t w[W];
    };
#pragma unroll
    for (int j = 0; j < (1 << R); ++j) {
        if (j & (1 << B)) continue;
        const Words a = __builtin_bit_cast(Words, x[j]);
        const Words b = __builtin_bit_cast(Words, x[j | (1 << B)]);
        Words na, nb;
#pragma unroll
        for (int i = 0; i < W; ++i) lane_exchange<H>(a.w[i], b.w[i], na.w[i], nb.w[i]);
        y[j] = __builtin_bit_cast(V, na);
        y[j | (1 << B)] = __builtin_bit_cast(V, nb);
    }
}

template <typename V, int R>
__device__ __forceinline__ void pp_copy(const V (&x)[1 << R], V (&y)[1 << R]) {
#pragma unroll
    for (int j = 0; j < (1 << R); ++j) y[j] = x[j];
}

// One program instruction from x into y.  (reg, thr) is the current layout,
// `dirty` whether another wave may still read the LDS scratch.  Programs
// hold valid instructions only (relayout, 1-qubit op on a register bit,
// 2-qubit op on register bits a > b, lane exchange); there is no copy case,
// whose moves the compiler would hoist in front of the dispatch.
template <typename V, int R>
__device__ __forceinline__ void pp_step(const V (&x)[1 << R], V (&y)[1 << R], Instr2 ins,
                                        const V *__restrict__ mats, unsigned char *lds,
                                        uint32_t tid, uint32_t k, uint32_t &reg, uint32_t &thr,
                                        bool &dirty) {
    const uint32_t type = ins.w0 & 3u, arg = ins.w0 >> 2;
    if (type == 0u) {  // relayout into (arg, ins.mat)
        uint32_t pr[1 << R];
        if (dirty) lds_barrier();
        uint32_t pd = lds_thread_part<V, R>(tid, k, reg, thr);
        lds_reg_part<V, R>(reg, pr);
#pragma unroll
        for (int j = 0; j < (1 << R); ++j) *reinterpret_cast<V *>(lds + (pd ^ pr[j])) = x[j];
        lds_barrier();
        pd = lds_thread_part<V, R>(tid, k, arg, ins.mat);
        lds_reg_part<V, R>(arg, pr);
#pragma unroll
        for (int j = 0; j < (1 << R); ++j) y[j] = *reinterpret_cast<const V *>(lds + (pd ^ pr[j]));
        dirty = true;
        reg = arg;
        thr = ins.mat;
    } else if (type == 1u) {
        const V *m = mats + ins.mat;
        switch (arg & 7u) {
        case 0: pp_op1<V, R, 0>(x, y, m); break;
        case 1: pp_op1<V, R, 1>(x, y, m); break;
        case 2: pp_op1<V, R, 2>(x, y, m); break;
        case 3: if constexpr (R > 3) { pp_op1<V, R, 3>(x, y, m); break; } [[fallthrough]];
        default: __builtin_unreachable();
        }
    } else if (type == 2u) {
        const V *m = mats + ins.mat;
        switch (arg & 63u) {
        case 1 | (0 << 3): pp_op2<V, R, 1, 0>(x, y, m); break;
        case 2 | (0 << 3): pp_op2<V, R, 2, 0>(x, y, m); break;
        case 2 | (1 << 3): pp_op2<V, R, 2, 1>(x, y, m); break;
        case 3 | (0 << 3): if constexpr (R > 3) { pp_op2<V, R, 3, 0>(x, y, m); break; } [[fallthrough]];
        case 3 | (1 << 3): if constexpr (R > 3) { pp_op2<V, R, 3, 1>(x, y, m); break; } [[fallthrough]];
        case 3 | (2 << 3): if constexpr (R > 3) { pp_op2<V, R, 3, 2>(x, y, m); break; } [[fallthrough]];
        default: __builtin_unreachable();
        }
    } else {  // lane exchange of register bit r with thread (lane) bit h
        const uint32_t r = arg & 7u, h = (arg >> 3) & 7u;
        switch (r | (h << 3)) {
#define TUSQ_EXCH_CASE(B, H) \
    case (B) | ((H) << 3): if constexpr ((B) < R) { pp_exch<V, R, B, H>(x, y); break; } [[fallthrough]];
#define TUSQ_EXCH_ROW(H) TUSQ_EXCH_CASE(0, H) TUSQ_EXCH_CASE(1, H) TUSQ_EXCH_CASE(2, H) TUSQ_EXCH_CASE(3, H)
            TUSQ_EXCH_ROW(0) TUSQ_EXCH_ROW(1) TUSQ_EXCH_ROW(2)
            TUSQ_EXCH_ROW(3) TUSQ_EXCH_ROW(4) TUSQ_EXCH_ROW(5)
#undef TUSQ_EXCH_ROW
#undef TUSQ_EXCH_CASE
        default: __builtin_unreachable();
        }
        const uint32_t ts = 4u * h, rs = 5u * r;
        const uint32_t rp = (reg >> rs) & 31u, tp = (thr >> ts) & 15u;
        reg = (reg & ~(31u << rs)) | (tp << rs);
        thr = (thr & ~(15u << ts)) | (rp << ts);
    }
}

template <typename V, int R>
__global__ void __launch_bounds__(1 << PP_TBITS) k_sweep_pp(V *__restrict__ psi, SweepArgs a,
                                                            const Instr2 *__restrict__ prog,
                                                            const V *__restrict__ mats,
                                                            uint32_t ntiles) {
    extern __shared__ unsigned char smem_raw[];
    const uint32_t k = a.k;
    const uint32_t tid = threadIdx.x;
    const uint32_t ib = a.inverse ? a.inv_begin : a.fwd_begin;
    const uint32_t ie = a.inverse ? a.inv_end : a.fwd_end;
    uint32_t t = blockIdx.x;
    if (t >= ntiles) return;

    // Addresses.  In the program's start layout the thread's amplitudes sit
    // at pin[base | roff_j] (pin folds in the thread-index bits, roff_j the
    // register bits: register bit i is global qubit byte i of rin), in its end
    // layout at pout[base | roff'_j] (rout).  base spreads the tile index over
    // the qubits outside the tile (mask `out`); walking tiles t, t + G, ...
    // advances it by a masked add: with the gaps filled with ones, carries
    // skip the tile qubits.
    uint64_t base, dG, out;
    uint32_t rin, rout;
    V *pin, *pout;
    {
        const QMap qm = qmap(a);
        pin = psi + layout_thread_offset<R>(tid, qm, k, a.lay_in_reg, a.lay_in_thr);
        pout = psi + layout_thread_offset<R>(tid, qm, k, a.lay_out_reg, a.lay_out_thr);
        rin = layout_reg_qubits<R>(qm, a.lay_in_reg);
        rout = layout_reg_qubits<R>(qm, a.lay_out_reg);
        uint64_t in = 0;
#pragma unroll
        for (int j = 0; j < 16; ++j)
            if (static_cast<uint32_t>(j) < k) in |= 1ull << qm.q[j];
        out = ~in;
        base = tile_base(t, qm, k);
        dG = tile_base(gridDim.x, qm, k);
    }
    // register offsets are rebuilt from rin / rout where used (the empty asm
    // keeps the compiler from hoisting all 2^R of them into scalar registers
    // that would stay live across the program loop)
    auto off = [&](uint32_t q, int j) {
        uint64_t o = 0;
#pragma unroll
        for (int i = 0; i < R; ++i)
            if (j >> i & 1) o |= 1ull << ((q >> (8 * i)) & 63u);
        return o;
    };
    V x[1 << R], y[1 << R], nx[1 << R];
    {
        uint32_t q = rin;
        asm volatile("" : "+s"(q));
#pragma unroll
        for (int j = 0; j < (1 << R); ++j) x[j] = pin[base | off(q, j)];
    }
    bool dirty = false;
    for (;;) {
        // this tile's amplitudes have landed before the next tile's loads are
        // issued: the program loop then waits on no vector-memory counter
        // (a wait there would also wait for the prefetch)
#pragma unroll
        for (int j = 0; j < (1 << R); ++j) asm volatile("" : "+v"(x[j].x), "+v"(x[j].y));
        const uint32_t tn = t + gridDim.x;
        if (tn < ntiles) {  // in flight while this tile computes
            const uint64_t nbase = ((base | ~out) + dG) & out;
            uint32_t q = rin;
            asm volatile("" : "+s"(q));
#pragma unroll
            for (int j = 0; j < (1 << R); ++j) nx[j] = pin[nbase | off(q, j)];
        }
        uint32_t reg = a.lay_in_reg, thr = a.lay_in_thr;
        for (uint32_t pc = ib; pc < ie; pc += 2) {
            const Instr2 i0 = prog[pc], i1 = prog[pc + 1];
            pp_step<V, R>(x, y, i0, mats, smem_raw, tid, k, reg, thr, dirty);
            pp_step<V, R>(y, x, i1, mats, smem_raw, tid, k, reg, thr, dirty);
        }
        {
            uint32_t q = rout;
            asm volatile("" : "+s"(q));
#pragma unroll
            for (int j = 0; j < (1 << R); ++j) pout[base | off(q, j)] = x[j];
        }
        if (tn >= ntiles) break;
        pp_copy<V, R>(nx, x);
        t = tn;
        base = ((base | ~out) + dG) & out;
    }
}

constexpr uint32_t PIPE_TILE_BYTES = 64 * 1024;

// Pipelined register-blocked sweep.  A persistent grid; each workgroup owns
// two tile buffers in LDS and walks tiles blockIdx.x, +gridDim.x, ...  The
// next tile streams from HBM straight into the idle buffer
// (global_load_lds_dwordx4) while the current one is computed in registers,
// so memory and FP64 work overlap inside one workgroup.
template <typename V, int R>
__global__ void __launch_bounds__(256) k_sweep_pipe(V *__restrict__ psi, SweepArgs a,
                                                    const Instr2 *__restrict__ prog,
                                                    const V *__restrict__ mats, uint32_t ntiles) {
    constexpr uint32_t E = 16 / sizeof(V);  // amplitudes per 16-byte lane transfer
    constexpr uint32_t NJ = (1u << R) / E;  // transfers per thread per tile
    // two statically placed tile buffers (64 KiB each), so that every LDS
    // access in an even or odd step names its buffer directly
    __shared__ V bufA[PIPE_TILE_BYTES / sizeof(V)];
    __shared__ V bufB[PIPE_TILE_BYTES / sizeof(V)];
    const uint32_t k = a.k, T = 1u << k, NT = T >> R;
    const uint32_t tid = threadIdx.x;
    const QMap qm = qmap(a);
    auto scat = [&](uint32_t l) { return scatter(l, qm, a.low, k); };
    auto base_of = [&](uint32_t t) { return tile_base(t, qm, k); };
    // register layout: thread tid holds local tid + j * NT
    const uint64_t toff = scat(tid);
    uint64_t roff[R];
#pragma unroll
    for (int i = 0; i < R; ++i) roff[i] = 1ull << qat(qm, k - R + i);
    // transfer layout: lane element m = (jj * NT + tid) * E, natural LDS order
    const uint64_t moff = scat(tid * E);
    uint64_t joff[NJ];
#pragma unroll
    for (uint32_t jj = 0; jj < NJ; ++jj) joff[jj] = scat(jj * NT * E);
    auto issue = [&](uint32_t t, V *buf) {
        const uint64_t base = base_of(t) | moff;
#pragma unroll
        for (uint32_t jj = 0; jj < NJ; ++jj) {
            const V *src = psi + (base | joff[jj]);
            V *dst = buf + (jj * NT + (tid & ~63u)) * E;
            __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)src,
                                             (__attribute__((address_space(3))) void *)dst, 16, 0, 0);
        }
    };
    const uint32_t ib = a.inverse ? a.inv_begin : a.fwd_begin;
    const uint32_t ie = a.inverse ? a.inv_end : a.fwd_end;
    uint32_t t = blockIdx.x;
    if (t >= ntiles) return;
    issue(t, bufA);
    auto step = [&](V *cur, V *nxt) {
        __builtin_amdgcn_s_waitcnt(0);  // this wave's transfers (and stores) are done
        __syncthreads();                // ... and every other wave's
        V v[1 << R];
#pragma unroll
        for (int j = 0; j < (1 << R); ++j) v[j] = cur[tid + j * NT];
        const uint32_t tn = t + gridDim.x;
        if (tn < ntiles) issue(tn, nxt);  // streams in while this tile computes
        run_program<V, R>(v, cur, tid, k, prog, ib, ie, mats, true);
        const uint64_t base = base_of(t) | toff;
#pragma unroll
        for (int j = 0; j < (1 << R); ++j) {
            uint64_t o = base;
#pragma unroll
            for (int i = 0; i < R; ++i)
                if (j >> i & 1) o |= roff[i];
            psi[o] = v[j];
        }
        t = tn;
    };
    for (;;) {
        step(bufA, bufB);
        if (t >= ntiles) break;
        step(bufB, bufA);
        if (t >= ntiles) break;
    }
}

// ---------------------------------------------------------------------------
// Leaf accumulation: 256 threads per chunk of C = 2^log_chunk amplitudes.
// Thread t sums elements t, t + 256, ... in order; the block combines the
// 256 partial sums by a fixed binary tree.
template <typename V>
__global__ void __launch_bounds__(256) k_leaf(const V *__restrict__ psi, uint32_t log_chunk,
                                              double *__restrict__ acc, double w,
                                              double *__restrict__ chunk_sum) {
    __shared__ double red[256];
    const uint64_t C = 1ull << log_chunk;
    const uint64_t base = static_cast<uint64_t>(blockIdx.x) * C;
    double s = 0.0;
    for (uint64_t i = threadIdx.x; i < C; i += blockDim.x) {
        const V v = psi[base + i];
        const double re = static_cast<double>(v.x), im = static_cast<double>(v.y);
        const double pr = re * re + im * im;
        s += pr;
        if (acc) acc[base + i] += w * pr;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (uint32_t h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) chunk_sum[blockIdx.x] = red[0];
}

// Inclusive prefix over nc chunk sums; thread t owns a contiguous run.
__global__ void __launch_bounds__(1024) k_scan(const double *__restrict__ chunk_sum, uint64_t nc,
                                               double *__restrict__ prefix,
                                               double *__restrict__ norm_out) {
    __shared__ double part[1024];
    const uint64_t per = (nc + blockDim.x - 1) / blockDim.x;
    const uint64_t lo = threadIdx.x * per;
    const uint64_t hi = lo + per < nc ? lo + per : nc;
    double s = 0.0;
    for (uint64_t i = lo; i < hi; ++i) s += chunk_sum[i];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = 0.0;
        for (uint32_t t = 0; t < blockDim.x; ++t) {
            const double v = part[t];
            part[t] = r;
            r += v;
        }
        *norm_out = r;
    }
    __syncthreads();
    double r = part[threadIdx.x];
    for (uint64_t i = lo; i < hi; ++i) {
        r += chunk_sum[i];
        prefix[i] = r;
    }
}

template <typename V>
__device__ __forceinline__ double prob(const V *psi, uint64_t i) {
    const V v = psi[i];
    const double re = static_cast<double>(v.x), im = static_cast<double>(v.y);
    return re * re + im * im;
}

// One wavefront per draw.  Draw d of leaf `leaf`: Philox stream 2, counter
// (d >> 1, leaf, 0), half d & 1; u = (v >> 11) 2^-53; target x = u * norm.
// Result: the first index whose running probability sum exceeds x.
template <typename V>
__global__ void __launch_bounds__(256) k_sample(const V *__restrict__ psi, uint32_t log_chunk,
                                                const double *__restrict__ prefix, uint64_t nc,
                                                const double *__restrict__ norm, uint64_t seed,
                                                uint32_t leaf, uint64_t shots, uint64_t base,
                                                uint64_t *__restrict__ out) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t d = static_cast<uint64_t>(blockIdx.x) * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (d >= shots) return;
    const uint64_t dd = base + d;  // draw index within the leaf
    const Pair64 r = philox_pair(seed, static_cast<uint32_t>(dd >> 1), leaf, 0, STREAM_SHOTS);
    const uint64_t v = (dd & 1) ? r.hi : r.lo;
    const double x = static_cast<double>(v >> 11) * 0x1p-53 * (*norm);
    // first chunk whose inclusive prefix exceeds x
    uint64_t lo = 0, hi = nc;
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (prefix[mid] > x) hi = mid; else lo = mid + 1;
    }
    const uint64_t c = lo < nc ? lo : nc - 1;
    double run = c ? prefix[c - 1] : 0.0;
    const uint64_t C = 1ull << log_chunk;
    const uint64_t per = C >= 64 ? C / 64 : 1;
    const uint64_t b0 = c * C + (C >= 64 ? lane * per : lane);
    const bool active = C >= 64 || lane < C;
    double s = 0.0;
    if (active)
        for (uint64_t i = 0; i < per; ++i) s += prob(psi, b0 + i);
    // inclusive wave scan of lane sums, fixed order
    double incl = s;
    for (uint32_t off = 1; off < 64; off <<= 1) {
        const double t = __shfl_up(incl, off, 64);
        if (lane >= off) incl += t;
    }
    const double before = run + incl - s;
    const bool hit = active && (run + incl > x);
    const unsigned long long mask = __ballot(hit);
    uint64_t result;
    if (mask) {
        const uint32_t first = __ffsll(mask) - 1;
        uint64_t idx = 0;
        if (lane == first) {
            double acc = before;
            idx = b0 + per - 1;
            for (uint64_t i = 0; i < per; ++i) {
                acc += prob(psi, b0 + i);
                if (acc > x) { idx = b0 + i; break; }
            }
        }
        result = __shfl(idx, first, 64);
    } else {
        // rounding left no running sum above x: take the last index of the
        // chunk with non-zero probability
        uint64_t last = 0;
        bool any = false;
        if (active)
            for (uint64_t i = 0; i < per; ++i)
                if (prob(psi, b0 + i) > 0.0) { last = b0 + i; any = true; }
        const unsigned long long m2 = __ballot(any);
        const uint32_t src = m2 ? 63 - __clzll(m2) : 0;
        result = m2 ? __shfl(last, src, 64) : c * C;
    }
    if (lane == 0) out[d] = result;
}

template <typename V>
__global__ void k_reset(V *psi, uint64_t N) {
    const uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < N) psi[i] = V{static_cast<typename RealOf<V>::T>(i == 0 ? 1 : 0), 0};
}

__global__ void k_to_c64(const double2 *src, float2 *dst, uint64_t N) {
    const uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < N) dst[i] = float2{static_cast<float>(src[i].x), static_cast<float>(src[i].y)};
}

__global__ void k_fill(double *p, uint64_t n, double v) {
    const uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------
// Launchers (host side).  Every launcher checks its shapes before launching.
#define TUSQ_CHECK_LAUNCH()                                  \
    do {                                                     \
        hipError_t e_ = hipGetLastError();                   \
        if (e_ != hipSuccess) return e_;                     \
    } while (0)

static unsigned grid1(uint64_t n, unsigned b) { return static_cast<unsigned>((n + b - 1) / b); }

template <typename V>
hipError_t launch_sweep(V *psi, uint32_t n, const SweepArgs &a, const DOp *ops, const V *mats,
                        hipStream_t s) {
    if (a.k > n || a.k > 16 || a.k < 1 || n - a.k > 31 || a.low > a.k) return hipErrorInvalidValue;
    const size_t lds = sizeof(V) << a.k;
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    const unsigned blocks = 1u << (n - a.k);
    hipLaunchKernelGGL(k_sweep<V>, dim3(blocks), dim3(256), lds, s, psi, a, ops, mats);
    TUSQ_CHECK_LAUNCH();
    return hipSuccess;
}

template <typename V, uint32_t R>
static hipError_t launch_reg_r(V *psi, uint32_t n, const SweepArgs &a, const Instr2 *prog,
                               const V *mats, hipStream_t s) {
    if (a.k > n || a.k > 16 || a.k < R || n - a.k > 31 || a.low > a.k) return hipErrorInvalidValue;
    if (a.k - R > 8) return hipErrorInvalidValue;  // at most 256 threads
    const size_t lds = sizeof(V) << a.k;
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    const unsigned blocks = 1u << (n - a.k);
    const unsigned threads = 1u << (a.k - R);
    hipLaunchKernelGGL((k_sweep_reg<V, R>), dim3(blocks), dim3(threads), lds, s, psi, a, prog, mats);
    TUSQ_CHECK_LAUNCH();
    return hipSuccess;
}

template <typename V>
hipError_t launch_sweep_reg(V *psi, uint32_t n, const SweepArgs &a, const Instr2 *prog,
                            const V *mats, uint32_t reg_qubits, hipStream_t s) {
    if (reg_qubits == 3) return launch_reg_r<V, 3>(psi, n, a, prog, mats, s);
    if (reg_qubits == 4) return launch_reg_r<V, 4>(psi, n, a, prog, mats, s);
    return hipErrorInvalidValue;
}

template <typename V, uint32_t R>
static hipError_t launch_pp_r(V *psi, uint32_t n, const SweepArgs &a, const Instr2 *prog,
                              const V *mats, uint32_t cus, hipStream_t s) {
    if (a.k > n || a.k > 16 || a.k < R || n - a.k > 31 || a.low > a.k) return hipErrorInvalidValue;
    if (a.k - R > static_cast<uint32_t>(PP_TBITS)) return hipErrorInvalidValue;  // at most 512 threads
    if (a.inverse ? (a.inv_end - a.inv_begin) & 1u : (a.fwd_end - a.fwd_begin) & 1u)
        return hipErrorInvalidValue;  // programs come in pairs of instructions
    const size_t lds = sizeof(V) << a.k;
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    const unsigned threads = 1u << (a.k - R);
    const uint32_t ntiles = 1u << (n - a.k);
    // resident workgroups per CU for this tile size (cached per kernel and k)
    static std::atomic<int> occ_cache[17];
    int occ = occ_cache[a.k].load(std::memory_order_relaxed);
    if (occ == 0) {
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &occ, reinterpret_cast<const void *>(k_sweep_pp<V, R>), static_cast<int>(threads), lds);
        if (e != hipSuccess) return e;
        if (occ < 1) occ = 1;
        occ_cache[a.k].store(occ, std::memory_order_relaxed);
    }
    const uint64_t want = static_cast<uint64_t>(occ) * (cus ? cus : 1u);
    const unsigned blocks = static_cast<unsigned>(want < ntiles ? want : ntiles);
    hipLaunchKernelGGL((k_sweep_pp<V, R>), dim3(blocks), dim3(threads), lds, s, psi, a, prog, mats,
                       ntiles);
    TUSQ_CHECK_LAUNCH();
    return hipSuccess;
}

template <typename V>
hipError_t launch_sweep_pp(V *psi, uint32_t n, const SweepArgs &a, const Instr2 *prog,
                           const V *mats, uint32_t reg_qubits, uint32_t cus, hipStream_t s) {
    if (reg_qubits == 3) return launch_pp_r<V, 3>(psi, n, a, prog, mats, cus, s);
    if (reg_qubits == 4) return launch_pp_r<V, 4>(psi, n, a, prog, mats, cus, s);
    return hipErrorInvalidValue;
}

template <typename V>
hipError_t launch_sweep_pipe(V *psi, uint32_t n, const SweepArgs &a, const Instr2 *prog,
                             const V *mats, uint32_t grid, hipStream_t s) {
    constexpr uint32_t R = sizeof(V) == 16 ? REG_QUBITS_C128 : REG_QUBITS_C64;
    constexpr uint32_t E = 16 / sizeof(V);
    if (a.k > n || a.k > 16 || a.k < R || n - a.k > 31 || a.low > a.k) return hipErrorInvalidValue;
    if (a.k - R > 8 || a.k - R < 6) return hipErrorInvalidValue;  // 64..256 threads, whole waves
    if (a.low < (E == 2 ? 1u : 0u)) return hipErrorInvalidValue;  // 16-byte transfers stay contiguous
    if ((sizeof(V) << a.k) > PIPE_TILE_BYTES) return hipErrorInvalidValue;
    const uint32_t ntiles = 1u << (n - a.k);
    const unsigned blocks = grid < ntiles ? grid : ntiles;
    const unsigned threads = 1u << (a.k - R);
    hipLaunchKernelGGL((k_sweep_pipe<V, R>), dim3(blocks), dim3(threads), 0, s, psi, a, prog, mats,
                       ntiles);
    TUSQ_CHECK_LAUNCH();
    return hipSuccess;
}

template <typename V>
hipError_t launch_leaf(const V *psi, uint32_t n, uint32_t log_chunk, double *acc, double w,
                       double *chunk_sum, double *prefix, double *norm_out, hipStream_t s) {
    if (log_chunk > n) return hipErrorInvalidValue;
    const uint64_t nc = 1ull << (n - log_chunk);
    hipLaunchKernelGGL(k_leaf<V>, dim3(static_cast<unsigned>(nc)), dim3(256), 0, s, psi, log_chunk,
                       acc, w, chunk_sum);
    TUSQ_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, chunk_sum, nc, prefix, norm_out);
    TUSQ_CHECK_LAUNCH();
    return hipSuccess;
}

template <typename V>
hipError_t launch_sample(const V *psi, uint32_t n, uint32_t log_chunk, const double *prefix,
                         const double *norm, uint64_t seed, uint32_t leaf, uint64_t shots,
                         uint64_t *out, hipStream_t s, uint64_t shot_base) {
    if (!shots) return hipSuccess;
    const uint64_t nc = 1ull << (n - log_chunk);
    const uint64_t blocks = (shots + 3) / 4;
    if (blocks > 0x7FFFFFFFull) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_sample<V>, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, psi,
                       log_chunk, prefix, nc, norm, seed, leaf, shots, shot_base, out);
    TUSQ_CHECK_LAUNCH();
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// Measurement layers.  Basis index = base(r) | dep(o): base(r) spreads the
// coset index r over the unmeasured bit positions (a zero inserted at every
// measured position, ascending), dep(o) puts outcome bit b at measured
// position q_b.
__device__ __forceinline__ uint64_t mcm_base(uint64_t r, const MeasArgs &a) {
    for (uint32_t b = 0; b < a.m; ++b) {
        const uint32_t q = a.q[b];
        r = ((r >> q) << (q + 1)) | (r & ((1ull << q) - 1));
    }
    return r;
}
__device__ __forceinline__ uint64_t mcm_dep(uint32_t o, const MeasArgs &a) {
    uint64_t x = 0;
    for (uint32_t b = 0; b < a.m; ++b) x |= static_cast<uint64_t>((o >> b) & 1u) << a.q[b];
    return x;
}

// partial[o * gridDim.x + block] = sum of |psi|^2 over outcome o's amplitudes
// that the block's threads visit (grid-stride over cosets, then a fixed tree)
template <typename V>
__global__ void __launch_bounds__(256) k_mcm_probs(const V *__restrict__ psi, uint64_t R,
                                                   MeasArgs a, double *__restrict__ partial) {
    __shared__ double red[256];
    const uint32_t no = 1u << a.m;
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    for (uint32_t o = 0; o < no; ++o) {
        const uint64_t dep = mcm_dep(o, a);
        double acc = 0.0;
        for (uint64_t r = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; r < R;
             r += stride)
            acc += prob(psi, mcm_base(r, a) | dep);
        red[threadIdx.x] = acc;
        __syncthreads();
        for (uint32_t h = 128; h > 0; h >>= 1) {
            if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0) partial[static_cast<uint64_t>(o) * gridDim.x + blockIdx.x] = red[0];
        __syncthreads();
    }
}

// P[o] = sum of partial[o * nblk + i] over i, one wavefront per outcome:
// lane l adds i = l, l + 64, ... in order, then a fixed shuffle tree
__global__ void __launch_bounds__(64) k_mcm_sum(const double *__restrict__ partial, uint32_t nblk,
                                                double *__restrict__ P) {
    const uint32_t o = blockIdx.x, lane = threadIdx.x;
    double s = 0.0;
    for (uint32_t i = lane; i < nblk; i += 64) s += partial[static_cast<uint64_t>(o) * nblk + i];
    for (uint32_t off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if (lane == 0) P[o] = s;
}

// dst[base | dep(p)] = (p == want) ? scale * src[base | dep(o)] : 0 for every
// outcome pattern p of the thread's coset (src == dst allowed)
template <typename V>
__global__ void __launch_bounds__(256) k_mcm_apply(const V *src, V *dst, uint64_t R, MeasArgs a,
                                                   uint32_t o, uint32_t want, double scale) {
    using T = typename RealOf<V>::T;
    const uint32_t no = 1u << a.m;
    const uint64_t dep_o = mcm_dep(o, a);
    const T sc = static_cast<T>(scale);
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    for (uint64_t r = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; r < R;
         r += stride) {
        const uint64_t base = mcm_base(r, a);
        V v = src[base | dep_o];
        v.x *= sc;
        v.y *= sc;
        V z;
        z.x = 0;
        z.y = 0;
        for (uint32_t p = 0; p < no; ++p) dst[base | mcm_dep(p, a)] = p == want ? v : z;
    }
}

constexpr uint32_t MCM_BLOCKS = 512;

template <typename V>
hipError_t launch_mcm_probs(const V *psi, uint32_t n, const MeasArgs &a, double *partial,
                            double *P, hipStream_t s) {
    if (a.m < 1 || a.m > 8 || a.m > n) return hipErrorInvalidValue;
    const uint64_t R = 1ull << (n - a.m);
    const uint32_t blocks = static_cast<uint32_t>(std::min<uint64_t>((R + 255) / 256, MCM_BLOCKS));
    hipLaunchKernelGGL(k_mcm_probs<V>, dim3(blocks), dim3(256), 0, s, psi, R, a, partial);
    TUSQ_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_mcm_sum, dim3(1u << a.m), dim3(64), 0, s, partial, blocks, P);
    TUSQ_CHECK_LAUNCH();
    return hipSuccess;
}

template <typename V>
hipError_t launch_mcm_apply(const V *src, V *dst, uint32_t n, const MeasArgs &a, uint32_t o,
                            uint32_t want, double scale, hipStream_t s) {
    if (a.m < 1 || a.m > 8 || a.m > n || o >= (1u << a.m) || want >= (1u << a.m))
        return hipErrorInvalidValue;
    const uint64_t R = 1ull << (n - a.m);
    const uint32_t blocks = static_cast<uint32_t>(std::min<uint64_t>((R + 255) / 256, 4096));
    hipLaunchKernelGGL(k_mcm_apply<V>, dim3(blocks), dim3(256), 0, s, src, dst, R, a, o, want,
                       scale);
    TUSQ_CHECK_LAUNCH();
    return hipSuccess;
}

template <typename V>
hipError_t launch_reset(V *psi, uint32_t n, hipStream_t s) {
    const uint64_t N = 1ull << n;
    hipLaunchKernelGGL(k_reset<V>, dim3(grid1(N, 256)), dim3(256), 0, s, psi, N);
    TUSQ_CHECK_LAUNCH();
    return hipSuccess;
}

hipError_t launch_to_c64(const double2 *src, float2 *dst, uint32_t n, hipStream_t s) {
    const uint64_t N = 1ull << n;
    hipLaunchKernelGGL(k_to_c64, dim3(grid1(N, 256)), dim3(256), 0, s, src, dst, N);
    TUSQ_CHECK_LAUNCH();
    return hipSuccess;
}

hipError_t launch_fill(double *p, uint64_t count, double v, hipStream_t s) {
    if (!count) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3(grid1(count, 256)), dim3(256), 0, s, p, count, v);
    TUSQ_CHECK_LAUNCH();
    return hipSuccess;
}

hipError_t sweep_kernel_setup() {
    const void *ks[10] = {reinterpret_cast<const void *>(k_sweep<double2>),
                         reinterpret_cast<const void *>(k_sweep<float2>),
                         reinterpret_cast<const void *>(k_sweep_reg<double2, 4>),
                         reinterpret_cast<const void *>(k_sweep_reg<float2, 4>),
                         reinterpret_cast<const void *>(k_sweep_reg<double2, 3>),
                         reinterpret_cast<const void *>(k_sweep_reg<float2, 3>),
                         reinterpret_cast<const void *>(k_sweep_pp<double2, 4>),
                         reinterpret_cast<const void *>(k_sweep_pp<float2, 4>),
                         reinterpret_cast<const void *>(k_sweep_pp<double2, 3>),
                         reinterpret_cast<const void *>(k_sweep_pp<float2, 3>)};
    for (const void *k : ks) {
        hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template hipError_t launch_sweep<double2>(double2 *, uint32_t, const SweepArgs &, const DOp *,
                                          const double2 *, hipStream_t);
template hipError_t launch_sweep<float2>(float2 *, uint32_t, const SweepArgs &, const DOp *,
                                         const float2 *, hipStream_t);
template hipError_t launch_sweep_reg<double2>(double2 *, uint32_t, const SweepArgs &,
                                              const Instr2 *, const double2 *, uint32_t, hipStream_t);
template hipError_t launch_sweep_reg<float2>(float2 *, uint32_t, const SweepArgs &,
                                             const Instr2 *, const float2 *, uint32_t, hipStream_t);
template hipError_t launch_sweep_pp<double2>(double2 *, uint32_t, const SweepArgs &,
                                              const Instr2 *, const double2 *, uint32_t, uint32_t,
                                              hipStream_t);
template hipError_t launch_sweep_pp<float2>(float2 *, uint32_t, const SweepArgs &, const Instr2 *,
                                             const float2 *, uint32_t, uint32_t, hipStream_t);
template hipError_t launch_sweep_pipe<double2>(double2 *, uint32_t, const SweepArgs &,
                                               const Instr2 *, const double2 *, uint32_t, hipStream_t);
template hipError_t launch_sweep_pipe<float2>(float2 *, uint32_t, const SweepArgs &, const Instr2 *,
                                              const float2 *, uint32_t, hipStream_t);
template hipError_t launch_leaf<double2>(const double2 *, uint32_t, uint32_t, double *, double,
                                         double *, double *, double *, hipStream_t);
template hipError_t launch_leaf<float2>(const float2 *, uint32_t, uint32_t, double *, double,
                                        double *, double *, double *, hipStream_t);
template hipError_t launch_sample<double2>(const double2 *, uint32_t, uint32_t, const double *,
                                           const double *, uint64_t, uint32_t, uint64_t,
                                           uint64_t *, hipStream_t, uint64_t);
template hipError_t launch_sample<float2>(const float2 *, uint32_t, uint32_t, const double *,
                                          const double *, uint64_t, uint32_t, uint64_t,
                                          uint64_t *, hipStream_t, uint64_t);
template hipError_t launch_mcm_probs<double2>(const double2 *, uint32_t, const MeasArgs &, double *,
                                              double *, hipStream_t);
template hipError_t launch_mcm_probs<float2>(const float2 *, uint32_t, const MeasArgs &, double *,
                                             double *, hipStream_t);
template hipError_t launch_mcm_apply<double2>(const double2 *, double2 *, uint32_t, const MeasArgs &,
                                              uint32_t, uint32_t, double, hipStream_t);
template hipError_t launch_mcm_apply<float2>(const float2 *, float2 *, uint32_t, const MeasArgs &,
                                             uint32_t, uint32_t, double, hipStream_t);
template hipError_t launch_reset<double2>(double2 *, uint32_t, hipStream_t);
template hipError_t launch_reset<float2>(float2 *, uint32_t, hipStream_t);

}  // namespace tusq
