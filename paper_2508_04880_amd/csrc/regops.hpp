// regops.hpp -- device helpers shared by the sweep kernels and the batched
// walk: complex arithmetic in the operands' precision, tile addressing, and
// register-blocked ops with LDS re-layouts driven by a host-compiled program
// (Instr).  Included by kernels.hip and batch.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace tusq {

// fused multiply-add in the precision of the operands (the double builtin
// would promote complex64 arithmetic to FP64)
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }


template <typename V> struct RealOf;
template <> struct RealOf<double2> { using T = double; };
template <> struct RealOf<float2> { using T = float; };

// acc + a * b as four fused multiply-adds
template <typename V>
__device__ __forceinline__ V cfma(V acc, V a, V b) {
    acc.x = fma_t(a.x, b.x, acc.x);
    acc.x = fma_t(-a.y, b.y, acc.x);
    acc.y = fma_t(a.x, b.y, acc.y);
    acc.y = fma_t(a.y, b.x, acc.y);
    return acc;
}
// a * b
template <typename V>
__device__ __forceinline__ V cmul(V a, V b) {
    V r;
    r.x = a.x * b.x;
    r.x = fma_t(-a.y, b.y, r.x);
    r.y = a.x * b.y;
    r.y = fma_t(a.y, b.x, r.y);
    return r;
}
template <typename V>
__device__ __forceinline__ V cconj(V a) {
    a.y = -a.y;
    return a;
}

__device__ __forceinline__ uint32_t insert0(uint32_t p, uint32_t bit) {
    const uint32_t lo = p & ((1u << bit) - 1u);
    return ((p >> bit) << (bit + 1)) | lo;
}

// The sweep's tile qubits, read from the kernel arguments with static
// indices only (a runtime index would turn every read into a dependent
// memory round trip).
struct QMap {
    uint32_t q[16];
};
__device__ __forceinline__ QMap qmap(const SweepArgs &a) {
    QMap m;
#pragma unroll
    for (int j = 0; j < 16; ++j) m.q[j] = a.q[j];
    return m;
}
__device__ __forceinline__ uint32_t qat(const QMap &m, uint32_t idx) {
    uint32_t r = 0;
#pragma unroll
    for (int j = 0; j < 16; ++j)
        if (static_cast<uint32_t>(j) == idx) r = m.q[j];
    return r;
}
// Tile base: spread the tile index over the qubits outside the tile.
__device__ __forceinline__ uint64_t tile_base(uint64_t t, const QMap &m, uint32_t k) {
#pragma unroll
    for (int j = 0; j < 16; ++j)
        if (static_cast<uint32_t>(j) < k) {
            const uint32_t q = m.q[j];
            t = ((t >> q) << (q + 1)) | (t & ((1ull << q) - 1ull));
        }
    return t;
}
// Global offset of local tile index l: bit j of l goes to qubit q[j].  The
// first `low` qubits are 0 .. low-1, so those bits stay in place.
__device__ __forceinline__ uint64_t scatter(uint32_t l, const QMap &m, uint32_t low, uint32_t k) {
    uint64_t off = l & ((1u << low) - 1u);
#pragma unroll
    for (int j = 0; j < 16; ++j)
        if (static_cast<uint32_t>(j) >= low && static_cast<uint32_t>(j) < k)
            off |= static_cast<uint64_t>((l >> j) & 1u) << m.q[j];
    return off;
}


// ---------------------------------------------------------------------------
// Register-blocked sweep.  A workgroup of 2^(k-R) threads owns one tile;
// thread t holds the 2^R amplitudes whose local index has t in the
// non-register bits and any value in the R register bits.  Ops on register
// qubits run entirely in registers (fully unrolled, matrix entries uniform);
// a re-layout writes the tile to LDS and reads it back with another set of
// register qubits.  LDS addresses are XOR-swizzled so that the power-of-two
// strides of a re-layout spread over all banks.
template <typename V>
struct Swz {
    static constexpr uint32_t SW = sizeof(V) == 16 ? 4 : 5;  // 256-byte bank row
    __device__ static __forceinline__ uint32_t phys(uint32_t l) {
        return l ^ (((l >> SW) ^ (l >> (2 * SW))) & ((1u << SW) - 1u));
    }
};

template <typename V, int R, int B>
__device__ __forceinline__ void reg_op1(V (&v)[1 << R], const V m0, const V m1, const V m2,
                                        const V m3) {
#pragma unroll
    for (int j = 0; j < (1 << R); ++j) {
        if (j & (1 << B)) continue;
        const V x0 = v[j], x1 = v[j | (1 << B)];
        v[j] = cfma(cmul(m0, x0), m1, x1);
        v[j | (1 << B)] = cfma(cmul(m2, x0), m3, x1);
    }
}

template <typename V, int R, int A, int B>
__device__ __forceinline__ void reg_op2(V (&v)[1 << R], const V *__restrict__ m) {
#pragma unroll
    for (int j = 0; j < (1 << R); ++j) {
        if (j & ((1 << A) | (1 << B))) continue;
        const int i[4] = {j, j | (1 << B), j | (1 << A), j | (1 << A) | (1 << B)};
        V x[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) x[r] = v[i[r]];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            V acc = cmul(m[4 * r], x[0]);
#pragma unroll
            for (int c = 1; c < 4; ++c) acc = cfma(acc, m[4 * r + c], x[c]);
            v[i[r]] = acc;
        }
    }
}

template <typename V, int R>
__device__ __forceinline__ void dispatch_op1(uint32_t b, V (&v)[1 << R], const V *m) {
    const V m0 = m[0], m1 = m[1], m2 = m[2], m3 = m[3];
    switch (b) {
    case 0: reg_op1<V, R, 0>(v, m0, m1, m2, m3); break;
    case 1: if constexpr (R > 1) reg_op1<V, R, 1>(v, m0, m1, m2, m3); break;
    case 2: if constexpr (R > 2) reg_op1<V, R, 2>(v, m0, m1, m2, m3); break;
    case 3: if constexpr (R > 3) reg_op1<V, R, 3>(v, m0, m1, m2, m3); break;
    case 4: if constexpr (R > 4) reg_op1<V, R, 4>(v, m0, m1, m2, m3); break;
    default: break;
    }
}

template <typename V, int R>
__device__ __forceinline__ void dispatch_op2(uint32_t ab, V (&v)[1 << R], const V *__restrict__ m) {
    switch (ab) {
#define TUSQ_OP2_CASE(A, B) \
    case (A) | ((B) << 3): if constexpr ((A) < R && (B) < R) reg_op2<V, R, A, B>(v, m); break;
        TUSQ_OP2_CASE(0, 1) TUSQ_OP2_CASE(0, 2) TUSQ_OP2_CASE(0, 3) TUSQ_OP2_CASE(0, 4)
        TUSQ_OP2_CASE(1, 0) TUSQ_OP2_CASE(1, 2) TUSQ_OP2_CASE(1, 3) TUSQ_OP2_CASE(1, 4)
        TUSQ_OP2_CASE(2, 0) TUSQ_OP2_CASE(2, 1) TUSQ_OP2_CASE(2, 3) TUSQ_OP2_CASE(2, 4)
        TUSQ_OP2_CASE(3, 0) TUSQ_OP2_CASE(3, 1) TUSQ_OP2_CASE(3, 2) TUSQ_OP2_CASE(3, 4)
        TUSQ_OP2_CASE(4, 0) TUSQ_OP2_CASE(4, 1) TUSQ_OP2_CASE(4, 2) TUSQ_OP2_CASE(4, 3)
#undef TUSQ_OP2_CASE
    default: break;
    }
}

// local index bits of thread t: t deposited into the positions of `free`
__device__ __forceinline__ uint32_t deposit(uint32_t t, uint32_t free, uint32_t k) {
    uint32_t out = 0, b = 0;
    for (uint32_t p = 0; p < k; ++p)
        if (free >> p & 1u) out |= ((t >> b++) & 1u) << p;
    return out;
}

template <int R>
__device__ __forceinline__ void unpack_set(uint32_t packed, uint32_t (&pos)[R], uint32_t &mask) {
    mask = 0;
#pragma unroll
    for (int i = 0; i < R; ++i) {
        pos[i] = (packed >> (5 * i)) & 31u;
        mask |= 1u << pos[i];
    }
}

// Workgroup barrier ordering LDS traffic only: s_waitcnt lgkmcnt(0)
// (vector-memory and export counters left at their maxima), then s_barrier.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_s_waitcnt(0xC07F);
    __builtin_amdgcn_s_barrier();
}

// Relayout addressing.  The swizzle is linear over GF(2) and the thread and
// register parts of a local index have disjoint bits, so
// phys(thread | reg) = phys(thread) ^ phys(reg): one XOR per element with a
// wave-uniform constant.
template <typename V, int R>
__device__ __forceinline__ void tile_addr(uint32_t tid, uint32_t k, uint32_t packed, uint32_t &pd,
                                          uint32_t (&pr)[1 << R]) {
    uint32_t pos[R], mask;
    unpack_set<R>(packed, pos, mask);
    pd = Swz<V>::phys(deposit(tid, ((1u << k) - 1u) & ~mask, k));
#pragma unroll
    for (int j = 0; j < (1 << R); ++j) {
        uint32_t l = 0;
#pragma unroll
        for (int i = 0; i < R; ++i)
            if (j >> i & 1) l |= 1u << pos[i];
        pr[j] = Swz<V>::phys(l);
    }
}

template <typename V, int R>
__device__ __forceinline__ void write_tile(const V (&v)[1 << R], V *lds, uint32_t tid, uint32_t k,
                                           uint32_t packed) {
    uint32_t pd, pr[1 << R];
    tile_addr<V, R>(tid, k, packed, pd, pr);
#pragma unroll
    for (int j = 0; j < (1 << R); ++j) lds[pd ^ pr[j]] = v[j];
}

template <typename V, int R>
__device__ __forceinline__ void read_tile(V (&v)[1 << R], const V *lds, uint32_t tid, uint32_t k,
                                          uint32_t packed) {
    uint32_t pd, pr[1 << R];
    tile_addr<V, R>(tid, k, packed, pd, pr);
#pragma unroll
    for (int j = 0; j < (1 << R); ++j) v[j] = lds[pd ^ pr[j]];
}

// Run a sweep program on the registers of one tile (see Instr).  `lds` is
// the tile-sized re-layout scratch; `dirty` says whether another thread may
// still be reading it.  The program starts and ends in the initial layout
// (register qubits = the top R local qubits).
template <typename V, int R>
__device__ __forceinline__ void run_program(V (&v)[1 << R], V *lds, uint32_t tid, uint32_t k,
                                            const Instr2 *__restrict__ prog, uint32_t ib,
                                            uint32_t ie, const V *__restrict__ mats, bool dirty) {
    uint32_t cur = 0;
#pragma unroll
    for (int i = 0; i < R; ++i) cur |= (k - R + i) << (5 * i);
    for (uint32_t pc = ib; pc < ie; ++pc) {
        const Instr2 ins = prog[pc];
        const uint32_t type = ins.w0 & 3u, arg = ins.w0 >> 2;
        if (type == 0u) {
            // a re-layout only needs the LDS traffic of the workgroup ordered:
            // wait for this wave's LDS operations, then meet at the barrier
            if (dirty) lds_barrier();
            write_tile<V, R>(v, lds, tid, k, cur);
            lds_barrier();
            read_tile<V, R>(v, lds, tid, k, arg);
            dirty = true;
            cur = arg;
        } else if (type == 1u) {
            dispatch_op1<V, R>(arg & 7u, v, mats + ins.mat);
        } else {
            dispatch_op2<V, R>(arg & 63u, v, mats + ins.mat);
        }
    }
}


}  // namespace tusq
