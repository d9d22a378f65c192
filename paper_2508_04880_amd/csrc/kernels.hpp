// kernels.hpp -- launch interface of the device kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace tusq {

// One dense op of a sweep: low byte = local qubit a, next byte = local qubit
// b (0xFF for a 1-qubit op); mat = offset into the complex matrix pool
// (2x2 or 4x4, row major, 4x4 basis index 2 * bit(a) + bit(b)).
struct alignas(8) DOp {
    uint32_t ab;
    uint32_t mat;
};

// One instruction of a register-blocked sweep program (layout of the
// host's Instr): w0 = type | arg << 2, mat = matrix offset.
struct alignas(8) Instr2 {
    uint32_t w0;
    uint32_t mat;
};

// register qubits per thread of the register-blocked sweep
constexpr uint32_t REG_QUBITS_C128 = 4;
constexpr uint32_t REG_QUBITS_C64 = 4;

// Arguments of one sweep launch, passed by value.
struct SweepArgs {
    uint32_t k;         // tile qubits
    uint32_t low;       // q[0 .. low) == 0 .. low-1
    uint32_t nops;
    uint32_t op_begin;
    uint32_t inverse;   // apply the ops' adjoints in reverse order
    uint32_t fwd_begin, fwd_end, inv_begin, inv_end;  // register programs
    // layouts (register word, thread word) the program of this direction
    // starts in (load) and ends in (store); thread word ~0u = positions
    // outside the register set in ascending order
    uint32_t lay_in_reg, lay_in_thr, lay_out_reg, lay_out_thr;
    uint8_t q[16];      // tile qubits, ascending
};

template <typename V>
hipError_t launch_sweep(V *psi, uint32_t n, const SweepArgs &a, const DOp *ops, const V *mats,
                        hipStream_t s);
template <typename V>
hipError_t launch_sweep_reg(V *psi, uint32_t n, const SweepArgs &a, const Instr2 *prog,
                            const V *mats, uint32_t reg_qubits, hipStream_t s);
// persistent ping-pong variant of launch_sweep_reg: min(tiles, resident
// workgroups per CU x cus) workgroups; programs must have even length
template <typename V>
hipError_t launch_sweep_pp(V *psi, uint32_t n, const SweepArgs &a, const Instr2 *prog,
                           const V *mats, uint32_t reg_qubits, uint32_t cus, hipStream_t s);
template <typename V>
hipError_t launch_sweep_pipe(V *psi, uint32_t n, const SweepArgs &a, const Instr2 *prog,
                             const V *mats, uint32_t grid, hipStream_t s);
template <typename V>
hipError_t launch_leaf(const V *psi, uint32_t n, uint32_t log_chunk, double *acc, double w,
                       double *chunk_sum, double *prefix, double *norm_out, hipStream_t s);
// draws shot_base .. shot_base + shots - 1 of leaf `leaf` into out[0 .. shots)
template <typename V>
hipError_t launch_sample(const V *psi, uint32_t n, uint32_t log_chunk, const double *prefix,
                         const double *norm, uint64_t seed, uint32_t leaf, uint64_t shots,
                         uint64_t *out, hipStream_t s, uint64_t shot_base = 0);

// A measurement layer: m (1..8) measured qubits, ascending.
struct MeasArgs {
    uint32_t m;
    uint8_t q[8];
};
// P[o] (2^m doubles) = FP64 weight of every outcome o of the layer; partial
// holds 512 * 2^m doubles of scratch.  Deterministic summation order.
template <typename V>
hipError_t launch_mcm_probs(const V *psi, uint32_t n, const MeasArgs &a, double *partial,
                            double *P, hipStream_t s);
// dst = the outcome-o part of src times scale, moved to pattern `want` (o
// itself, or 0 for a reset); every other pattern zero.  src == dst allowed.
template <typename V>
hipError_t launch_mcm_apply(const V *src, V *dst, uint32_t n, const MeasArgs &a, uint32_t o,
                            uint32_t want, double scale, hipStream_t s);
template <typename V>
hipError_t launch_reset(V *psi, uint32_t n, hipStream_t s);
hipError_t launch_to_c64(const double2 *src, float2 *dst, uint32_t n, hipStream_t s);
hipError_t launch_fill(double *p, uint64_t count, double v, hipStream_t s);
hipError_t sweep_kernel_setup();

}  // namespace tusq
