/*
 * tusq.h -- C ABI of the MI355X (gfx950) noisy statevector engine.
 *
 * The engine implements the noisy-simulation method of TUSQ (Dangwal,
 * Oberoi, Sailopal, Shah, Chong; arXiv 2508.04880): the problem statement of
 * its Fig. 3 (inputs: a circuit in a 1-qubit + CNOT basis with Pauli noise
 * channels, a shot count and the pruning knobs alpha and beta; output: the
 * averaged output distribution, sampled as shots), the Error
 * Characterisation Module of Sec. III-A (error realisation (ER) sampling,
 * ER tallying, ER commutation, pruning with Eq. (2)) as host code, and the
 * Depth First Tree Traversal of Sec. III-B as HIP kernels.
 *
 * Conventions shared by every call:
 *   - Return value: TUSQ_OK (0) or a negative TUSQ_E* status.  No C++
 *     exception crosses this boundary.  tusq_last_error() returns a
 *     thread-local message describing the last failure on the calling
 *     thread (valid until the next failing call on that thread).
 *   - Ownership: every *_create / *_build / run call that hands out an
 *     object has a matching *_destroy; passing NULL to a destroy is a no-op.
 *     The library owns the device memory it allocates; caller buffers are
 *     only read or written during the call, except for *_device variants,
 *     which enqueue work on the caller's HIP stream.
 *   - Bit order: bit q of a basis index or of a sampled bitstring is
 *     qubit q (little endian).  Circuits take up to 34 qubits; a run needs
 *     its state (2^n x 16 B complex128, 2^n x 8 B complex64 plus a 2^n x
 *     16 B complex128 recompute state) and, with TUSQ_WANT_DIST, a 2^n x 8
 *     B accumulator in the context's budget (TUSQ_ENOMEM otherwise).  On
 *     one 288 GB device 33 qubits fit in either precision (complex128: 128
 *     GiB state + 64 GiB distribution; complex64: 64 + 128 + 64 GiB), 34
 *     do not; the largest run tested is 30 qubits.
 *   - Threading: circuits, trees and results may be used from any thread
 *     but not concurrently; a context is thread safe for
 *     tusq_submit / tusq_poll / tusq_wait / tusq_cancel.
 */
#ifndef TUSQ_ABI_H_
#define TUSQ_ABI_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TUSQ_ABI_VERSION 10u

/* status codes */
#define TUSQ_OK 0
#define TUSQ_EINVAL (-1)        /* bad argument: qubit out of range or repeated,
                                   probabilities negative / NaN / summing above
                                   1 + 1e-12, unknown gate kind, noise of the
                                   wrong arity, buffer too small, ...          */
#define TUSQ_ENOMEM (-2)        /* host allocation failed, or the job can
                                   never fit the context's HBM budget        */
#define TUSQ_EUNSUPPORTED (-3)  /* request outside what the engine does     */
#define TUSQ_EDEVICE (-4)       /* a HIP call failed                          */
#define TUSQ_EBUSY (-5)         /* job not finished (tusq_poll)               */
#define TUSQ_ECANCELED (-6)     /* job was cancelled                          */

/* gate kinds (Sec. III-A.3: circuits are in a 1-qubit + CNOT basis).
 * Matrices (no paper fixes them; these are the usual ones):
 *   U3(t, f, l) = [[cos t/2, -e^{il} sin t/2], [e^{if} sin t/2, e^{i(f+l)} cos t/2]]
 *   RX/RY/RZ(t) = exp(-i t P / 2);  S = diag(1, i);  T = diag(1, e^{i pi/4});
 *   SDG, TDG their adjoints; CX(c, t) flips t where c is 1.               */
enum {
    TUSQ_U3 = 0, TUSQ_RX, TUSQ_RY, TUSQ_RZ, TUSQ_H, TUSQ_S, TUSQ_SDG, TUSQ_T,
    TUSQ_TDG, TUSQ_X, TUSQ_Y, TUSQ_Z, TUSQ_CX, TUSQ_NUM_KINDS
};
/* kinds of the mid-circuit measurement layers tusq_circuit_measure appends
 * (not accepted by tusq_circuit_gate) */
enum { TUSQ_MEASURE = 13, TUSQ_MEASURE_RESET = 14 };
/* a caller's unitary (beyond the paper's named gates; its matrix is the
 * gate's params, see tusq_circuit_gate).  No error commutes through one:
 * a Pauli that reaches it stays just before it. */
enum { TUSQ_UNITARY1 = 15, TUSQ_UNITARY2 = 16 };
#define TUSQ_MAX_MEASURED 8u

/* amplitude precision of the sweeps; reductions are always FP64 */
enum { TUSQ_C128 = 0, TUSQ_C64 = 1 };

/* traversal policy between consecutive leaves (Sec. III-B):
 *   DFTT   undo the previous leaf back to the deepest shared node with
 *          inverse gates, then compute the new leaf from there;
 *   NAIVE  recompute every leaf from |0...0> ("DFTT switched off");
 *   HYBRID undo only when that costs strictly fewer gate and Pauli
 *          applications than recomputing from the root.                     */
/* traversals: plain DFTT (undo to the shared node), naive (restart from the
 * root), hybrid (undo only when cheaper), checkpoint (DFTT whose branch
 * states are kept in spare device memory: the next leaf restores the state
 * at its branch depth instead of undoing; Fig. 6E), caching (DFTT+Caching
 * for circuits with mid-circuit measurement layers, Sec. III-B.2: DFTT
 * within the stretches between layers, a LIFO cache of the pre-measurement
 * states of the cache_capacity layers closest to the leaves, uncached ones
 * recomputed from the root; cache_capacity 0 switches DFTT off).  Circuits
 * with measurement layers run only with TUSQ_CACHING, and without pruning:
 * every shot draws its own outcome from the Born weights of the layer (Philox
 * stream 3, counter (shot within its leaf, leaf, layer), half 0; the
 * smallest outcome o with u T < P_0 + ... + P_o), so a node's shots split
 * into outcome branches, each weighing its shots / S.                       */
enum { TUSQ_DFTT = 0, TUSQ_NAIVE = 1, TUSQ_HYBRID = 2, TUSQ_CHECKPOINT = 3, TUSQ_CACHING = 4 };

/* what a run returns */
#define TUSQ_WANT_DIST 1u      /* FP64 averaged distribution, 2^n values */
#define TUSQ_WANT_SAMPLES 2u   /* one u64 bitstring per shot             */
#define TUSQ_WANT_NORMS 4u     /* FP64 norm of every leaf state          */

typedef struct tusq_ctx tusq_ctx;
typedef struct tusq_circuit tusq_circuit;
typedef struct tusq_tree tusq_tree;
typedef struct tusq_result tusq_result;

typedef struct {
    uint64_t shots;            /* S (1 .. 2^32 - 1)                            */
    uint64_t seed;             /* Philox4x32-10 key for ER sampling (stream 0),
                                  pruning selection (1) and shot sampling (2) */
    uint32_t alpha_num;        /* significance: alpha_den * s_i >=            */
    uint32_t alpha_den;        /*   alpha_num * s_max (Sec. III-A.4)          */
    uint32_t beta;             /* insignificant circuits kept (Eq. (2))       */
    uint32_t precision;        /* TUSQ_C128 | TUSQ_C64                        */
    uint32_t traversal;        /* TUSQ_DFTT | NAIVE | HYBRID | CHECKPOINT |
                                  CACHING                                     */
    uint32_t commute;          /* ER commutation on/off (Sec. III-A.2)         */
    uint32_t prune;            /* pruning on/off                               */
    double drift_bound;        /* C64 only: recompute a leaf from the root in
                                  complex128 when |norm - 1| exceeds this     */
    uint32_t max_passes_between_recompute; /* C64 only: also recompute after
                                  this many sweeps since the last exact state
                                  (0 = never)                                  */
    uint64_t leaf_begin;       /* run leaves [leaf_begin, leaf_end) of the    */
    uint64_t leaf_end;         /*   depth-first leaf list (0, 0 = all)        */
    uint32_t want;             /* TUSQ_WANT_* bitmask                          */
    uint32_t fusion_max_qubits;/* qubits per fused sweep tile (0 = auto)      */
    uint32_t fusion_max_ops;   /* dense ops per fused sweep (0 = auto)        */
    uint32_t fusion_low_qubits;/* low qubits every tile keeps (0 = auto)      */
    uint32_t profile;          /* 1: time every sweep with HIP events         */
    int32_t debug_fail_at_step;/* >= 0: fail with TUSQ_EDEVICE before that
                                  schedule step (tests of error paths)        */
    uint32_t host_threads;     /* host threads for the ECM (0 = all cores)    */
    uint32_t sweep_kernel;     /* 0 auto (= 4), 1 register-blocked, one tile
                                  per workgroup (16 amplitudes per thread),
                                  2 the same with the next tile prefetched
                                  into LDS (persistent grid), 3 as 1 with 8
                                  amplitudes per thread, 4 persistent
                                  register-blocked with the next tile
                                  prefetched into registers (16 per thread),
                                  5 as 4 with 8 per thread                   */
    uint32_t cache_capacity;   /* TUSQ_CACHING: pre-measurement states kept
                                  (K of Sec. III-B.2; device slots of one
                                  state each)                                 */
    uint32_t checkpoint_slots; /* TUSQ_CHECKPOINT: most branch states kept
                                  (0 = as many as the walk needs).  When a save
                                  finds them all in use, the state farthest
                                  from the leaves is dropped, and a leaf
                                  branching at a dropped depth undoes the
                                  previous leaf back to it instead (a hybrid
                                  of checkpointing and uncomputation)        */
    uint32_t fusion_search;    /* how a sweep picks its tile qubits: 0 auto
                                  (= 2), 1 the qubits the tokens claim in
                                  circuit order, 2 also every window of
                                  consecutive qubits above the low ones (the
                                  candidate taking the most tokens wins)    */
} tusq_opts;

typedef struct {
    uint64_t fwd_gates, inv_gates;      /* gate applications (forward / undo)    */
    uint64_t fwd_paulis, inv_paulis;    /* Pauli error applications              */
    uint64_t resets, leaves, draws;
    uint64_t ret_gates, ret_paulis;     /* a final return to the root would undo
                                           these (the paper's 2|E| counts it)   */
    uint64_t passes_fwd, passes_inv;    /* fused HBM sweeps                       */
    uint64_t leaf_sweeps;               /* leaf accumulation sweeps               */
    uint64_t recomputes, recompute_passes;
    uint64_t sweep_bytes;               /* algorithmic bytes of all sweeps        */
    uint64_t checkpoint_saves, checkpoint_restores; /* checkpoint traversal */
    uint64_t sweep_flops;               /* real floating-point operations of the
                                           sweeps' dense ops: 16 per amplitude for
                                           a 2x2, 32 for a 4x4 (one complex
                                           multiply-add = 8)                     */
    uint64_t mcm_edges;                 /* measurement edges applied (forward)   */
    uint64_t paper_ops;                 /* the operation count of Sec. III-B.2:
                                           1 per 1-qubit gate or Pauli applied
                                           (either direction), 4 per CX, 1 per
                                           measurement edge, 0 for resets and
                                           cache fetches (Eq. (3)'s N)           */
    uint64_t pass_events;               /* sweeps timed with events (profile)    */
    double pass_seconds;                /* their summed device time               */
    double host_ecm_seconds, host_plan_seconds, device_seconds;
    double max_norm_drift;              /* max |norm - 1| over leaves (FP64);
                                           complex64: before any recompute       */
    uint64_t batch_graph_reused;        /* tusq_run_batch: 1 when the call
                                           replayed the graph an earlier call
                                           captured, 0 when it captured one     */
} tusq_counters;

typedef struct {
    uint64_t n_leaves, n_events, n_raw_events;
    uint64_t raw_unique, canonical_unique, significant, insignificant;
    uint64_t s_insig, d_selected, s_max;
} tusq_tree_info;

const char *tusq_last_error(void);
uint32_t tusq_abi_version(void);

/* alpha = 1/100, beta = 100 (the paper's defaults, Sec. III-A.4 and V-B),
 * C128, plain DFTT, commutation and pruning on, drift_bound 1e-6, all
 * leaves, want = DIST | SAMPLES, automatic fusion, host_threads 0.       */
void tusq_opts_default(tusq_opts *opts);

/* ---- circuits ----------------------------------------------------------- */
int tusq_circuit_create(uint32_t n_qubits, tusq_circuit **out);
/* Append a gate.  qubits: 1 entry (2 for CX: control, target); params: 3
 * doubles (U3: theta, phi, lambda; RX/RY/RZ: angle first), may be NULL for
 * parameterless kinds.  TUSQ_UNITARY1: params holds the 2x2 matrix, row-
 * major, as 8 doubles (re, im pairs); TUSQ_UNITARY2: two distinct qubits
 * and the 4x4 as 32 doubles, basis index 2 * bit(qubits[0]) + bit(qubits[1]);
 * EINVAL unless the matrix is finite and unitary to 1e-10 (max entry of
 * U^H U - I).  The matrix is copied.  gate_index_out (may be NULL)
 * receives its index.                                                      */
int tusq_circuit_gate(tusq_circuit *c, uint32_t kind, const uint32_t *qubits,
                      const double *params, uint32_t *gate_index_out);
/* Attach a Pauli channel right after gate gate_index (Sec. II, Eq. (4) form):
 * 1-qubit gate: n_probs = 3, (pX, pY, pZ);  CX or UNITARY2: n_probs = 15,
 * entry k - 1 for the Pauli k = 4a + b (a on the first qubit -- a CX's
 * control --, b on the second; I=0 X=1 Y=2 Z=3).
 * The identity takes the remaining probability.  One channel per gate.      */
int tusq_circuit_pauli_noise(tusq_circuit *c, uint32_t gate_index, const double *probs,
                             uint32_t n_probs);
/* Pauli-twirled thermal relaxation (Sec. VI-A, Eq. (4)): over a duration t
 * with relaxation time T1 and dephasing time T2 the channel becomes
 * pX = pY = (1 - exp(-t/T1)) / 4, pZ = (1 - exp(-t/T2)) / 2 - (1 - exp(-t/T1)) / 4.
 * probs[0..2] receive (pX, pY, pZ).  EINVAL unless t >= 0, T1 > 0,
 * 0 < T2 <= 2 T1 (pZ >= 0) and probs is not NULL.                          */
int tusq_thermal_pauli_probs(double t, double t1, double t2, double *probs);
/* Attach that channel after a gate: a 1-qubit gate gets (pX, pY, pZ); a CX
 * gets the product of the two qubits' independent channels (15 outcomes,
 * ordered as in tusq_circuit_pauli_noise).  Same rules as
 * tusq_circuit_pauli_noise otherwise.                                      */
int tusq_circuit_thermal_noise(tusq_circuit *c, uint32_t gate_index, double t, double t1,
                               double t2);
/* Read-out (measurement) error (Sec. IV-D lists it among the noise models;
 * Sec. VI-A: a Pauli channel as it stands): the final read-out of `qubit`
 * reports the flipped bit with probability p.  That is an X error just
 * before the read-out, so the call appends RZ(0) -- the identity -- on the
 * qubit with the channel (pX, pY, pZ) = (p, 0, 0).  Call it after the
 * qubit's last gate: a gate appended later acts after the flip.  EINVAL
 * unless 0 <= p <= 1; nothing is appended then.  gate_index_out (may be
 * NULL) receives the appended gate's index.                                */
int tusq_circuit_readout_noise(tusq_circuit *c, uint32_t qubit, double p,
                               uint32_t *gate_index_out);
/* Append a layer of concurrent Z-basis measurements of `count` distinct
 * qubits (1 .. TUSQ_MAX_MEASURED), one non-invertible edge of the circuit
 * tree (Sec. III-B.2); reset != 0 returns the measured qubits to |0>
 * afterwards.  Outcome o of the layer has bit b = the value of the b-th
 * measured qubit in ascending order.  A layer takes no noise channel;
 * errors do not commute through a measurement of their qubit.            */
int tusq_circuit_measure(tusq_circuit *c, const uint32_t *qubits, uint32_t count, int reset,
                         uint32_t *gate_index_out);
int tusq_circuit_destroy(tusq_circuit *c);

/* ---- host-only error characterisation (no GPU needed) -------------------- */
/* Sample every channel for every shot (Philox4x32-10: shot j, channel c uses
 * counter (c >> 1, j, 0, 0), half c & 1, against integer thresholds of the
 * cumulative probabilities), tally identical ERs, push every error right by
 * rules 1-6 to its canonical position (just before the first gate it cannot
 * pass), re-tally, prune (Eq. (2)) and order the leaves depth first.       */
int tusq_ecm_build(const tusq_circuit *c, const tusq_opts *opts, tusq_tree **out);
int tusq_tree_get_info(const tusq_tree *t, tusq_tree_info *out);
/* Byte image of the tree (little endian): u32 0x51535554, u32 1, u32 n,
 * u32 G, u64 shots, u64 leaves, then per leaf u64 count, u64 shots,
 * u64 weight numerator, u64 weight denominator, u32 n_events and n_events x
 * (u32 slot, u32 qubit, u8 pauli).  With buf == NULL only *len_out is set. */
int tusq_tree_serialize(const tusq_tree *t, uint8_t *buf, size_t cap, size_t *len_out);
/* Raw (pre-commutation) events sorted by (shot, channel); cap = entries. */
int tusq_tree_raw_events(const tusq_tree *t, uint32_t *shot, uint32_t *channel,
                         uint8_t *outcome, uint64_t cap, uint64_t *n_out);
/* SHA-256 (FIPS 180-4) of those raw events, in that order, each as 9 bytes:
 * u32 shot, u32 channel (little endian), u8 outcome -- a fingerprint of the
 * error-sampling stage (Sec. III-A.1) for comparing runs and
 * implementations without moving the list.  Writes 32 bytes.            */
int tusq_raw_er_hash(const tusq_tree *t, uint8_t *sha256_out);
int tusq_tree_destroy(tusq_tree *t);
/* Schedule and fuse without a device; fills the host-side counters a run
 * with these options would report (gate / Pauli applications, sweeps).     */
int tusq_plan_counters(const tusq_circuit *c, const tusq_tree *t, const tusq_opts *opts,
                       tusq_counters *out);
/* Dump the fused sweeps of a plan (for inspection): for sweep i, its tile
 * qubits and dense ops.  Returns the number of sweeps in *n_passes; arrays
 * may be NULL to query sizes.  qubits: 16 per sweep (unused = 0xFFFFFFFF);
 * op: (first op, op count) per sweep; ops: (local a, local b or 0xFF, matrix
 * offset in complex numbers) per op; mats: complex128 entries.           */
int tusq_plan_dump(const tusq_circuit *c, const tusq_tree *t, const tusq_opts *opts,
                   uint64_t *n_steps, int64_t *steps, uint64_t *n_passes, uint32_t *qubits,
                   uint64_t *op_range, uint64_t *n_ops, uint32_t *ops, uint64_t *n_mats,
                   double *mats);

/* Dump the register-blocked programs of a plan's sweeps.  A layout of a
 * tile is a register word (bits 5i.. = local position of register bit i)
 * and a thread word (bits 4b.. = local position of thread-index bit b, or
 * 0xFFFFFFFF: the positions outside the register set, ascending).  instr
 * holds 2 u32 per instruction, (w0 = type | arg << 2, m):
 *   type 0  re-layout into (register word arg, thread word m);
 *   type 1  2x2 op on register bit arg & 7, matrix offset m (complex);
 *   type 2  4x4 op on register bits arg & 7 (high bit of the 4x4 index)
 *           and (arg >> 3) & 7, matrix offset m;
 *   type 3  swap register bit arg & 7 with thread (lane) bit (arg >> 3) & 7.
 * ranges holds 12 u32 per sweep: forward begin, end, undo begin, end, then
 * the forward program's start layout (2 words) and end layout (2 words),
 * then the same for the undo program.  *reg_qubits receives R.  Arrays may
 * be NULL to query sizes.                                                  */
int tusq_plan_dump_programs(const tusq_circuit *c, const tusq_tree *t, const tusq_opts *opts,
                            uint64_t *n_instr, uint32_t *instr, uint64_t *n_passes,
                            uint32_t *ranges, uint32_t *reg_qubits);

/* ---- device execution ----------------------------------------------------- */
/* A context owns device buffers, streams and the HBM accounting of one GPU.
 * hbm_budget_bytes = 0 means the device's free memory at creation.         */
int tusq_ctx_create(int hip_device, uint64_t hbm_budget_bytes, tusq_ctx **out);
int tusq_ctx_destroy(tusq_ctx *ctx);

/* Run one job to completion: ECM on the host, then the depth-first walk on
 * the device on hip_stream (a hipStream_t; NULL = the context's stream).
 * Synchronises before returning.  The FP64 distribution (TUSQ_WANT_DIST)
 * stays in the device memory it was accumulated in, held by the result
 * until tusq_result_destroy; tusq_result_distribution copies it to the
 * host, tusq_result_distribution_device to caller device memory.  Samples,
 * norms and counters are on the host.  (Served and batched jobs return
 * their distribution on the host.)                                          */
int tusq_run(tusq_ctx *ctx, const tusq_circuit *c, const tusq_opts *opts, void *hip_stream,
             tusq_result **out);
/* Same, for a tree built earlier with tusq_ecm_build (host stages untimed). */
int tusq_run_tree(tusq_ctx *ctx, const tusq_circuit *c, const tusq_tree *t,
                  const tusq_opts *opts, void *hip_stream, tusq_result **out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * run as tusq_run_tree with no device allocation and no device copy back.
 * The state, the complex128 recompute state (TUSQ_C64), the sampler's chunk
 * sums and prefix, the leaf norms, the uploaded plan and any checkpoint
 * slots live in a static device array of TUSQ_NOALLOC_SCRATCH_BYTES per
 * GPU, held until the process ends; a job whose buffers do not fit fails
 * with TUSQ_ENOMEM before any device work (about 21 qubits at most in
 * complex128 with a small plan).  dist_dev receives the 2^n FP64
 * probabilities (required with TUSQ_WANT_DIST, else ignored) and
 * samples_dev the job's samples (samples_len u64, at least the slice's
 * shots, required with TUSQ_WANT_SAMPLES); both are caller device memory
 * on the context's device.  counters_out (host, may be NULL) receives the
 * counters.  Runs on hip_stream (NULL = the context's stream) and returns
 * when the work has completed.  Measurement circuits: TUSQ_EUNSUPPORTED.
 * Every call on one GPU shares that GPU's array, whichever context makes
 * it: calls that overlap in time on one GPU race and give wrong results. */
#define TUSQ_NOALLOC_SCRATCH_BYTES (64ull << 20)
int tusq_run_tree_noalloc(tusq_ctx *ctx, const tusq_circuit *c, const tusq_tree *t,
                          const tusq_opts *opts, void *hip_stream, double *dist_dev,
                          uint64_t *samples_dev, uint64_t samples_len,
                          tusq_counters *counters_out);

/* Autotuner: time a few candidate sweep shapes (tile qubits, low qubits,
 * dense ops per sweep, amplitudes per thread) on the depth-first slice
 * [opts->leaf_begin, opts->leaf_begin + probe_leaves) of tree t and write
 * the fastest into *tuned (a copy of *opts with fusion_max_qubits,
 * fusion_low_qubits, fusion_max_ops and sweep_kernel set).  The choice is
 * cached in the context per (qubits, precision, gate count).  States that
 * fit one tile need no tuning and are returned unchanged.                */
int tusq_autotune(tusq_ctx *ctx, const tusq_circuit *c, const tusq_tree *t, const tusq_opts *opts,
                  uint32_t probe_leaves, tusq_opts *tuned);

/* Serving: asynchronous jobs admitted by HBM need (state + recompute buffer
 * + FP64 accumulator + sampler scratch) against the context budget.  Jobs
 * that arrive while others run are admitted as memory and execution lanes
 * free up and run concurrently on separate streams in bounded chunks.     */
int tusq_submit(tusq_ctx *ctx, const tusq_circuit *c, const tusq_opts *opts,
                uint64_t *job_id);
int tusq_poll(tusq_ctx *ctx, uint64_t job_id, int *state_out); /* 0 queued, 1 running,
                                                                   2 done, 3 failed,
                                                                   4 cancelled */
int tusq_wait(tusq_ctx *ctx, uint64_t job_id, tusq_result **out);
int tusq_cancel(tusq_ctx *ctx, uint64_t job_id);
/* Timestamps (seconds, context clock) of a finished job: submitted, admitted,
 * finished. */
int tusq_job_times(tusq_ctx *ctx, uint64_t job_id, double *submitted, double *admitted,
                   double *finished);

/* Batching: many small independent jobs (n <= 16) with independent
 * sub-trees walked in parallel (Sec. III-B, Fig. 6E).  Each job's leaves are
 * cut into work units (job, leaf range) that start from |0...0>; units of
 * one qubit count run in one persistent launch that takes them from a
 * device queue (largest first), with the state in LDS (up to 2^13
 * amplitudes complex128, 2^14 complex64) or in a per-workgroup global slot
 * swept tile by tile.  The launches of a call (queue reset, one per qubit
 * count, combine) form one hipGraph; a later call whose launch shapes match
 * and whose buffers fit replays it (counters.batch_graph_reused).  Job i
 * uses seed opts->seed + i; outs[i] receives its result.  complex64 jobs
 * have no recompute: counters.max_norm_drift reports each job's largest
 * |norm - 1|.  Several threads may call it on one context: their host
 * stages run concurrently, their device work one call at a time.         */
int tusq_run_batch(tusq_ctx *ctx, const tusq_circuit *const *circs, const tusq_opts *opts,
                   size_t n_jobs, tusq_result **outs);

/* Batch autotuner: for every qubit count among the jobs (at opts->precision)
 * not tuned yet in this context, time candidate launch shapes -- threads
 * per workgroup (256 / 512 / 1024), and for states kept in global memory
 * the tile qubits, the low qubits always in a tile and the dense ops per
 * sweep, op lists in LDS or register-blocked programs -- on its
 * probe_jobs jobs with the most gates (at the call's shot count, at most
 * 10^4), each shape timed twice, and keep the fastest if it beats the
 * default shape by 3 %; tusq_run_batch then uses it for jobs of that size.
 * With the environment variable TUSQ_TUNE_LOG set, each shape's time goes
 * to stderr. */
int tusq_batch_autotune(tusq_ctx *ctx, const tusq_circuit *const *circs, const tusq_opts *opts,
                        size_t n_jobs, uint32_t probe_jobs);
/* The launch shape tusq_run_batch uses for n-qubit jobs at a precision:
 * shape[0] threads per workgroup, [1] tile qubits (n itself when the state
 * stays in LDS), [2] low qubits, [3] dense ops per sweep (0 = the planner's
 * default), [4] 1 when states in global slots are swept by register-blocked
 * programs (16 amplitudes per thread), 0 by op lists in LDS; returns 1 in
 * *tuned when it came from the autotuner.                                  */
int tusq_batch_shape(tusq_ctx *ctx, uint32_t n_qubits, uint32_t precision, uint32_t shape[5],
                     int *tuned);

/* ---- results --------------------------------------------------------------- */
int tusq_result_distribution(const tusq_result *r, double *out, uint64_t len);
/* The same 2^n FP64 values written into caller device memory (e.g. a
 * framework tensor's data pointer) on the caller's HIP stream (NULL = the
 * null stream); dptr must hold 2^n doubles on the device the result came
 * from.  Returns once the copy has completed.  EINVAL without a
 * distribution or with a NULL pointer; EDEVICE if the copy fails.        */
int tusq_result_distribution_device(const tusq_result *r, void *dptr, void *hip_stream);
int tusq_result_samples(const tusq_result *r, uint64_t *out, uint64_t len);
int tusq_result_norms(const tusq_result *r, double *out, uint64_t len);
int tusq_result_counters(const tusq_result *r, tusq_counters *out);
int tusq_result_num_samples(const tusq_result *r, uint64_t *out);
int tusq_result_destroy(tusq_result *r);

#ifdef __cplusplus
}
#endif
#endif /* TUSQ_ABI_H_ */
