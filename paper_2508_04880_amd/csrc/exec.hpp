// exec.hpp -- device context and plan execution.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <atomic>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "engine.hpp"

namespace tusq {

void hip_check(hipError_t e, const char *what);

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    bool owned = true;  // false: a view of memory owned elsewhere, never freed
    // set: allocate and free in stream order on it (hipMallocAsync /
    // hipFreeAsync), so that growing a buffer does not wait for work that
    // other streams have queued, as hipFree does
    hipStream_t stream = nullptr;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf();
    void alloc(size_t b);
    void ensure(size_t b);  // reallocate only when larger than what is held;
                            // a borrowed view fails with TUSQ_ENOMEM instead
    void borrow(void *q, size_t b);
    void release();
};

// Device buffers of one running job, reusable by the next job on the same
// execution lane (they only grow).
struct Ctx;

struct Workspace {
    DevBuf psi, psi128, acc, csum, prefix, norms, samples, dops, mats, mats128, prog;
    DevBuf ckpt;  // checkpoint traversal: saved branch states; caching: cached nodes
    DevBuf mcm;   // measurement layers: per-block partial weights and P
    // acc and samples are the caller's device buffers: the run leaves the
    // distribution and samples there and copies neither back to the host
    bool device_outputs = false;
    // jobs running on the device now (serving lanes); while others run, a
    // persistent sweep leaves an eighth of the CUs' workgroup slots free so
    // that their kernels start without waiting for it
    const std::atomic<uint32_t> *co_running = nullptr;
    // serving lanes: two events with which a run keeps at most two windows
    // of work queued ahead on its stream, so that each launch sees how many
    // jobs run at its own time and a small job's kernels never queue behind
    // seconds of a large job's sweeps
    hipEvent_t window[2] = {nullptr, nullptr};
    // host word for the per-leaf norm readback of complex64 runs: one of
    // the context's pinned words, taken on first use (a copy into pageable
    // memory goes through a staging buffer), else `spare`; the
    // no-allocation run lends an ordinary host word
    double *host_word = nullptr;
    Ctx *word_ctx = nullptr;  // set while host_word is the context's
    double spare = 0.0;
    Workspace() = default;
    Workspace(const Workspace &) = delete;
    Workspace &operator=(const Workspace &) = delete;
    ~Workspace();
    double *readback_word(Ctx &ctx);
    uint64_t bytes() const;
    void release();
    void set_stream(hipStream_t s);  // every buffer allocates in order on s
};

struct Result {
    uint32_t n = 0;
    std::vector<double> dist;  // the distribution on the host, or empty ...
    std::shared_ptr<DevBuf> dist_dev;  // ... while it stays in device memory
    int device = 0;
    std::vector<uint64_t> samples;
    std::vector<double> norms;
    tusq_counters counters{};
    bool has_dist() const { return !dist.empty() || (dist_dev && dist_dev->p); }
    // write the 2^n probabilities to host memory
    void dist_copy(double *out) const;
};

struct Serving;     // request loop state (serve.cpp)
struct BatchCache;  // batched launches: reusable graph and its buffers (batch.hip)
void batch_cache_free(BatchCache *b);

// Launch shape of batched jobs of one qubit count: threads per workgroup,
// tile qubits (the qubit count itself when the state stays in LDS), low
// qubits always in a tile, dense ops per sweep (0 = the planner's default),
// and for states in global slots whether the sweeps run register-blocked
// programs (threads = 2^(tile qubits - 4)) or op lists in LDS.
struct BatchShape {
    uint32_t threads = 256, tile_qubits = 0, low_qubits = 0, max_ops = 0, reg = 0;
};

struct Ctx {
    int device = 0;
    int cus = 1;
    uint64_t budget = 0;
    hipStream_t stream = nullptr;
    std::mutex mu;
    std::vector<hipEvent_t> pool;
    Serving *serving = nullptr;
    std::map<uint64_t, std::array<uint32_t, 4>> tuned;  // autotuner choices
    void *scratch = nullptr;  // this device's copy of the static scratch array
    std::map<uint64_t, BatchShape> batch_tuned;  // (qubits << 8 | precision) -> shape
    BatchCache *batch = nullptr;
    std::mutex batch_mu;
    // pinned host words for complex64 norm readbacks, allocated with the
    // context: a host allocation during a run can wait for every stream's
    // queued work, which would stall a job behind the others on the device
    static constexpr uint32_t HOST_WORDS = 64;
    double *host_words = nullptr;
    std::vector<uint32_t> free_words;  // under mu

    Ctx(int dev, uint64_t budget);
    ~Ctx();
    hipEvent_t event();
    void recycle(std::vector<hipEvent_t> &evs);
    double *take_word();  // nullptr when all are taken
    void give_word(double *w);
};

// Size of the file-scope device array behind execute_plan_static: the
// no-allocation run keeps its state, sampler sums, norms and plan there.
constexpr uint64_t STATIC_SCRATCH_BYTES = TUSQ_NOALLOC_SCRATCH_BYTES;

// Device bytes a job needs (state, recompute buffer, accumulator, sampler
// scratch, samples, plan) -- used for admission.
uint64_t job_device_bytes(uint32_t n, uint32_t precision, uint64_t shots, bool want_dist);
// device bytes of a plan's checkpoint slots (checkpoint traversal)
uint64_t checkpoint_bytes(uint32_t n, uint32_t precision, uint64_t slots);

void execute_plan(Ctx &ctx, const Tree &t, const Plan &plan, const tusq_opts &o, hipStream_t s,
                  Result &res, Workspace *ws = nullptr, const std::atomic<bool> *cancel = nullptr);
// The same run with no device allocation: every work buffer is carved from
// the context's static scratch (TUSQ_ENOMEM when the job does not fit), the
// distribution is accumulated in dist (2^n doubles, or NULL without
// TUSQ_WANT_DIST) and the samples written to samples (samples_len u64)
// in caller device memory; neither is copied to the host.
void execute_plan_static(Ctx &ctx, const Tree &t, const Plan &plan, const tusq_opts &o,
                         hipStream_t s, Result &res, double *dist, uint64_t *samples,
                         uint64_t samples_len);
// DFTT+Caching over a circuit with measurement layers (host-driven walk: the
// outcome weights of every pre-measurement node come back to the host, which
// splits the node's shots and chooses the next launches)
void execute_mcm(Ctx &ctx, const Tree &t, const McmPlan &mp, const tusq_opts &o, hipStream_t s,
                 Result &res);
// device bytes of the measurement walk beyond a plain job: K cached states
// and the weight scratch
uint64_t mcm_bytes(uint32_t n, uint32_t precision, uint32_t K);

}  // namespace tusq

struct tusq_ctx {
    tusq::Ctx *c;
};
struct tusq_result {
    tusq::Result r;
};
