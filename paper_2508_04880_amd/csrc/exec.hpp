// exec.hpp -- device context and plan execution.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <atomic>
#include <map>
#include <mutex>
#include <vector>

#include "engine.hpp"

namespace tusq {

void hip_check(hipError_t e, const char *what);

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf();
    void alloc(size_t b);
    void ensure(size_t b);  // reallocate only when larger than what is held
    void release();
};

// Device buffers of one running job, reusable by the next job on the same
// execution lane (they only grow).
struct Workspace {
    DevBuf psi, psi128, acc, csum, prefix, norms, samples, dops, mats, mats128, prog;
    DevBuf ckpt;  // checkpoint traversal: saved branch states; caching: cached nodes
    DevBuf mcm;   // measurement layers: per-block partial weights and P
    uint64_t bytes() const;
    void release();
};

struct Result {
    uint32_t n = 0;
    std::vector<double> dist;
    std::vector<uint64_t> samples;
    std::vector<double> norms;
    tusq_counters counters{};
};

struct Serving;  // request loop state (serve.cpp)

struct Ctx {
    int device = 0;
    int cus = 1;
    uint64_t budget = 0;
    hipStream_t stream = nullptr;
    std::mutex mu;
    std::vector<hipEvent_t> pool;
    Serving *serving = nullptr;
    std::map<uint64_t, std::array<uint32_t, 4>> tuned;  // autotuner choices

    Ctx(int dev, uint64_t budget);
    ~Ctx();
    hipEvent_t event();
    void recycle(std::vector<hipEvent_t> &evs);
};

// Device bytes a job needs (state, recompute buffer, accumulator, sampler
// scratch, samples, plan) -- used for admission.
uint64_t job_device_bytes(uint32_t n, uint32_t precision, uint64_t shots, bool want_dist);
// device bytes of a plan's checkpoint slots (checkpoint traversal)
uint64_t checkpoint_bytes(uint32_t n, uint32_t precision, uint64_t slots);

void execute_plan(Ctx &ctx, const Tree &t, const Plan &plan, const tusq_opts &o, hipStream_t s,
                  Result &res, Workspace *ws = nullptr, const std::atomic<bool> *cancel = nullptr);
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
