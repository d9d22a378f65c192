// serve.hpp -- asynchronous request loop and batched execution.
#pragma once

#include <vector>

#include "exec.hpp"

namespace tusq {

uint64_t serving_submit(Ctx &ctx, const Circuit &c, const tusq_opts &o);
int serving_poll(Ctx &ctx, uint64_t id);
void serving_wait(Ctx &ctx, uint64_t id, Result &out);
void serving_cancel(Ctx &ctx, uint64_t id);
void serving_times(Ctx &ctx, uint64_t id, double *submitted, double *admitted, double *finished);
void serving_shutdown(Ctx &ctx);

void run_batch(Ctx &ctx, const std::vector<const Circuit *> &circs, const tusq_opts &o,
               std::vector<Result> &out);
// time candidate launch shapes per qubit count (see tusq_batch_autotune)
void batch_autotune(Ctx &ctx, const std::vector<const Circuit *> &circs, const tusq_opts &o,
                    uint32_t probe_jobs);
// the shape run_batch uses for n-qubit jobs; *tuned: from the autotuner
BatchShape batch_shape(Ctx &ctx, uint32_t n, uint32_t precision, bool *tuned);

}  // namespace tusq
