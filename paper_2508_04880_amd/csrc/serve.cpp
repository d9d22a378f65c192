#include "serve.hpp"
namespace tusq {
uint64_t serving_submit(Ctx &, const Circuit &, const tusq_opts &) { fail(TUSQ_EUNSUPPORTED, "serving not available"); }
int serving_poll(Ctx &, uint64_t) { fail(TUSQ_EUNSUPPORTED, "serving not available"); }
void serving_wait(Ctx &, uint64_t, Result &) { fail(TUSQ_EUNSUPPORTED, "serving not available"); }
void serving_cancel(Ctx &, uint64_t) { fail(TUSQ_EUNSUPPORTED, "serving not available"); }
void serving_times(Ctx &, uint64_t, double *, double *, double *) { fail(TUSQ_EUNSUPPORTED, "serving not available"); }
void serving_shutdown(Ctx &) {}
}
