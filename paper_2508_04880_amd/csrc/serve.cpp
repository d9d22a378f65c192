// serve.cpp -- asynchronous noisy-simulation requests with continuous
// admission.
//
// A submitted job first gets its host work (error characterisation and
// plan) on a planner thread.  Execution lanes, each with its own HIP stream
// and reusable device workspace (allocated in stream order), take planned
// jobs in arrival order, skipping jobs whose device memory (state,
// complex128 recompute buffer, FP64 accumulator, sampler scratch, samples,
// plan) does not fit what the context budget has left; two of the four
// lanes take jobs of at most 22 qubits only.  A job admitted while others
// run overlaps with them on the device: every lane keeps at most two
// windows of work queued ahead, and while several jobs run its persistent
// sweeps leave an eighth of the workgroup slots to the others, so that a
// small job's kernels do not wait for a large job's sweeps.  Jobs
// run their schedule in chunks and stop at a chunk boundary when cancelled.
// Every job owns its buffers and the kernels' reductions have a fixed
// order, so a job's result is the same alone or in any mix.
#include <algorithm>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>

#include "serve.hpp"

namespace tusq {

namespace {
enum : int { JS_QUEUED = 0, JS_RUNNING = 1, JS_DONE = 2, JS_FAILED = 3, JS_CANCELLED = 4 };
constexpr unsigned N_LANES = 4;     // one per hardware queue of the device
constexpr unsigned N_PLANNERS = 2;  // host threads for the ECM and planning
// the last lanes take small jobs only, so that a small request never waits
// behind large ones that hold every lane (a 30-qubit job runs for a minute)
constexpr unsigned N_SMALL_LANES = 2;
constexpr uint32_t SMALL_LANE_MAX_QUBITS = 22;
}  // namespace

struct Job {
    uint64_t id = 0;
    Circuit c;
    tusq_opts o{};
    int state = JS_QUEUED;
    bool planned = false;
    Tree tree;
    Plan plan;
    uint64_t need = 0;
    Result res;
    int err_code = 0;
    std::string err_msg;
    double t_submit = 0, t_admit = 0, t_finish = 0, ecm_s = 0, plan_s = 0;
    std::atomic<bool> cancel{false};
};

struct Serving {
    Ctx &ctx;
    std::mutex mu;
    std::condition_variable cv;
    std::map<uint64_t, std::shared_ptr<Job>> jobs;
    std::deque<std::shared_ptr<Job>> to_plan, ready;
    std::vector<uint64_t> lane_charge;
    std::atomic<uint32_t> running{0};  // jobs on the device now
    uint64_t next_id = 1;
    bool stop = false;
    std::vector<std::thread> threads;

    explicit Serving(Ctx &c) : ctx(c), lane_charge(N_LANES, 0) {
        for (unsigned i = 0; i < N_PLANNERS; ++i) threads.emplace_back([this] { planner(); });
        for (unsigned i = 0; i < N_LANES; ++i) threads.emplace_back([this, i] { lane(i); });
    }
    ~Serving() {
        {
            std::lock_guard<std::mutex> g(mu);
            stop = true;
        }
        cv.notify_all();
        for (auto &t : threads) t.join();
    }

    uint64_t used() const {
        uint64_t u = 0;
        for (uint64_t c : lane_charge) u += c;
        return u;
    }

    void finish(const std::shared_ptr<Job> &j, int state, int code, const std::string &msg) {
        std::lock_guard<std::mutex> g(mu);
        j->state = state;
        j->err_code = code;
        j->err_msg = msg;
        j->t_finish = now_seconds();
        j->tree = Tree();
        j->plan = Plan();
        cv.notify_all();
    }

    void planner() {
        for (;;) {
            std::shared_ptr<Job> j;
            {
                std::unique_lock<std::mutex> g(mu);
                cv.wait(g, [&] { return stop || !to_plan.empty(); });
                if (stop) return;
                j = to_plan.front();
                to_plan.pop_front();
            }
            if (j->cancel.load()) {
                finish(j, JS_CANCELLED, TUSQ_ECANCELED, "job cancelled");
                continue;
            }
            try {
                const double t0 = now_seconds();
                j->tree = build_tree(j->c, j->o);
                const double t1 = now_seconds();
                j->plan = build_plan(j->c, j->tree, j->o, j->o.precision == TUSQ_C64);
                j->ecm_s = t1 - t0;
                j->plan_s = now_seconds() - t1;
                // checkpoint slots join the job's device memory
                j->need += checkpoint_bytes(j->c.n, j->o.precision, j->plan.checkpoint_slots);
                if (j->need > ctx.budget)
                    fail(TUSQ_ENOMEM, "job's checkpoints exceed the device memory budget");
            } catch (const Error &e) {
                finish(j, JS_FAILED, e.code, e.msg);
                continue;
            } catch (const std::exception &e) {
                finish(j, JS_FAILED, TUSQ_ENOMEM, e.what());
                continue;
            }
            if (j->cancel.load()) {  // cancelled while its host work ran
                finish(j, JS_CANCELLED, TUSQ_ECANCELED, "job cancelled");
                continue;
            }
            {
                std::lock_guard<std::mutex> g(mu);
                j->planned = true;
                ready.push_back(j);
            }
            cv.notify_all();
        }
    }

    void lane(unsigned id) {
        hipStream_t s = nullptr;
        if (hipSetDevice(ctx.device) != hipSuccess ||
            hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess)
            return;
        Workspace ws;
        ws.co_running = &running;
        ws.set_stream(s);
        for (hipEvent_t &e : ws.window)
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming | hipEventBlockingSync) != hipSuccess)
                e = nullptr;
        for (;;) {
            std::shared_ptr<Job> j;
            {
                std::unique_lock<std::mutex> g(mu);
                for (;;) {
                    if (stop) break;
                    // first planned job, in arrival order, that fits the budget
                    // (and, on a small-job lane, is small)
                    const uint64_t others = used() - lane_charge[id];
                    const bool small_only = id >= N_LANES - N_SMALL_LANES;
                    auto it = std::find_if(ready.begin(), ready.end(), [&](const std::shared_ptr<Job> &x) {
                        if (small_only && x->c.n > SMALL_LANE_MAX_QUBITS) return false;
                        return others + std::max<uint64_t>(ws.bytes(), x->need) <= ctx.budget;
                    });
                    if (it != ready.end()) {
                        j = *it;
                        ready.erase(it);
                        lane_charge[id] = std::max<uint64_t>(ws.bytes(), j->need);
                        running.fetch_add(1);
                        j->state = JS_RUNNING;
                        j->t_admit = now_seconds();
                        break;
                    }
                    // nothing fits: give back this lane's cached buffers if
                    // a job this lane may take waits for memory (a small-job
                    // lane keeps them while only large jobs wait)
                    const bool eligible_waits =
                        std::any_of(ready.begin(), ready.end(), [&](const std::shared_ptr<Job> &x) {
                            return !small_only || x->c.n <= SMALL_LANE_MAX_QUBITS;
                        });
                    if (eligible_waits && ws.bytes()) {
                        g.unlock();
                        ws.release();
                        g.lock();
                        lane_charge[id] = 0;
                        cv.notify_all();
                        continue;
                    }
                    cv.wait(g);
                }
                if (stop) break;
            }
            int state = JS_DONE, code = 0;
            std::string msg;
            try {
                execute_plan(ctx, j->tree, j->plan, j->o, s, j->res, &ws, &j->cancel);
                j->res.counters.host_ecm_seconds = j->ecm_s;
                j->res.counters.host_plan_seconds = j->plan_s;
            } catch (const Error &e) {
                state = e.code == TUSQ_ECANCELED ? JS_CANCELLED : JS_FAILED;
                code = e.code;
                msg = e.msg;
                (void)hipStreamSynchronize(s);
            }
            running.fetch_sub(1);
            {
                std::lock_guard<std::mutex> g(mu);
                lane_charge[id] = ws.bytes();
            }
            finish(j, state, code, msg);
        }
        ws.release();
        for (hipEvent_t e : ws.window)
            if (e) (void)hipEventDestroy(e);
        (void)hipStreamDestroy(s);
    }
};

static Serving &serving(Ctx &ctx) {
    std::lock_guard<std::mutex> g(ctx.mu);
    if (!ctx.serving) ctx.serving = new Serving(ctx);
    return *ctx.serving;
}

static std::shared_ptr<Job> find_job(Serving &sv, uint64_t id) {
    auto it = sv.jobs.find(id);
    if (it == sv.jobs.end()) fail(TUSQ_EINVAL, "unknown job id");
    return it->second;
}

uint64_t serving_submit(Ctx &ctx, const Circuit &c, const tusq_opts &o) {
    Circuit cc = c;
    cc.finalize();
    const uint64_t need = job_device_bytes(cc.n, o.precision, o.shots, o.want & TUSQ_WANT_DIST);
    if (need > ctx.budget) fail(TUSQ_ENOMEM, "job needs more device memory than the budget");
    Serving &sv = serving(ctx);
    auto j = std::make_shared<Job>();
    j->c = std::move(cc);
    j->o = o;
    j->need = need;
    j->t_submit = now_seconds();
    {
        std::lock_guard<std::mutex> g(sv.mu);
        j->id = sv.next_id++;
        sv.jobs[j->id] = j;
        sv.to_plan.push_back(j);
    }
    sv.cv.notify_all();
    return j->id;
}

int serving_poll(Ctx &ctx, uint64_t id) {
    Serving &sv = serving(ctx);
    std::lock_guard<std::mutex> g(sv.mu);
    return find_job(sv, id)->state;
}

void serving_wait(Ctx &ctx, uint64_t id, Result &out) {
    Serving &sv = serving(ctx);
    std::unique_lock<std::mutex> g(sv.mu);
    auto j = find_job(sv, id);
    sv.cv.wait(g, [&] { return j->state >= JS_DONE; });
    if (j->state != JS_DONE) fail(j->err_code ? j->err_code : TUSQ_EINVAL, j->err_msg);
    out = std::move(j->res);
    j->res = Result();
}

void serving_cancel(Ctx &ctx, uint64_t id) {
    Serving &sv = serving(ctx);
    std::shared_ptr<Job> j;
    {
        std::lock_guard<std::mutex> g(sv.mu);
        j = find_job(sv, id);
        j->cancel.store(true);
        auto it = std::find(sv.ready.begin(), sv.ready.end(), j);
        if (it != sv.ready.end()) sv.ready.erase(it);
        else return;  // still planning (the planner drops it) or running (stops at a chunk)
    }
    sv.finish(j, JS_CANCELLED, TUSQ_ECANCELED, "job cancelled");
}

void serving_times(Ctx &ctx, uint64_t id, double *submitted, double *admitted, double *finished) {
    Serving &sv = serving(ctx);
    std::lock_guard<std::mutex> g(sv.mu);
    auto j = find_job(sv, id);
    if (j->state < JS_DONE) fail(TUSQ_EBUSY, "job not finished");
    *submitted = j->t_submit;
    *admitted = j->t_admit;
    *finished = j->t_finish;
}

void serving_shutdown(Ctx &ctx) {
    Serving *sv = nullptr;
    {
        std::lock_guard<std::mutex> g(ctx.mu);
        sv = ctx.serving;
        ctx.serving = nullptr;
    }
    delete sv;
}

}  // namespace tusq
