// exec.hip -- runs a plan on one GPU: uploads the fused ops, walks the step
// list launching sweeps / leaf reductions / samplers on the caller's stream,
// and (complex64 mode) watches the FP64 leaf norm, recomputing a leaf from
// |0...0> in complex128 when its drift passes the bound.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>

#include "exec.hpp"
#include "kernels.hpp"
#include "rng.hpp"

namespace tusq {

void hip_check(hipError_t e, const char *what) {
    if (e != hipSuccess)
        fail(TUSQ_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

DevBuf::~DevBuf() { release(); }
void DevBuf::release() {
    if (p && owned) (void)(stream ? hipFreeAsync(p, stream) : hipFree(p));
    p = nullptr;
    bytes = 0;
    owned = true;
}
void DevBuf::alloc(size_t b) {
    release();
    if (!b) return;
    hip_check(stream ? hipMallocAsync(&p, b, stream) : hipMalloc(&p, b), "hipMalloc");
    bytes = b;
}
void DevBuf::ensure(size_t b) {
    if (b <= bytes && p) return;
    if (!owned) fail(TUSQ_ENOMEM, "internal: a borrowed device buffer is too small");
    alloc(b);
}
void DevBuf::borrow(void *q, size_t b) {
    release();
    p = q;
    bytes = b;
    owned = false;
}

// Work memory of the no-allocation run (execute_plan_static).  Every device
// the library runs on holds its own copy until the process ends; host code
// reaches it only through the address hipGetSymbolAddress gives for the
// current device (Ctx::scratch), never through this name.
static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

namespace {
std::mutex scratch_mu;
std::map<int, void *> scratch_ptrs;  // device -> address of its scratch copy

// The scratch address on device dev, which must be current; looked up once
// per device.
void *scratch_address(int dev) {
    std::lock_guard<std::mutex> g(scratch_mu);
    auto it = scratch_ptrs.find(dev);
    if (it != scratch_ptrs.end()) return it->second;
    void *ptr = nullptr;
    hip_check(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (!ptr) fail(TUSQ_EDEVICE, "static scratch has no device address");
    scratch_ptrs[dev] = ptr;
    return ptr;
}
}  // namespace

void Result::dist_copy(double *out) const {
    if (!dist.empty()) {
        std::memcpy(out, dist.data(), dist.size() * 8);
        return;
    }
    if (!dist_dev || !dist_dev->p) fail(TUSQ_EINVAL, "result holds no distribution");
    hip_check(hipSetDevice(device), "hipSetDevice");
    hip_check(hipMemcpy(out, dist_dev->p, (1ull << n) * 8, hipMemcpyDeviceToHost), "dist readback");
}

Workspace::~Workspace() {
    if (word_ctx) word_ctx->give_word(host_word);
}
double *Workspace::readback_word(Ctx &ctx) {
    if (!host_word) {
        host_word = ctx.take_word();
        if (host_word) word_ctx = &ctx;
        else host_word = &spare;
    }
    return host_word;
}

uint64_t Workspace::bytes() const {
    uint64_t b = 0;
    for (const DevBuf *d : {&psi, &psi128, &acc, &csum, &prefix, &norms, &samples, &dops, &mats,
                            &mats128, &prog, &ckpt, &mcm})
        b += d->bytes;
    return b;
}
void Workspace::set_stream(hipStream_t s) {
    for (DevBuf *d : {&psi, &psi128, &acc, &csum, &prefix, &norms, &samples, &dops, &mats, &mats128,
                      &prog, &ckpt, &mcm})
        d->stream = s;
}
void Workspace::release() {
    for (DevBuf *d : {&psi, &psi128, &acc, &csum, &prefix, &norms, &samples, &dops, &mats, &mats128,
                      &prog, &ckpt, &mcm})
        d->release();
}

uint64_t job_device_bytes(uint32_t n, uint32_t precision, uint64_t shots, bool want_dist) {
    const uint64_t N = 1ull << n;
    uint64_t b = N * (precision == TUSQ_C64 ? 8 : 16);
    if (precision == TUSQ_C64) b += N * 16;        // complex128 recompute buffer
    if (want_dist) b += N * 8;                     // FP64 accumulator
    const uint32_t lc = std::min<uint32_t>(n, 11);
    b += 2 * (N >> lc) * 8 + shots * 8 + (64ull << 20);  // chunk sums, prefix, samples, plan
    return b;
}

uint64_t checkpoint_bytes(uint32_t n, uint32_t precision, uint64_t slots) {
    return slots * ((1ull << n) * (precision == TUSQ_C64 ? 8 : 16));
}

static_assert(sizeof(Instr) == sizeof(Instr2), "program layout shared with the kernels");

namespace {

void to_device_ops(const Plan &plan, std::vector<DOp> &dops) {
    dops.resize(plan.ops.size());
    for (size_t i = 0; i < plan.ops.size(); ++i)
        dops[i] = DOp{static_cast<uint32_t>(plan.ops[i].a) | (static_cast<uint32_t>(plan.ops[i].b) << 8),
                      plan.ops[i].mat};
}

SweepArgs sweep_args(const Pass &p, bool inverse) {
    SweepArgs a{};
    a.k = p.k;
    a.low = 0;
    while (a.low < p.k && p.q[a.low] == a.low) ++a.low;
    a.nops = p.op_end - p.op_begin;
    a.op_begin = p.op_begin;
    a.inverse = inverse ? 1 : 0;
    a.fwd_begin = p.fwd_begin;
    a.fwd_end = p.fwd_end;
    a.inv_begin = p.inv_begin;
    a.inv_end = p.inv_end;
    const uint32_t *lay = p.lay[inverse ? 1 : 0];
    a.lay_in_reg = lay[0];
    a.lay_in_thr = lay[1];
    a.lay_out_reg = lay[2];
    a.lay_out_thr = lay[3];
    for (uint32_t j = 0; j < p.k; ++j) a.q[j] = static_cast<uint8_t>(p.q[j]);
    return a;
}

// Copies a plan's ops, programs and matrices (complex64 and, for the
// recompute path, complex128) into the workspace.  The host copies live in
// `st`, which must outlive the asynchronous copies (the caller synchronises
// the stream before it goes out of scope).
struct Staged {
    std::vector<DOp> dops;
    std::vector<double2> m128;
    std::vector<float2> m64;
};

void upload_plan_into(const Plan &plan, Workspace &ws, bool c64, hipStream_t s, Staged &st) {
    DevBuf &dops_b = ws.dops, &mats_b = ws.mats, &mats128_b = ws.mats128, &prog_b = ws.prog;
    std::vector<DOp> &dops = st.dops;
    to_device_ops(plan, dops);
    dops_b.ensure(std::max<size_t>(dops.size(), 1) * sizeof(DOp));
    if (!dops.empty())
        hip_check(hipMemcpyAsync(dops_b.p, dops.data(), dops.size() * sizeof(DOp), hipMemcpyHostToDevice, s),
                  "upload ops");
    prog_b.ensure(std::max<size_t>(plan.prog.size(), 1) * sizeof(Instr2));
    if (!plan.prog.empty())
        hip_check(hipMemcpyAsync(prog_b.p, plan.prog.data(), plan.prog.size() * sizeof(Instr2),
                                 hipMemcpyHostToDevice, s), "upload programs");
    std::vector<double2> &m128 = st.m128;
    m128.resize(plan.mats.size());
    for (size_t i = 0; i < plan.mats.size(); ++i) m128[i] = double2{plan.mats[i].real(), plan.mats[i].imag()};
    if (c64) {
        std::vector<float2> &m64 = st.m64;
        std::vector<float> flat;
        mats_to_c64(plan, flat);
        m64.resize(plan.mats.size());
        for (size_t i = 0; i < plan.mats.size(); ++i) m64[i] = float2{flat[2 * i], flat[2 * i + 1]};
        mats_b.ensure(std::max<size_t>(m64.size(), 1) * sizeof(float2));
        if (!m64.empty())
            hip_check(hipMemcpyAsync(mats_b.p, m64.data(), m64.size() * sizeof(float2), hipMemcpyHostToDevice, s),
                      "upload mats");
        mats128_b.ensure(std::max<size_t>(m128.size(), 1) * sizeof(double2));
        if (!m128.empty())
            hip_check(hipMemcpyAsync(mats128_b.p, m128.data(), m128.size() * sizeof(double2),
                                     hipMemcpyHostToDevice, s), "upload mats");
    } else {
        mats_b.ensure(std::max<size_t>(m128.size(), 1) * sizeof(double2));
        if (!m128.empty())
            hip_check(hipMemcpyAsync(mats_b.p, m128.data(), m128.size() * sizeof(double2),
                                     hipMemcpyHostToDevice, s), "upload mats");
    }
}

template <typename V>
void run_typed(Ctx &ctx, const Tree &t, const Plan &plan, const tusq_opts &o, hipStream_t s,
               Result &res, Workspace &ws, const std::atomic<bool> *cancel) {
    const uint32_t n = plan.n;
    const uint64_t N = 1ull << n;
    const bool c64 = std::is_same<V, float2>::value;
    const uint32_t lc = std::min<uint32_t>(n, 11);
    const uint64_t nc = N >> lc;
    uint64_t lb = o.leaf_begin, le = o.leaf_end;
    if (lb == 0 && le == 0) le = t.leaves();
    uint64_t total_shots = 0;
    for (uint64_t l = lb; l < le; ++l) total_shots += t.shots[l];
    const bool want_dist = o.want & TUSQ_WANT_DIST;
    const bool want_samples = o.want & TUSQ_WANT_SAMPLES;

    DevBuf &psi = ws.psi, &psi128 = ws.psi128, &acc = ws.acc, &csum = ws.csum, &prefix = ws.prefix,
           &norms = ws.norms, &samples = ws.samples, &dops_b = ws.dops, &mats_b = ws.mats,
           &mats128_b = ws.mats128, &prog_b = ws.prog;
    psi.ensure(N * sizeof(V));
    if (c64) psi128.ensure(N * sizeof(double2));
    if (want_dist) acc.ensure(N * 8);
    csum.ensure(nc * 8);
    prefix.ensure(nc * 8);
    norms.ensure(std::max<uint64_t>(le - lb, 1) * 8);
    if (want_samples && total_shots) samples.ensure(total_shots * 8);
    if (plan.checkpoint_slots) ws.ckpt.ensure(plan.checkpoint_slots * N * sizeof(V));
    V *ckpt = static_cast<V *>(ws.ckpt.p);

    Staged staged;
    upload_plan_into(plan, ws, c64, s, staged);
    if (want_dist) hip_check(launch_fill(static_cast<double *>(acc.p), N, 0.0, s), "fill");

    V *st = static_cast<V *>(psi.p);
    const DOp *dop = static_cast<const DOp *>(dops_b.p);
    const V *mat = static_cast<const V *>(mats_b.p);
    const Instr2 *prog = static_cast<const Instr2 *>(prog_b.p);
    // register-blocked sweeps wherever the tile spans at least R qubits
    const bool pipelined = o.sweep_kernel == 2;
    const bool one_tile_per_wg = o.sweep_kernel == 1 || o.sweep_kernel == 3;
    const uint32_t pipe_grid = static_cast<uint32_t>(ctx.cus);  // one 128-KiB workgroup per CU
    auto sweep = [&](const Pass &p, bool inverse) {
        const SweepArgs a = sweep_args(p, inverse);
        if (p.k >= plan.reg_qubits) {
            if (pipelined && plan.reg_qubits == 4 && p.k - plan.reg_qubits >= 6 &&
                (sizeof(V) << p.k) <= 64 * 1024)
                return launch_sweep_pipe<V>(st, n, a, prog, mat, pipe_grid, s);
            if (one_tile_per_wg) return launch_sweep_reg<V>(st, n, a, prog, mat, plan.reg_qubits, s);
            uint32_t cus = static_cast<uint32_t>(ctx.cus);
            if (ws.co_running && ws.co_running->load(std::memory_order_relaxed) > 1) cus -= cus / 8;
            return launch_sweep_pp<V>(st, n, a, prog, mat, plan.reg_qubits, cus, s);
        }
        return launch_sweep<V>(st, n, a, dop, mat, s);
    };

    const bool prof = o.profile != 0;
    std::vector<hipEvent_t> evs;
    auto &ct = res.counters;
    ct = plan.counters;
    ct.max_norm_drift = 0.0;
    uint64_t passes_since_exact = 0;
    uint64_t sample_off = 0;
    double *hnorm = c64 ? ws.readback_word(ctx) : nullptr;

    // queued-work windows of a serving lane: each step counts 2^n amplitudes
    // of work; at the end of a window the host waits for the one before it
    // (about 35 ms of 30-qubit sweeps)
    constexpr uint64_t WINDOW_AMPS = 1ull << 31;
    const bool windows = ws.window[0] && ws.window[1];
    uint64_t window_work = 0;
    bool window_pending[2] = {false, false};
    unsigned window_cur = 0;
    auto end_window = [&] {
        const unsigned prev = window_cur ^ 1u;
        if (window_pending[prev]) hip_check(hipEventSynchronize(ws.window[prev]), "window");
        window_pending[prev] = false;
        hip_check(hipEventRecord(ws.window[window_cur], s), "window");
        window_pending[window_cur] = true;
        window_cur = prev;
    };

    const double t0 = now_seconds();
    hip_check(hipStreamSynchronize(s), "sync");
    for (size_t si = 0; si < plan.steps.size(); ++si) {
        if (windows && (window_work += N) >= WINDOW_AMPS) {
            window_work = 0;
            end_window();
        }
        if (o.debug_fail_at_step >= 0 && static_cast<size_t>(o.debug_fail_at_step) == si)
            fail(TUSQ_EDEVICE, "injected failure at schedule step " + std::to_string(si));
        // chunk boundary: a cancelled job stops here (work already queued on
        // the stream finishes on its own)
        if (cancel && (si & 255u) == 0 && cancel->load(std::memory_order_relaxed)) {
            (void)hipStreamSynchronize(s);
            fail(TUSQ_ECANCELED, "job cancelled");
        }
        const Step &sp = plan.steps[si];
        switch (sp.kind) {
        case ST_RESET:
            hip_check(launch_reset<V>(st, n, s), "reset");
            passes_since_exact = 0;
            break;
        case ST_SAVE:
            hip_check(hipMemcpyAsync(ckpt + sp.id * N, st, N * sizeof(V), hipMemcpyDeviceToDevice, s),
                      "checkpoint save");
            break;
        case ST_RESTORE:
            hip_check(hipMemcpyAsync(st, ckpt + sp.id * N, N * sizeof(V), hipMemcpyDeviceToDevice, s),
                      "checkpoint restore");
            break;
        case ST_FWD:
        case ST_INV: {
            const Pass &pp = plan.passes[sp.id];
            if (prof) {
                hipEvent_t e0 = ctx.event(), e1 = ctx.event();
                hip_check(hipEventRecord(e0, s), "event");
                hip_check(sweep(pp, sp.kind == ST_INV), "sweep");
                hip_check(hipEventRecord(e1, s), "event");
                evs.push_back(e0);
                evs.push_back(e1);
            } else {
                hip_check(sweep(pp, sp.kind == ST_INV), "sweep");
            }
            ++passes_since_exact;
            break;
        }
        case ST_LEAF: {
            const uint64_t l = sp.id;
            const uint64_t li = l - lb;
            double *nrm = static_cast<double *>(norms.p) + li;
            if (c64) {
                // drift control: FP64 norm of the complex64 state first
                hip_check(launch_leaf<V>(st, n, lc, nullptr, 0.0, static_cast<double *>(csum.p),
                                         static_cast<double *>(prefix.p), nrm, s), "norm");
                hip_check(hipMemcpyAsync(hnorm, nrm, 8, hipMemcpyDeviceToHost, s), "norm readback");
                hip_check(hipStreamSynchronize(s), "sync");
                const double drift = std::fabs(hnorm[0] - 1.0);
                ct.max_norm_drift = std::max(ct.max_norm_drift, drift);
                const bool by_count = o.max_passes_between_recompute &&
                                      passes_since_exact > o.max_passes_between_recompute;
                if (drift > o.drift_bound || by_count) {
                    if (plan.path_off.size() < li + 2)
                        fail(TUSQ_EINVAL, "a complex128 recompute came due on a plan built without recompute paths");
                    double2 *s128 = static_cast<double2 *>(psi128.p);
                    hip_check(launch_reset<double2>(s128, n, s), "reset128");
                    const double2 *mat128 = static_cast<const double2 *>(mats128_b.p);
                    for (uint64_t k = plan.path_off[li]; k < plan.path_off[li + 1]; ++k) {
                        const Pass &pp = plan.passes[plan.path[k]];
                        const SweepArgs a = sweep_args(pp, false);
                        // the sweep programs are precision independent
                        hip_check(pp.k >= plan.reg_qubits
                                      ? launch_sweep_pp<double2>(s128, n, a, prog, mat128,
                                                                 plan.reg_qubits,
                                                                 static_cast<uint32_t>(ctx.cus), s)
                                      : launch_sweep<double2>(s128, n, a, dop, mat128, s),
                                  "recompute sweep");
                    }
                    hip_check(launch_to_c64(s128, reinterpret_cast<float2 *>(st), n, s), "convert");
                    ct.recomputes++;
                    ct.recompute_passes += plan.path_off[li + 1] - plan.path_off[li];
                    passes_since_exact = 0;
                }
            }
            hip_check(launch_leaf<V>(st, n, lc, want_dist ? static_cast<double *>(acc.p) : nullptr,
                                     static_cast<double>(t.wnum[l]) / static_cast<double>(t.wden[l]),
                                     static_cast<double *>(csum.p), static_cast<double *>(prefix.p), nrm, s),
                      "leaf");
            if (want_samples && t.shots[l])
                hip_check(launch_sample<V>(st, n, lc, static_cast<const double *>(prefix.p), nrm, o.seed,
                                           static_cast<uint32_t>(l), t.shots[l],
                                           static_cast<uint64_t *>(samples.p) + sample_off, s),
                          "sample");
            sample_off += t.shots[l];
            break;
        }
        }
    }
    hip_check(hipStreamSynchronize(s), "sync");
    ct.device_seconds = now_seconds() - t0;
    if (prof) {
        double tot = 0.0;
        for (size_t i = 0; i < evs.size(); i += 2) {
            float ms = 0.f;
            hip_check(hipEventElapsedTime(&ms, evs[i], evs[i + 1]), "elapsed");
            tot += ms * 1e-3;
        }
        ct.pass_seconds = tot;
        ct.pass_events = evs.size() / 2;
        ctx.recycle(evs);
    }
    res.n = n;
    res.device = ctx.device;
    if (want_dist && !ws.device_outputs && ws.co_running) {
        // a serving lane keeps its buffers for the next job: the
        // distribution goes to the host on the lane's own stream
        res.dist.resize(N);
        hip_check(hipMemcpyAsync(res.dist.data(), acc.p, N * 8, hipMemcpyDeviceToHost, s), "dist readback");
    } else if (want_dist && !ws.device_outputs) {
        // the accumulator becomes the result's: the distribution stays in
        // device memory until the caller asks for it
        res.dist.clear();
        res.dist_dev = std::make_shared<DevBuf>();
        res.dist_dev->p = acc.p;
        res.dist_dev->bytes = acc.bytes;
        acc.p = nullptr;
        acc.bytes = 0;
    }
    if (want_samples && total_shots && !ws.device_outputs) {
        res.samples.resize(total_shots);
        hip_check(hipMemcpyAsync(res.samples.data(), samples.p, total_shots * 8, hipMemcpyDeviceToHost, s),
                  "samples readback");
    }
    res.norms.resize(le - lb);
    if (le > lb)
        hip_check(hipMemcpyAsync(res.norms.data(), norms.p, (le - lb) * 8, hipMemcpyDeviceToHost, s),
                  "norms readback");
    // readbacks on the job's own stream (a blocking copy would go through
    // the null stream, behind other jobs' work)
    hip_check(hipStreamSynchronize(s), "sync");
    for (double v : res.norms) ct.max_norm_drift = std::max(ct.max_norm_drift, std::fabs(v - 1.0));
}


// ---------------------------------------------------------------------------
// DFTT+Caching over stages separated by measurement layers (Sec. III-B.2).
// The walk is the oracle's: plain DFTT inside a stage; at the end of a stage
// path (a pre-measurement node) the layer's outcome weights come back to the
// host, every shot of the node draws its outcome (stream 3, counter (shot,
// leaf, layer)), and each outcome with shots is walked in turn; the node is
// pushed on the cache if its layer is one of the K closest to the leaves,
// else it is recomputed from the root when needed again.
template <typename V>
struct McmWalk {
    Ctx &ctx;
    const Tree &t;
    const McmPlan &mp;
    const Plan &plan;
    const tusq_opts &o;
    hipStream_t s;
    Result &res;
    uint32_t n;
    uint64_t N;
    uint32_t lc;
    V *psi;
    V *slots;              // K cached states
    double *partial, *Pdev;
    const DOp *dop;
    const V *mat;
    const Instr2 *prog;
    double *acc, *csum, *prefix, *norms;
    uint64_t *samples;
    bool want_dist, want_samples, prof;
    std::vector<hipEvent_t> evs;
    std::vector<uint32_t> rep, out;              // per stage / layer on the current path
    std::vector<std::array<double, 256>> P;      // weights of each layer's node on the path
    std::vector<uint64_t> sbase;                 // draws taken per leaf
    uint64_t sample_off = 0, vleaf = 0;
    tusq_counters ct{};

    struct Grp {
        std::vector<uint64_t> leaf, off;
        std::vector<uint32_t> shot;
    };

    McmWalk(Ctx &c, const Tree &tr, const McmPlan &m, const tusq_opts &op, hipStream_t st, Result &r)
        : ctx(c), t(tr), mp(m), plan(m.plan), o(op), s(st), res(r) {}

    bool cached(uint32_t k) const { return mp.K > 0 && k + mp.K >= mp.M; }
    V *slot(uint32_t k) { return slots + static_cast<uint64_t>(k + mp.K - mp.M) * N; }
    uint32_t path_of(uint64_t l, uint32_t st) const { return mp.leaf_path[(l - mp.lb) * (mp.M + 1) + st]; }
    uint64_t len(uint32_t id) const { return mp.paths[id].code.size(); }

    hipError_t sweep(const Pass &p, bool inverse) {
        const SweepArgs a = sweep_args(p, inverse);
        if (p.k >= plan.reg_qubits) {
            if (o.sweep_kernel == 1 || o.sweep_kernel == 3)
                return launch_sweep_reg<V>(psi, n, a, prog, mat, plan.reg_qubits, s);
            return launch_sweep_pp<V>(psi, n, a, prog, mat, plan.reg_qubits,
                                      static_cast<uint32_t>(ctx.cus), s);
        }
        return launch_sweep<V>(psi, n, a, dop, mat, s);
    }
    void run_pass(uint32_t pi, bool inverse) {
        const Pass &pp = plan.passes[pi];
        if (prof) {
            hipEvent_t e0 = ctx.event(), e1 = ctx.event();
            hip_check(hipEventRecord(e0, s), "event");
            hip_check(sweep(pp, inverse), "sweep");
            hip_check(hipEventRecord(e1, s), "event");
            evs.push_back(e0);
            evs.push_back(e1);
        } else {
            hip_check(sweep(pp, inverse), "sweep");
        }
        ct.sweep_bytes += 2ull * N * sizeof(V);
        ct.sweep_flops += plan_pass_flops(plan, pi);
    }
    // tokens [from, to) of a path forward, or [to, from) undone (from > to);
    // both ends are cut points of the path
    void fwd(uint32_t id, uint64_t from, uint64_t to) {
        const McmPath &p = mp.paths[id];
        for (size_t i = 0; i < p.seg.size(); ++i) {
            if (p.cut[i] < from || p.cut[i + 1] > to) continue;
            const McmSeg &sg = p.seg[i];
            for (uint32_t q = sg.p0; q < sg.p1; ++q) run_pass(q, false);
            ct.passes_fwd += sg.p1 - sg.p0;
            ct.fwd_gates += sg.gates;
            ct.fwd_paulis += sg.paulis;
            ct.paper_ops += sg.ops;
        }
    }
    void inv(uint32_t id, uint64_t from, uint64_t to) {
        const McmPath &p = mp.paths[id];
        for (size_t i = p.seg.size(); i > 0; --i) {
            if (p.cut[i - 1] < to || p.cut[i] > from) continue;
            const McmSeg &sg = p.seg[i - 1];
            for (uint32_t q = sg.p1; q > sg.p0; --q) run_pass(q - 1, true);
            ct.passes_inv += sg.p1 - sg.p0;
            ct.inv_gates += sg.gates;
            ct.inv_paulis += sg.paulis;
            ct.paper_ops += sg.ops;
        }
    }
    void check_cut(uint32_t id, uint64_t d) const {
        const auto &c = mp.paths[id].cut;
        if (!std::binary_search(c.begin(), c.end(), d))
            fail(TUSQ_EINVAL, "internal: a transition stops inside a fused segment");
    }
    MeasArgs layer_args(uint32_t k) const {
        MeasArgs a{};
        a.m = mp.layers[k].m;
        for (uint32_t b = 0; b < a.m; ++b) a.q[b] = static_cast<uint8_t>(mp.layers[k].q[b]);
        return a;
    }
    void weights(uint32_t k) {
        const MeasArgs a = layer_args(k);
        hip_check(launch_mcm_probs<V>(psi, n, a, partial, Pdev, s), "measurement weights");
        hip_check(hipMemcpyAsync(P[k].data(), Pdev, sizeof(double) << a.m, hipMemcpyDeviceToHost, s),
                  "weights readback");
        hip_check(hipStreamSynchronize(s), "sync");
    }
    // measurement edge of layer k with outcome o, reading src (psi or a slot)
    void edge(uint32_t k, uint32_t oc, const V *src) {
        const MeasArgs a = layer_args(k);
        const uint32_t want = mp.layers[k].reset ? 0u : oc;
        hip_check(launch_mcm_apply<V>(src, psi, n, a, oc, want, 1.0 / std::sqrt(P[k][oc]), s),
                  "measurement edge");
        ct.mcm_edges++;
        ct.paper_ops++;
    }
    void reach_root(uint32_t st) {
        if (st == 0) {
            hip_check(launch_reset<V>(psi, n, s), "reset");
            ct.resets++;
            return;
        }
        reach_pre(st - 1);
        edge(st - 1, out[st - 1], psi);
    }
    void reach_pre(uint32_t k) {
        if (cached(k)) {
            hip_check(hipMemcpyAsync(psi, slot(k), N * sizeof(V), hipMemcpyDeviceToDevice, s), "fetch");
            ct.checkpoint_restores++;
            return;
        }
        reach_root(k);
        fwd(rep[k], 0, len(rep[k]));
    }
    void final_leaf(uint64_t l, uint64_t c) {
        double *nrm = norms + vleaf;
        hip_check(launch_leaf<V>(psi, n, lc, want_dist ? acc : nullptr,
                                 static_cast<double>(c) / static_cast<double>(t.S), csum, prefix, nrm, s),
                  "leaf");
        if (want_samples && c)
            hip_check(launch_sample<V>(psi, n, lc, prefix, nrm, o.seed, static_cast<uint32_t>(l), c,
                                       samples + sample_off, s, sbase[l - mp.lb]),
                      "sample");
        sample_off += c;
        sbase[l - mp.lb] += c;
        ++vleaf;
        ct.leaves++;
        ct.leaf_sweeps++;
        ct.draws += c;
    }
    static uint32_t pick(const double *Pw, uint32_t no, double u) {
        double T = 0.0;
        for (uint32_t q = 0; q < no; ++q) T = T + Pw[q];
        const double x = u * T;
        double C = 0.0;
        for (uint32_t q = 0; q < no; ++q) {
            C = C + Pw[q];
            if (x < C) return q;
        }
        uint32_t q = no - 1;
        while (q > 0 && Pw[q] == 0.0) --q;
        return q;
    }
    void walk(uint32_t st, const Grp &g) {
        const bool naive = mp.K == 0;
        size_t i = 0, prev = SIZE_MAX;
        bool valid = true;
        while (i < g.leaf.size()) {
            const uint32_t id = path_of(g.leaf[i], st);
            size_t j = i + 1;
            while (j < g.leaf.size() && path_of(g.leaf[j], st) == id) ++j;
            const uint64_t L = len(id);
            if (prev != SIZE_MAX) {
                const uint32_t pid = path_of(g.leaf[prev], st);
                const auto &u = mp.paths[pid].code, &v = mp.paths[id].code;
                uint64_t d = 0;
                while (d < u.size() && d < v.size() && u[d] == v[d]) ++d;
                check_cut(pid, d);
                check_cut(id, d);
                if (valid && !naive) {
                    inv(pid, u.size(), d);
                } else {
                    reach_root(st);
                    fwd(id, 0, d);
                }
                fwd(id, d, L);
            } else {
                fwd(id, 0, L);
            }
            if (st == mp.M) {
                if (j != i + 1) fail(TUSQ_EINVAL, "internal: two leaves with one final path");
                final_leaf(g.leaf[i], g.off[i + 1] - g.off[i]);
                valid = !naive;
            } else {
                rep[st] = id;
                weights(st);
                const uint32_t no = 1u << mp.layers[st].m;
                std::vector<uint32_t> oc(g.off[j] - g.off[i]);
                std::vector<uint64_t> cnt(no, 0);
                for (size_t e = i; e < j; ++e)
                    for (uint64_t x = g.off[e]; x < g.off[e + 1]; ++x) {
                        const Pair64 r = philox_pair(o.seed, g.shot[x], static_cast<uint32_t>(g.leaf[e]),
                                                     st, STREAM_OUTCOMES);
                        const uint32_t q = pick(P[st].data(), no, static_cast<double>(r.lo >> 11) * 0x1p-53);
                        oc[x - g.off[i]] = q;
                        cnt[q]++;
                    }
                const bool cch = cached(st);
                if (cch) {
                    hip_check(hipMemcpyAsync(slot(st), psi, N * sizeof(V), hipMemcpyDeviceToDevice, s),
                              "cache push");
                    ct.checkpoint_saves++;
                }
                bool first = true;
                for (uint32_t q = 0; q < no; ++q) {
                    if (!cnt[q]) continue;
                    Grp h;
                    h.off.push_back(0);
                    for (size_t e = i; e < j; ++e) {
                        const size_t y0 = h.shot.size();
                        for (uint64_t x = g.off[e]; x < g.off[e + 1]; ++x)
                            if (oc[x - g.off[i]] == q) h.shot.push_back(g.shot[x]);
                        if (h.shot.size() > y0) {
                            h.leaf.push_back(g.leaf[e]);
                            h.off.push_back(h.shot.size());
                        }
                    }
                    out[st] = q;
                    if (first) {
                        edge(st, q, psi);
                    } else if (cch) {
                        // a fetch of the cached node fused with the edge
                        ct.checkpoint_restores++;
                        edge(st, q, slot(st));
                    } else {
                        reach_pre(st);
                        edge(st, q, psi);
                    }
                    walk(st + 1, h);
                    first = false;
                }
                if (cch) {
                    hip_check(hipMemcpyAsync(psi, slot(st), N * sizeof(V), hipMemcpyDeviceToDevice, s),
                              "fetch");
                    ct.checkpoint_restores++;
                    valid = true;
                } else {
                    valid = false;
                }
            }
            prev = i;
            i = j;
        }
    }

    void run() {
        n = plan.n;
        N = 1ull << n;
        lc = std::min<uint32_t>(n, 11);
        const uint64_t nc = N >> lc;
        const bool c64 = std::is_same<V, float2>::value;
        want_dist = o.want & TUSQ_WANT_DIST;
        want_samples = o.want & TUSQ_WANT_SAMPLES;
        prof = o.profile != 0;
        uint64_t total = 0;
        for (uint64_t l = mp.lb; l < mp.le; ++l) total += t.shots[l];
        Workspace ws;
        ws.psi.ensure(N * sizeof(V));
        if (want_dist) ws.acc.ensure(N * 8);
        ws.csum.ensure(nc * 8);
        ws.prefix.ensure(nc * 8);
        ws.norms.ensure(std::max<uint64_t>(total, 1) * 8);  // final leaves <= shots
        if (want_samples && total) ws.samples.ensure(total * 8);
        if (mp.K) ws.ckpt.ensure(static_cast<uint64_t>(mp.K) * N * sizeof(V));
        ws.mcm.ensure((512ull * 256 + 256) * 8);
        Staged staged;
        upload_plan_into(plan, ws, c64, s, staged);
        psi = static_cast<V *>(ws.psi.p);
        slots = static_cast<V *>(ws.ckpt.p);
        partial = static_cast<double *>(ws.mcm.p);
        Pdev = partial + 512ull * 256;
        dop = static_cast<const DOp *>(ws.dops.p);
        mat = static_cast<const V *>(ws.mats.p);
        prog = static_cast<const Instr2 *>(ws.prog.p);
        acc = static_cast<double *>(ws.acc.p);
        csum = static_cast<double *>(ws.csum.p);
        prefix = static_cast<double *>(ws.prefix.p);
        norms = static_cast<double *>(ws.norms.p);
        samples = static_cast<uint64_t *>(ws.samples.p);
        rep.assign(mp.M + 1, 0);
        out.assign(mp.M + 1, 0);
        P.assign(mp.M + 1, {});
        sbase.assign(mp.le - mp.lb, 0);
        if (want_dist) hip_check(launch_fill(acc, N, 0.0, s), "fill");
        const double t0 = now_seconds();
        hip_check(hipStreamSynchronize(s), "sync");
        if (mp.le > mp.lb) {
            Grp g;
            g.off.push_back(0);
            for (uint64_t l = mp.lb; l < mp.le; ++l) {
                g.leaf.push_back(l);
                for (uint64_t k = 0; k < t.shots[l]; ++k) g.shot.push_back(static_cast<uint32_t>(k));
                g.off.push_back(g.shot.size());
            }
            hip_check(launch_reset<V>(psi, n, s), "reset");
            ct.resets++;
            walk(0, g);
        }
        hip_check(hipStreamSynchronize(s), "sync");
        ct.device_seconds = now_seconds() - t0;
        if (prof) {
            double tot = 0.0;
            for (size_t k = 0; k < evs.size(); k += 2) {
                float ms = 0.f;
                hip_check(hipEventElapsedTime(&ms, evs[k], evs[k + 1]), "elapsed");
                tot += ms * 1e-3;
            }
            ct.pass_seconds = tot;
            ct.pass_events = evs.size() / 2;
            ctx.recycle(evs);
        }
        res.n = n;
        if (want_dist) {
            res.dist.resize(N);
            hip_check(hipMemcpy(res.dist.data(), acc, N * 8, hipMemcpyDeviceToHost), "dist readback");
        }
        if (want_samples && total) {
            res.samples.resize(total);
            hip_check(hipMemcpy(res.samples.data(), samples, total * 8, hipMemcpyDeviceToHost),
                      "samples readback");
        }
        res.norms.resize(vleaf);
        if (vleaf)
            hip_check(hipMemcpy(res.norms.data(), norms, vleaf * 8, hipMemcpyDeviceToHost), "norms readback");
        for (double v : res.norms) ct.max_norm_drift = std::max(ct.max_norm_drift, std::fabs(v - 1.0));
        res.counters = ct;
    }
};

}  // namespace

Ctx::Ctx(int dev, uint64_t budget_) : device(dev) {
    int count = 0;
    hip_check(hipGetDeviceCount(&count), "hipGetDeviceCount");
    if (dev < 0 || dev >= count) fail(TUSQ_EINVAL, "no such device");
    hip_check(hipSetDevice(dev), "hipSetDevice");
    hip_check(sweep_kernel_setup(), "kernel setup");
    scratch = scratch_address(dev);
    hip_check(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "attr");
    size_t fr = 0, tot = 0;
    hip_check(hipMemGetInfo(&fr, &tot), "hipMemGetInfo");
    budget = budget_ ? budget_ : static_cast<uint64_t>(fr);
    hip_check(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking), "stream");
    // one word per 64 bytes
    const hipError_t e = hipHostMalloc(reinterpret_cast<void **>(&host_words), HOST_WORDS * 64, hipHostMallocDefault);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(stream);  // the destructor does not run for a throwing constructor
        hip_check(e, "hipHostMalloc");
    }
    for (uint32_t i = HOST_WORDS; i-- > 0;) free_words.push_back(i);
}

Ctx::~Ctx() {
    (void)hipSetDevice(device);
    if (host_words) (void)hipHostFree(host_words);
    batch_cache_free(batch);
    for (auto e : pool) (void)hipEventDestroy(e);
    if (stream) (void)hipStreamDestroy(stream);
}

double *Ctx::take_word() {
    std::lock_guard<std::mutex> g(mu);
    if (free_words.empty()) return nullptr;
    const uint32_t i = free_words.back();
    free_words.pop_back();
    return host_words + 8 * i;
}

void Ctx::give_word(double *w) {
    std::lock_guard<std::mutex> g(mu);
    free_words.push_back(static_cast<uint32_t>((w - host_words) / 8));
}

hipEvent_t Ctx::event() {
    std::lock_guard<std::mutex> g(mu);
    if (!pool.empty()) {
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    hipEvent_t e;
    hip_check(hipEventCreate(&e), "hipEventCreate");
    return e;
}

void Ctx::recycle(std::vector<hipEvent_t> &evs) {
    std::lock_guard<std::mutex> g(mu);
    pool.insert(pool.end(), evs.begin(), evs.end());
    evs.clear();
}

uint64_t mcm_bytes(uint32_t n, uint32_t precision, uint32_t K) {
    return static_cast<uint64_t>(K) * ((1ull << n) * (precision == TUSQ_C64 ? 8 : 16)) +
           (512ull * 256 + 256) * 8;
}

void execute_mcm(Ctx &ctx, const Tree &t, const McmPlan &mp, const tusq_opts &o, hipStream_t s,
                 Result &res) {
    hip_check(hipSetDevice(ctx.device), "hipSetDevice");
    if (!s) s = ctx.stream;
    if (mp.plan.n > 34) fail(TUSQ_EUNSUPPORTED, "more than 34 qubits");
    if (o.precision == TUSQ_C64) McmWalk<float2>(ctx, t, mp, o, s, res).run();
    else if (o.precision == TUSQ_C128) McmWalk<double2>(ctx, t, mp, o, s, res).run();
    else fail(TUSQ_EINVAL, "unknown precision");
}

void execute_plan(Ctx &ctx, const Tree &t, const Plan &plan, const tusq_opts &o, hipStream_t s,
                  Result &res, Workspace *ws, const std::atomic<bool> *cancel) {
    hip_check(hipSetDevice(ctx.device), "hipSetDevice");
    if (!s) s = ctx.stream;
    if (plan.n > 34) fail(TUSQ_EUNSUPPORTED, "more than 34 qubits");
    Workspace local;
    Workspace &w = ws ? *ws : local;
    if (o.precision == TUSQ_C64) run_typed<float2>(ctx, t, plan, o, s, res, w, cancel);
    else if (o.precision == TUSQ_C128) run_typed<double2>(ctx, t, plan, o, s, res, w, cancel);
    else fail(TUSQ_EINVAL, "unknown precision");
}

void execute_plan_static(Ctx &ctx, const Tree &t, const Plan &plan, const tusq_opts &o,
                         hipStream_t s, Result &res, double *dist, uint64_t *samples,
                         uint64_t samples_len) {
    hip_check(hipSetDevice(ctx.device), "hipSetDevice");
    if (!s) s = ctx.stream;
    if (!ctx.scratch) fail(TUSQ_EDEVICE, "static scratch not set up");
    const uint32_t n = plan.n;
    const uint64_t N = 1ull << n;
    const bool c64 = o.precision == TUSQ_C64;
    const uint64_t B = c64 ? sizeof(float2) : sizeof(double2);
    uint64_t lb = o.leaf_begin, le = o.leaf_end;
    if (lb == 0 && le == 0) le = t.leaves();
    uint64_t total_shots = 0;
    for (uint64_t l = lb; l < le; ++l) total_shots += t.shots[l];
    const bool want_dist = o.want & TUSQ_WANT_DIST;
    const bool want_samples = (o.want & TUSQ_WANT_SAMPLES) && total_shots;
    if (want_dist && !dist) fail(TUSQ_EINVAL, "TUSQ_WANT_DIST needs a device distribution buffer");
    if (want_samples && (!samples || samples_len < total_shots))
        fail(TUSQ_EINVAL, "the samples buffer holds " + std::to_string(samples_len) + " values, the job draws " +
                              std::to_string(total_shots));
    const uint32_t lc = std::min<uint32_t>(n, 11);
    const uint64_t nc = N >> lc;
    // the work buffers, each on a 256-byte boundary, in the order they are
    // carved; sizes as run_typed and upload_plan_into ask for them
    const uint64_t sizes[] = {
        N * B,                                                      // psi
        c64 ? N * sizeof(double2) : 0,                              // psi128
        nc * 8,                                                     // csum
        nc * 8,                                                     // prefix
        std::max<uint64_t>(le - lb, 1) * 8,                         // norms
        std::max<uint64_t>(plan.ops.size(), 1) * sizeof(DOp),       // dops
        std::max<uint64_t>(plan.mats.size(), 1) * B,                // mats
        c64 ? std::max<uint64_t>(plan.mats.size(), 1) * sizeof(double2) : 0,  // mats128
        std::max<uint64_t>(plan.prog.size(), 1) * sizeof(Instr2),   // prog
        plan.checkpoint_slots * N * B,                              // ckpt
    };
    uint64_t off[10], total = 0;
    for (int i = 0; i < 10; ++i) {
        off[i] = total;
        total += (sizes[i] + 255) & ~255ull;
    }
    if (total > STATIC_SCRATCH_BYTES)
        fail(TUSQ_ENOMEM, "the job needs " + std::to_string(total) + " bytes of work memory; the static scratch holds " +
                              std::to_string(STATIC_SCRATCH_BYTES));
    unsigned char *base = static_cast<unsigned char *>(ctx.scratch);
    Workspace ws;
    DevBuf *bufs[] = {&ws.psi, &ws.psi128, &ws.csum, &ws.prefix, &ws.norms,
                      &ws.dops, &ws.mats, &ws.mats128, &ws.prog, &ws.ckpt};
    for (int i = 0; i < 10; ++i)
        if (sizes[i]) bufs[i]->borrow(base + off[i], sizes[i]);
    if (want_dist) ws.acc.borrow(dist, N * 8);
    if (want_samples) ws.samples.borrow(samples, samples_len * 8);
    ws.device_outputs = true;
    double norm_word = 0.0;  // pageable: this run allocates nothing
    ws.host_word = &norm_word;
    tusq_opts oo = o;
    oo.profile = 0;  // no event pool growth
    if (c64) run_typed<float2>(ctx, t, plan, oo, s, res, ws, nullptr);
    else if (o.precision == TUSQ_C128) run_typed<double2>(ctx, t, plan, oo, s, res, ws, nullptr);
    else fail(TUSQ_EINVAL, "unknown precision");
}

}  // namespace tusq
