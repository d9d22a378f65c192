// exec.hip -- runs a plan on one GPU: uploads the fused ops, walks the step
// list launching sweeps / leaf reductions / samplers on the caller's stream,
// and (complex64 mode) watches the FP64 leaf norm, recomputing a leaf from
// |0...0> in complex128 when its drift passes the bound.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "exec.hpp"
#include "kernels.hpp"

namespace tusq {

void hip_check(hipError_t e, const char *what) {
    if (e != hipSuccess)
        fail(TUSQ_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

DevBuf::~DevBuf() { release(); }
void DevBuf::release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
}
void DevBuf::alloc(size_t b) {
    release();
    if (!b) return;
    hip_check(hipMalloc(&p, b), "hipMalloc");
    bytes = b;
}
void DevBuf::ensure(size_t b) {
    if (b <= bytes && p) return;
    alloc(b);
}

uint64_t Workspace::bytes() const {
    uint64_t b = 0;
    for (const DevBuf *d : {&psi, &psi128, &acc, &csum, &prefix, &norms, &samples, &dops, &mats,
                            &mats128, &prog, &ckpt})
        b += d->bytes;
    return b;
}
void Workspace::release() {
    for (DevBuf *d : {&psi, &psi128, &acc, &csum, &prefix, &norms, &samples, &dops, &mats, &mats128,
                      &prog, &ckpt})
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

    std::vector<DOp> dops;
    to_device_ops(plan, dops);
    dops_b.ensure(std::max<size_t>(dops.size(), 1) * sizeof(DOp));
    if (!dops.empty())
        hip_check(hipMemcpyAsync(dops_b.p, dops.data(), dops.size() * sizeof(DOp), hipMemcpyHostToDevice, s),
                  "upload ops");
    prog_b.ensure(std::max<size_t>(plan.prog.size(), 1) * sizeof(Instr2));
    if (!plan.prog.empty())
        hip_check(hipMemcpyAsync(prog_b.p, plan.prog.data(), plan.prog.size() * sizeof(Instr2),
                                 hipMemcpyHostToDevice, s), "upload programs");
    std::vector<double2> m128(plan.mats.size());
    for (size_t i = 0; i < plan.mats.size(); ++i) m128[i] = double2{plan.mats[i].real(), plan.mats[i].imag()};
    std::vector<float2> m64;
    if (c64) {
        m64.resize(plan.mats.size());
        for (size_t i = 0; i < plan.mats.size(); ++i)
            m64[i] = float2{static_cast<float>(plan.mats[i].real()), static_cast<float>(plan.mats[i].imag())};
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
            return launch_sweep_pp<V>(st, n, a, prog, mat, plan.reg_qubits,
                                      static_cast<uint32_t>(ctx.cus), s);
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
    std::vector<double> hnorm(1);

    const double t0 = now_seconds();
    hip_check(hipStreamSynchronize(s), "sync");
    for (size_t si = 0; si < plan.steps.size(); ++si) {
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
                hip_check(hipMemcpyAsync(hnorm.data(), nrm, 8, hipMemcpyDeviceToHost, s), "norm readback");
                hip_check(hipStreamSynchronize(s), "sync");
                const double drift = std::fabs(hnorm[0] - 1.0);
                ct.max_norm_drift = std::max(ct.max_norm_drift, drift);
                const bool by_count = o.max_passes_between_recompute &&
                                      passes_since_exact > o.max_passes_between_recompute;
                if (drift > o.drift_bound || by_count) {
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
    if (want_dist) {
        res.dist.resize(N);
        hip_check(hipMemcpy(res.dist.data(), acc.p, N * 8, hipMemcpyDeviceToHost), "dist readback");
    }
    if (want_samples && total_shots) {
        res.samples.resize(total_shots);
        hip_check(hipMemcpy(res.samples.data(), samples.p, total_shots * 8, hipMemcpyDeviceToHost),
                  "samples readback");
    }
    res.norms.resize(le - lb);
    if (le > lb)
        hip_check(hipMemcpy(res.norms.data(), norms.p, (le - lb) * 8, hipMemcpyDeviceToHost), "norms readback");
    for (double v : res.norms) ct.max_norm_drift = std::max(ct.max_norm_drift, std::fabs(v - 1.0));
}

}  // namespace

Ctx::Ctx(int dev, uint64_t budget_) : device(dev) {
    int count = 0;
    hip_check(hipGetDeviceCount(&count), "hipGetDeviceCount");
    if (dev < 0 || dev >= count) fail(TUSQ_EINVAL, "no such device");
    hip_check(hipSetDevice(dev), "hipSetDevice");
    hip_check(sweep_kernel_setup(), "kernel setup");
    hip_check(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "attr");
    size_t fr = 0, tot = 0;
    hip_check(hipMemGetInfo(&fr, &tot), "hipMemGetInfo");
    budget = budget_ ? budget_ : static_cast<uint64_t>(fr);
    hip_check(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking), "stream");
}

Ctx::~Ctx() {
    (void)hipSetDevice(device);
    for (auto e : pool) (void)hipEventDestroy(e);
    if (stream) (void)hipStreamDestroy(stream);
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

}  // namespace tusq
