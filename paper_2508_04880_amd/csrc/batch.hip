// batch.hip -- many small independent jobs in one persistent launch.
//
// Every job gets its own tree (host ECM) and its leaves are split into work
// units (job, leaf range); a unit starts from |0...0> at its first leaf and
// walks the rest of its range depth first (TUSQ Sec. III-B; independent
// sub-trees walked in parallel as in its Fig. 6E).  One persistent grid of
// workgroups pulls units from a device queue (largest first).  A state that
// fits in LDS stays there for the whole unit; a larger one (up to 16 qubits)
// lives in a per-workgroup global slot and each fused sweep runs over its
// tiles.  Each unit accumulates w |psi|^2 into its own FP64 partial in leaf
// order and draws its leaves' shots; a combine kernel sums the partials of a
// job in unit order, so results are bitwise reproducible.  The three
// launches (queue reset, persistent walk, combine) are captured in a
// hipGraph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <numeric>
#include <thread>

#include "kernels.hpp"
#include "rng.hpp"
#include "serve.hpp"

namespace tusq {

// fused multiply-add in the precision of the operands (the double builtin
// would promote complex64 arithmetic to FP64)
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }


struct BUnit {
    uint32_t job, n, resident, k;
    uint32_t step_begin, step_end;
    uint64_t partial_off;   // doubles
    uint64_t sample_base;   // job's first sample
    uint64_t seed;
    double work;            // estimated cost (for ordering)
};
struct BStep {
    uint32_t kind;  // 0 reset, 1 forward sweep, 2 undo sweep, 3 leaf
    uint32_t arg;   // sweep index or leaf record
};
struct BPass {
    uint32_t k, low, op_begin, op_end;
    uint8_t q[16];
};
struct BLeaf {
    double w;
    uint64_t shots;
    uint64_t sample_off;  // within the job
    uint32_t leaf;        // leaf index in the job's tree (RNG counter)
    uint32_t pad;
};

// acc + a * b as four fused multiply-adds
template <typename V>
__device__ __forceinline__ V bfma(V acc, V a, V b) {
    acc.x = fma_t(a.x, b.x, acc.x);
    acc.x = fma_t(-a.y, b.y, acc.x);
    acc.y = fma_t(a.x, b.y, acc.y);
    acc.y = fma_t(a.y, b.x, acc.y);
    return acc;
}

__device__ __forceinline__ uint32_t ins0(uint32_t p, uint32_t bit) {
    return ((p >> bit) << (bit + 1)) | (p & ((1u << bit) - 1u));
}

// Apply the ops of a sweep to a tile of 2^k amplitudes held in LDS.
template <typename V>
__device__ void tile_ops(V *tile, uint32_t k, const DOp *ops, uint32_t ob, uint32_t oe, bool inverse,
                         const V *mats) {
    const uint32_t T = 1u << k, tid = threadIdx.x, nt = blockDim.x;
    const uint32_t nops = oe - ob;
    for (uint32_t i = 0; i < nops; ++i) {
        const DOp op = ops[ob + (inverse ? nops - 1 - i : i)];
        const uint32_t qa = op.ab & 0xFFu, qb = (op.ab >> 8) & 0xFFu;
        const V *m = mats + op.mat;
        if (qb == 0xFFu) {
            V m0 = m[0], m1 = m[1], m2 = m[2], m3 = m[3];
            if (inverse) {
                const V t = m1;
                m0.y = -m0.y; m3.y = -m3.y;
                m1 = V{m2.x, -m2.y}; m2 = V{t.x, -t.y};
            }
            const uint32_t bit = 1u << qa;
            for (uint32_t p = tid; p < (T >> 1); p += nt) {
                const uint32_t i0 = ins0(p, qa), i1 = i0 | bit;
                const V v0 = tile[i0], v1 = tile[i1];
                V r0{0, 0}, r1{0, 0};
                tile[i0] = bfma(bfma(r0, m0, v0), m1, v1);
                tile[i1] = bfma(bfma(r1, m2, v0), m3, v1);
            }
        } else {
            V mm[16];
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const V x = inverse ? m[4 * c + r] : m[4 * r + c];
                    mm[4 * r + c] = inverse ? V{x.x, -x.y} : x;
                }
            const uint32_t lo = qa < qb ? qa : qb, hi = qa < qb ? qb : qa;
            const uint32_t A = 1u << qa, B = 1u << qb;
            for (uint32_t p = tid; p < (T >> 2); p += nt) {
                const uint32_t i0 = ins0(ins0(p, lo), hi);
                const uint32_t idx[4] = {i0, i0 | B, i0 | A, i0 | A | B};
                V v[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) v[r] = tile[idx[r]];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    V acc{0, 0};
#pragma unroll
                    for (int c = 0; c < 4; ++c) acc = bfma(acc, mm[4 * r + c], v[c]);
                    tile[idx[r]] = acc;
                }
            }
        }
        __syncthreads();
    }
}

template <typename V>
__device__ __forceinline__ double pr(V v) {
    const double re = static_cast<double>(v.x), im = static_cast<double>(v.y);
    return re * re + im * im;
}

constexpr uint32_t BATCH_CHUNK_LOG = 6;   // 64 amplitudes per sampling chunk
constexpr uint32_t BATCH_MAX_CHUNKS = 1024;

template <typename V>
__global__ void __launch_bounds__(256) k_batch(const BUnit *__restrict__ units, uint32_t n_units,
                                               uint32_t *queue, const BStep *__restrict__ steps,
                                               const BPass *__restrict__ passes,
                                               const DOp *__restrict__ ops, const V *__restrict__ mats,
                                               const BLeaf *__restrict__ leaves, V *scratch,
                                               uint64_t slot_elems, double *partial,
                                               uint64_t *samples, uint32_t lds_elems) {
    extern __shared__ unsigned char smem_raw[];
    V *tile = reinterpret_cast<V *>(smem_raw);
    double *cpre = reinterpret_cast<double *>(smem_raw + sizeof(V) * lds_elems);
    __shared__ uint32_t s_unit;
    __shared__ double s_norm;
    const uint32_t tid = threadIdx.x, nt = blockDim.x;
    V *slot = scratch + static_cast<uint64_t>(blockIdx.x) * slot_elems;
    for (;;) {
        __syncthreads();
        if (tid == 0) s_unit = atomicAdd(queue, 1u);
        __syncthreads();
        const uint32_t u = s_unit;
        if (u >= n_units) break;
        const BUnit U = units[u];
        const uint32_t n = U.n;
        const uint64_t N = 1ull << n;
        V *st = U.resident ? tile : slot;   // where the state lives between steps
        double *acc = partial ? partial + U.partial_off : nullptr;
        for (uint32_t si = U.step_begin; si < U.step_end; ++si) {
            const BStep S = steps[si];
            if (S.kind == 0) {
                for (uint64_t i = tid; i < N; i += nt) st[i] = V{0, 0};
                __syncthreads();
                if (tid == 0) st[0] = V{1, 0};
                if (!U.resident) __threadfence();
                __syncthreads();
            } else if (S.kind == 1 || S.kind == 2) {
                const BPass P = passes[S.arg];
                const bool inv = S.kind == 2;
                if (U.resident) {
                    tile_ops<V>(tile, n, ops, P.op_begin, P.op_end, inv, mats);
                } else {
                    const uint32_t k = P.k, T = 1u << k;
                    for (uint64_t t = 0; t < (N >> k); ++t) {
                        uint64_t base = t;
                        for (uint32_t j = 0; j < k; ++j) {
                            const uint32_t q = P.q[j];
                            base = ((base >> q) << (q + 1)) | (base & ((1ull << q) - 1ull));
                        }
                        for (uint32_t l = tid; l < T; l += nt) {
                            uint64_t off = l & ((1u << P.low) - 1u);
                            for (uint32_t j = P.low; j < k; ++j)
                                off |= static_cast<uint64_t>((l >> j) & 1u) << P.q[j];
                            tile[l] = slot[base + off];
                        }
                        __syncthreads();
                        tile_ops<V>(tile, k, ops, P.op_begin, P.op_end, inv, mats);
                        for (uint32_t l = tid; l < T; l += nt) {
                            uint64_t off = l & ((1u << P.low) - 1u);
                            for (uint32_t j = P.low; j < k; ++j)
                                off |= static_cast<uint64_t>((l >> j) & 1u) << P.q[j];
                            slot[base + off] = tile[l];
                        }
                        __threadfence();
                        __syncthreads();
                    }
                }
            } else {
                const BLeaf L = leaves[S.arg];
                const uint32_t clog = n < BATCH_CHUNK_LOG ? n : BATCH_CHUNK_LOG;
                const uint32_t C = 1u << clog, nch = static_cast<uint32_t>(N >> clog);
                for (uint32_t c = tid; c < nch; c += nt) {
                    double s = 0.0;
                    for (uint32_t i = 0; i < C; ++i) {
                        const uint64_t idx = static_cast<uint64_t>(c) * C + i;
                        const double p = pr(st[idx]);
                        s += p;
                        if (acc) acc[idx] += L.w * p;
                    }
                    cpre[c] = s;
                }
                __syncthreads();
                if (tid == 0) {
                    double r = 0.0;
                    for (uint32_t c = 0; c < nch; ++c) {
                        r += cpre[c];
                        cpre[c] = r;
                    }
                    s_norm = r;
                }
                __syncthreads();
                const double norm = s_norm;
                for (uint64_t d = tid; d < L.shots; d += nt) {
                    const Pair64 rr = philox_pair(U.seed, static_cast<uint32_t>(d >> 1), L.leaf, 0,
                                                  STREAM_SHOTS);
                    const uint64_t v = (d & 1) ? rr.hi : rr.lo;
                    const double x = static_cast<double>(v >> 11) * 0x1p-53 * norm;
                    uint32_t lo = 0, hi = nch;
                    while (lo < hi) {
                        const uint32_t mid = (lo + hi) >> 1;
                        if (cpre[mid] > x) hi = mid; else lo = mid + 1;
                    }
                    const uint32_t c = lo < nch ? lo : nch - 1;
                    double run = c ? cpre[c - 1] : 0.0;
                    uint64_t res = static_cast<uint64_t>(c) * C + (C - 1);
                    uint64_t last_nz = static_cast<uint64_t>(c) * C;
                    bool found = false;
                    for (uint32_t i = 0; i < C; ++i) {
                        const uint64_t idx = static_cast<uint64_t>(c) * C + i;
                        const double p = pr(st[idx]);
                        if (p > 0.0) last_nz = idx;
                        run += p;
                        if (run > x) { res = idx; found = true; break; }
                    }
                    samples[U.sample_base + L.sample_off + d] = found ? res : last_nz;
                }
                __syncthreads();
            }
        }
    }
}

__global__ void k_batch_combine(const double *partial, const uint64_t *job_unit_off,
                                const uint64_t *unit_partial_off, const uint64_t *job_dist_off,
                                const uint32_t *job_n, uint32_t n_jobs, double *dist) {
    const uint32_t j = blockIdx.y;
    if (j >= n_jobs) return;
    const uint64_t N = 1ull << job_n[j];
    for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < N;
         i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
        double s = 0.0;
        for (uint64_t u = job_unit_off[j]; u < job_unit_off[j + 1]; ++u) s += partial[unit_partial_off[u] + i];
        dist[job_dist_off[j] + i] = s;
    }
}

__global__ void k_fill_batch(double *p, uint64_t n) {
    for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
        p[i] = 0.0;
}

__global__ void k_set_u32(uint32_t *p, uint32_t v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

// ---------------------------------------------------------------------------
namespace {

template <typename T>
struct HostDev {
    std::vector<T> h;
    DevBuf d;
    void upload(hipStream_t s) {
        d.alloc(std::max<size_t>(h.size(), 1) * sizeof(T));
        if (!h.empty()) hip_check(hipMemcpyAsync(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s), "upload");
    }
    T *ptr() { return static_cast<T *>(d.p); }
};

template <typename V>
void batch_typed(Ctx &ctx, const std::vector<const Circuit *> &circs, const tusq_opts &o,
                 std::vector<Result> &out) {
    const size_t J = circs.size();
    const bool c64 = std::is_same<V, float2>::value;
    const uint32_t KL = c64 ? 14 : 13;        // LDS-resident up to 2^KL amplitudes (128 KiB)
    const uint32_t KT = c64 ? 13 : 12;        // tile qubits for larger states (64 KiB)
    for (const Circuit *c : circs)
        if (c->n > 16 || c->n < 1) fail(TUSQ_EUNSUPPORTED, "batched jobs need 1..16 qubits");
    if (o.traversal == TUSQ_CHECKPOINT || o.traversal == TUSQ_CACHING)
        fail(TUSQ_EUNSUPPORTED, "the batched path has no checkpoint or caching traversal");
    if (J == 0) { out.clear(); return; }
    if (J > 65535) fail(TUSQ_EUNSUPPORTED, "at most 65535 jobs per batch");
    const bool want_dist = o.want & TUSQ_WANT_DIST;
    hip_check(hipSetDevice(ctx.device), "hipSetDevice");
    hipStream_t s = ctx.stream;
    const double t0 = now_seconds();

    // 1. host: trees for every job (threads over jobs), seed = opts.seed + job
    std::vector<Tree> trees(J);
    {
        const unsigned nt = host_threads(o);
        std::vector<std::thread> th;
        std::atomic<size_t> next{0};
        std::vector<std::string> errs(nt);
        for (unsigned t = 0; t < nt; ++t)
            th.emplace_back([&, t] {
                try {
                    tusq_opts oj = o;
                    oj.host_threads = 1;
                    for (size_t j; (j = next++) < J;) {
                        oj.seed = o.seed + j;
                        trees[j] = build_tree(*circs[j], oj);
                    }
                } catch (const Error &e) {
                    errs[t] = e.msg;
                } catch (const std::exception &e) {
                    errs[t] = e.what();
                }
            });
        for (auto &x : th) x.join();
        for (auto &e : errs)
            if (!e.empty()) fail(TUSQ_EINVAL, e);
    }
    const double t_ecm = now_seconds() - t0;

    // 2. work units: leaf ranges of similar cost; one plan per unit
    HostDev<BUnit> units;
    HostDev<BStep> steps;
    HostDev<BPass> passes;
    HostDev<DOp> dops;
    HostDev<V> mats;
    HostDev<BLeaf> leaves;
    std::vector<uint64_t> job_unit_off(J + 1, 0), unit_poff, job_dist_off(J + 1, 0), job_sample_off(J + 1, 0);
    std::vector<uint32_t> job_n(J);
    uint64_t partial_elems = 0;
    std::vector<tusq_counters> jc(J);
    const double t1 = now_seconds();
    struct UnitPlan {
        size_t job;
        uint64_t lb, le;
    };
    std::vector<UnitPlan> ups;
    for (size_t j = 0; j < J; ++j) {
        const Tree &t = trees[j];
        job_n[j] = circs[j]->n;
        job_dist_off[j + 1] = job_dist_off[j] + (want_dist ? (1ull << circs[j]->n) : 0);
        uint64_t S = 0;
        for (uint64_t l = 0; l < t.leaves(); ++l) S += t.shots[l];
        job_sample_off[j + 1] = job_sample_off[j] + S;
        // about 64 leaves per unit, fewer units for cheap jobs
        const uint64_t L = t.leaves();
        const uint64_t per = std::max<uint64_t>(1, std::min<uint64_t>(64, (L + 3) / 4));
        for (uint64_t a = 0; a < L; a += per) ups.push_back(UnitPlan{j, a, std::min(L, a + per)});
        job_unit_off[j + 1] = ups.size();
    }
    auto unit_opts = [&](const UnitPlan &up) {
        const Circuit &c = *circs[up.job];
        tusq_opts ou = o;
        ou.seed = o.seed + up.job;
        ou.leaf_begin = up.lb;
        ou.leaf_end = up.le;
        ou.fusion_max_qubits = c.n <= KL ? c.n : KT;
        ou.fusion_low_qubits = c.n <= KL ? 0 : 5;
        if (c.n > KL && o.fusion_max_ops) ou.fusion_max_ops = o.fusion_max_ops;
        return ou;
    };
    // units are planned on host threads a window at a time (op lists only)
    // and appended in order, so the arrays do not depend on the thread count
    const unsigned nt_plan = host_threads(o);
    const size_t window = std::max<size_t>(4 * nt_plan, 1);
    std::vector<Plan> win;
    for (size_t ui = 0; ui < ups.size(); ++ui) {
        if (ui % window == 0) {
            const size_t w1 = std::min(ups.size(), ui + window);
            win.clear();
            win.resize(w1 - ui);
            std::vector<std::thread> th;
            std::atomic<size_t> next{ui};
            std::vector<std::string> errs(nt_plan);
            for (unsigned t = 0; t < nt_plan; ++t)
                th.emplace_back([&, t, ui, w1] {
                    try {
                        for (size_t x; (x = next++) < w1;)
                            win[x - ui] = build_plan(*circs[ups[x].job], trees[ups[x].job],
                                                     unit_opts(ups[x]), false, false);
                    } catch (const Error &e) {
                        errs[t] = e.msg;
                    } catch (const std::exception &e) {
                        errs[t] = e.what();
                    }
                });
            for (auto &x : th) x.join();
            for (auto &e : errs)
                if (!e.empty()) fail(TUSQ_EINVAL, e);
        }
        const UnitPlan &up = ups[ui];
        const Circuit &c = *circs[up.job];
        const tusq_opts ou = unit_opts(up);
        Plan p = std::move(win[ui % window]);
        BUnit U{};
        U.job = static_cast<uint32_t>(up.job);
        U.n = c.n;
        U.resident = c.n <= KL;
        U.k = ou.fusion_max_qubits;
        U.step_begin = static_cast<uint32_t>(steps.h.size());
        U.partial_off = partial_elems;
        U.sample_base = job_sample_off[up.job];
        U.seed = o.seed + up.job;
        if (want_dist) partial_elems += 1ull << c.n;
        unit_poff.push_back(U.partial_off);
        const uint32_t pass0 = static_cast<uint32_t>(passes.h.size());
        const uint32_t op0 = static_cast<uint32_t>(dops.h.size());
        const uint32_t mat0 = static_cast<uint32_t>(mats.h.size());
        for (const Pass &pp : p.passes) {
            BPass bp{};
            bp.k = pp.k;
            bp.low = 0;
            while (bp.low < pp.k && pp.q[bp.low] == bp.low) ++bp.low;
            bp.op_begin = op0 + pp.op_begin;
            bp.op_end = op0 + pp.op_end;
            for (uint32_t j2 = 0; j2 < pp.k; ++j2) bp.q[j2] = static_cast<uint8_t>(pp.q[j2]);
            passes.h.push_back(bp);
        }
        for (const Op &op : p.ops)
            dops.h.push_back(DOp{static_cast<uint32_t>(op.a) | (static_cast<uint32_t>(op.b) << 8), mat0 + op.mat});
        // nearest rounding for complex64: small batched jobs have no drift
        // check to keep below its bound, and the norm-keeping rounding of the
        // single-job path would add a serial host pass over every matrix
        for (const cd &m : p.mats) {
            using R = decltype(V{}.x);
            mats.h.push_back(V{static_cast<R>(m.real()), static_cast<R>(m.imag())});
        }
        uint64_t soff = 0;
        for (uint64_t l = 0; l < up.lb; ++l) soff += trees[up.job].shots[l];
        double work = 0;
        for (const Step &sp : p.steps) {
            BStep b{};
            b.kind = static_cast<uint32_t>(sp.kind);
            if (sp.kind == ST_FWD || sp.kind == ST_INV) {
                b.arg = pass0 + static_cast<uint32_t>(sp.id);
                work += static_cast<double>(p.passes[sp.id].op_end - p.passes[sp.id].op_begin + 1) *
                        static_cast<double>(1ull << c.n);
            } else if (sp.kind == ST_LEAF) {
                const Tree &t = trees[up.job];
                BLeaf L{};
                L.w = static_cast<double>(t.wnum[sp.id]) / static_cast<double>(t.wden[sp.id]);
                L.shots = t.shots[sp.id];
                L.sample_off = soff;
                L.leaf = static_cast<uint32_t>(sp.id);
                soff += t.shots[sp.id];
                b.arg = static_cast<uint32_t>(leaves.h.size());
                leaves.h.push_back(L);
                work += static_cast<double>(1ull << c.n);
            }
            steps.h.push_back(b);
        }
        U.step_end = static_cast<uint32_t>(steps.h.size());
        U.work = work;
        units.h.push_back(U);
        tusq_counters &ct = jc[up.job];
        const tusq_counters &pc = p.counters;
        ct.fwd_gates += pc.fwd_gates; ct.inv_gates += pc.inv_gates;
        ct.fwd_paulis += pc.fwd_paulis; ct.inv_paulis += pc.inv_paulis;
        ct.resets += pc.resets; ct.leaves += pc.leaves; ct.draws += pc.draws;
        ct.passes_fwd += pc.passes_fwd; ct.passes_inv += pc.passes_inv;
        ct.leaf_sweeps += pc.leaf_sweeps; ct.sweep_bytes += pc.sweep_bytes;
        ct.sweep_flops += pc.sweep_flops;
    }
    const double t_plan = now_seconds() - t1;
    // largest units first
    std::vector<uint32_t> order(units.h.size());
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return units.h[a].work > units.h[b].work; });
    {
        std::vector<BUnit> sorted(units.h.size());
        for (size_t i = 0; i < order.size(); ++i) sorted[i] = units.h[order[i]];
        units.h.swap(sorted);
    }

    // 3. device buffers and the graph
    units.upload(s);
    steps.upload(s);
    passes.upload(s);
    dops.upload(s);
    mats.upload(s);
    leaves.upload(s);
    HostDev<uint64_t> d_juo, d_upo, d_jdo;
    HostDev<uint32_t> d_jn;
    d_juo.h = job_unit_off;
    d_upo.h = unit_poff;
    d_jdo.h = job_dist_off;
    d_jn.h = job_n;
    d_juo.upload(s);
    d_upo.upload(s);
    d_jdo.upload(s);
    d_jn.upload(s);
    int cus = 0;
    hip_check(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx.device), "attr");
    const uint32_t lds_elems = 1u << std::max(KL, KT);
    const size_t lds_bytes = sizeof(V) * lds_elems + 8 * BATCH_MAX_CHUNKS;
    const uint32_t grid = static_cast<uint32_t>(std::max(1, cus));
    uint32_t maxn = 0;
    for (auto n : job_n) maxn = std::max(maxn, n);
    const uint64_t slot_elems = maxn > KL ? (1ull << maxn) : 1;
    DevBuf scratch, partial, samples, dist, queue;
    scratch.alloc(slot_elems * grid * sizeof(V));
    if (want_dist) {
        partial.alloc(std::max<uint64_t>(partial_elems, 1) * 8);
        dist.alloc(std::max<uint64_t>(job_dist_off[J], 1) * 8);
    }
    samples.alloc(std::max<uint64_t>(job_sample_off[J], 1) * 8);
    queue.alloc(4);
    hip_check(hipFuncSetAttribute(reinterpret_cast<const void *>(k_batch<V>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds_bytes)),
              "batch attr");
    hip_check(hipStreamSynchronize(s), "sync");

    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hip_check(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "capture");
    hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(64), 0, s, static_cast<uint32_t *>(queue.p), 0u);
    if (want_dist)
        hipLaunchKernelGGL(k_fill_batch, dim3(static_cast<unsigned>(std::min<uint64_t>((partial_elems + 255) / 256, 65535))),
                           dim3(256), 0, s, static_cast<double *>(partial.p), partial_elems);
    hipLaunchKernelGGL(k_batch<V>, dim3(grid), dim3(256), lds_bytes, s, units.ptr(),
                       static_cast<uint32_t>(units.h.size()), static_cast<uint32_t *>(queue.p), steps.ptr(),
                       passes.ptr(), dops.ptr(), mats.ptr(), leaves.ptr(), static_cast<V *>(scratch.p), slot_elems,
                       want_dist ? static_cast<double *>(partial.p) : nullptr, static_cast<uint64_t *>(samples.p),
                       lds_elems);
    if (want_dist)
        hipLaunchKernelGGL(k_batch_combine, dim3(64, static_cast<unsigned>(J)), dim3(256), 0, s,
                           static_cast<const double *>(partial.p), d_juo.ptr(), d_upo.ptr(), d_jdo.ptr(),
                           d_jn.ptr(), static_cast<uint32_t>(J), static_cast<double *>(dist.p));
    hipError_t ce = hipStreamEndCapture(s, &graph);
    hip_check(ce, "end capture");
    hip_check(hipGetLastError(), "batch launch");
    hip_check(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "graph instantiate");
    const double t2 = now_seconds();
    hip_check(hipGraphLaunch(exec, s), "graph launch");
    hip_check(hipStreamSynchronize(s), "sync");
    const double t_dev = now_seconds() - t2;
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);

    // 4. results
    std::vector<double> hdist(want_dist ? job_dist_off[J] : 0);
    std::vector<uint64_t> hs(job_sample_off[J]);
    if (want_dist && !hdist.empty())
        hip_check(hipMemcpy(hdist.data(), dist.p, hdist.size() * 8, hipMemcpyDeviceToHost), "dist");
    if (!hs.empty()) hip_check(hipMemcpy(hs.data(), samples.p, hs.size() * 8, hipMemcpyDeviceToHost), "samples");
    out.resize(J);
    for (size_t j = 0; j < J; ++j) {
        Result &r = out[j];
        r.n = circs[j]->n;
        if (want_dist) r.dist.assign(hdist.begin() + job_dist_off[j], hdist.begin() + job_dist_off[j + 1]);
        r.samples.assign(hs.begin() + job_sample_off[j], hs.begin() + job_sample_off[j + 1]);
        r.counters = jc[j];
        r.counters.host_ecm_seconds = t_ecm;
        r.counters.host_plan_seconds = t_plan;
        r.counters.device_seconds = t_dev;
    }
}

}  // namespace

void run_batch(Ctx &ctx, const std::vector<const Circuit *> &circs, const tusq_opts &o,
               std::vector<Result> &out) {
    if (o.precision == TUSQ_C64) batch_typed<float2>(ctx, circs, o, out);
    else batch_typed<double2>(ctx, circs, o, out);
}

}  // namespace tusq
