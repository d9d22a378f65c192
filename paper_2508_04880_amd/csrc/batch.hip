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
#include <map>
#include <mutex>
#include <cstdio>
#include <cstdlib>
#include <thread>

#include "kernels.hpp"
#include "regops.hpp"
#include "rng.hpp"
#include "serve.hpp"

namespace tusq {


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
    // register-blocked programs (forward, undo) of a sweep over a state in a
    // global slot: empty where the sweep runs as an op list in LDS
    uint32_t prog_fwd_begin, prog_fwd_end, prog_inv_begin, prog_inv_end;
    uint8_t q[16];
};

// register qubits of the batched walk's programs: 16 amplitudes per thread
constexpr uint32_t BATCH_REG_QUBITS = 4;
constexpr uint32_t BATCH_REG_TILE = 13;  // default tile of those programs
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

// REG: the class's states sit in global slots and its sweeps run the
// register-blocked programs where the workgroup matches the tile (one
// thread per 2^4 amplitudes), an instance of its own so that the LDS-resident
// classes keep their register budget.
template <typename V, int NT, bool REG>
__global__ void __launch_bounds__(NT) k_batch(const BUnit *__restrict__ units,
                                              const uint32_t *__restrict__ range, uint32_t *queue,
                                              const BStep *__restrict__ steps,
                                              const BPass *__restrict__ passes,
                                              const DOp *__restrict__ ops, const V *__restrict__ mats,
                                              const BLeaf *__restrict__ leaves, V *scratch,
                                              uint64_t slot_elems, double *partial,
                                              uint64_t *samples, double *norms, uint32_t lds_elems,
                                              const Instr2 *__restrict__ prog) {
    extern __shared__ unsigned char smem_raw[];
    V *tile = reinterpret_cast<V *>(smem_raw);
    double *cpre = reinterpret_cast<double *>(smem_raw + sizeof(V) * lds_elems);
    __shared__ uint32_t s_unit;
    __shared__ double s_norm;
    const uint32_t tid = threadIdx.x, nt = blockDim.x;
    V *slot = scratch + static_cast<uint64_t>(blockIdx.x) * slot_elems;
    for (;;) {
        __syncthreads();
        if (tid == 0) s_unit = range[0] + atomicAdd(queue, 1u);
        __syncthreads();
        const uint32_t u = s_unit;
        if (u >= range[1]) break;
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
                constexpr uint32_t R = BATCH_REG_QUBITS;
                const uint32_t pb = inv ? P.prog_inv_begin : P.prog_fwd_begin;
                const uint32_t pe = inv ? P.prog_inv_end : P.prog_fwd_end;
                if (U.resident) {
                    tile_ops<V>(tile, n, ops, P.op_begin, P.op_end, inv, mats);
                } else if constexpr (REG) {
                    // slot state, register-blocked: one thread per 2^R
                    // amplitudes of a tile; a sweep of k < the class's tile
                    // qubits runs nt / 2^(k-R) tiles at once, one per thread
                    // group, each with its own part of the LDS scratch.  All
                    // groups run the program in every round (a group with no
                    // tile left runs it on idle registers) so that the
                    // re-layout barriers match.  The host guarantees
                    // R <= k <= the class's tile qubits and a program.
                    const uint32_t k = P.k;
                    const uint32_t gsz = 1u << (k - R), groups = nt / gsz;
                    const uint32_t g = tid / gsz, ltid = tid % gsz;
                    V *glds = tile + (static_cast<size_t>(g) << k);
                    QMap qm;
#pragma unroll
                    for (int j = 0; j < 16; ++j) qm.q[j] = P.q[j];
                    const uint64_t toff = scatter(ltid, qm, P.low, k);
                    uint64_t roff[R];
#pragma unroll
                    for (uint32_t i = 0; i < R; ++i) roff[i] = 1ull << qat(qm, k - R + i);
                    const uint64_t tiles = N >> k;
                    for (uint64_t t0 = 0; t0 < tiles; t0 += groups) {
                        const uint64_t t = t0 + g;
                        const bool live = t < tiles;
                        const uint64_t base = live ? tile_base(t, qm, k) : 0;
                        V v[1 << R];
#pragma unroll
                        for (int j = 0; j < (1 << R); ++j) {
                            uint64_t o = base | toff;
#pragma unroll
                            for (uint32_t i = 0; i < R; ++i)
                                if (j >> i & 1) o |= roff[i];
                            v[j] = live ? slot[o] : V{0, 0};
                        }
                        run_program<V, R>(v, glds, ltid, k, prog, pb, pe, mats, true);
                        if (live) {
#pragma unroll
                            for (int j = 0; j < (1 << R); ++j) {
                                uint64_t o = base | toff;
#pragma unroll
                                for (uint32_t i = 0; i < R; ++i)
                                    if (j >> i & 1) o |= roff[i];
                                slot[o] = v[j];
                            }
                        }
                    }
                    __threadfence();
                    __syncthreads();
                } else if constexpr (!REG) {
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
                    norms[S.arg] = r;
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

// Sizes of one call, read by the graph's kernels from device memory so that
// a captured graph serves later calls of other sizes.
struct BDesc {
    uint64_t partial_elems;
    uint64_t n_jobs;
};

// dist of job j = the sum of its units' partials in unit order (fixed
// order: bitwise reproducible); blocks walk jobs, threads amplitudes
__global__ void k_batch_combine(const double *partial, const uint64_t *job_unit_off,
                                const uint64_t *unit_partial_off, const uint64_t *job_dist_off,
                                const uint32_t *job_n, const BDesc *desc, double *dist) {
    const uint64_t J = desc->n_jobs;
    for (uint64_t j = blockIdx.x; j < J; j += gridDim.x) {
        const uint64_t N = 1ull << job_n[j];
        for (uint64_t i = threadIdx.x; i < N; i += blockDim.x) {
            double s = 0.0;
            for (uint64_t u = job_unit_off[j]; u < job_unit_off[j + 1]; ++u)
                s += partial[unit_partial_off[u] + i];
            dist[job_dist_off[j] + i] = s;
        }
    }
}

__global__ void k_fill_batch(double *p, const BDesc *desc) {
    const uint64_t n = desc->partial_elems;
    for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
        p[i] = 0.0;
}

__global__ void k_zero_u32(uint32_t *p, uint32_t n) {
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0u;
}

// ---------------------------------------------------------------------------
// Host side: plans, launch shapes, the reusable graph.

constexpr uint32_t resident_max(bool c64) { return c64 ? 14u : 13u; }  // 128 KiB of LDS
constexpr uint32_t tile_default(bool c64) { return c64 ? 13u : 12u; }   // op lists: 64 KiB tiles

// Grow-only device buffer; ensure() reports whether the address changed (a
// graph captured with the old address no longer fits).
struct GrowBuf {
    DevBuf d;
    bool ensure(size_t b) {
        b = std::max<size_t>(b, 8);
        if (d.p && b <= d.bytes) return false;
        d.alloc(b + b / 4);
        return true;
    }
    template <typename T>
    T *ptr() const { return static_cast<T *>(d.p); }
};

// The buffers of the batched launches and the graph over them, kept in the
// context so that a later call with the same launch shapes replays it:
// every size the kernels need comes from device memory (unit ranges per
// qubit count, BDesc), uploaded before each replay.
struct BatchCache {
    GrowBuf units, range, steps, passes, dops, mats, leaves, prog, juo, upo, jdo, jn, desc;
    GrowBuf scratch, partial, dist, samples, norms, queues;
    std::vector<uint64_t> sig;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void drop_graph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        sig.clear();
    }
    ~BatchCache() { drop_graph(); }
};

void batch_cache_free(BatchCache *b) { delete b; }

namespace {

template <typename T>
void upload(GrowBuf &g, const std::vector<T> &h, hipStream_t s, bool &moved) {
    moved |= g.ensure(h.size() * sizeof(T));
    if (!h.empty()) hip_check(hipMemcpyAsync(g.d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s), "upload");
}

BatchShape default_shape(uint32_t n, bool c64) {
    BatchShape b;
    const bool res = n <= resident_max(c64);
    // slot states: register-blocked programs over tiles of 2^13 amplitudes
    // (128 KiB of complex128 in LDS), one thread per 16 amplitudes; measured
    // 1.7-1.8x faster than op lists in LDS for complex128 and about 10 %
    // for complex64
    b.tile_qubits = res ? n : BATCH_REG_TILE;
    b.low_qubits = res ? 0 : 5;
    b.max_ops = 0;
    b.reg = res ? 0 : 1;
    b.threads = res ? 256 : (1u << (b.tile_qubits - BATCH_REG_QUBITS));
    return b;
}

uint64_t shape_key(uint32_t n, uint32_t precision) { return (static_cast<uint64_t>(n) << 8) | precision; }

// the most LDS a batched launch asks for: a 2^13-amplitude complex128 (or
// 2^14 complex64) state and the sampler's chunk prefix
constexpr size_t BATCH_LDS_MAX = (16u << 13) + 8 * BATCH_MAX_CHUNKS;

template <typename V, int NT, bool REG>
void set_lds_attr() {
    static std::once_flag once;  // the attribute is per kernel, once per process
    std::call_once(once, [] {
        hip_check(hipFuncSetAttribute(reinterpret_cast<const void *>(k_batch<V, NT, REG>),
                                      hipFuncAttributeMaxDynamicSharedMemorySize,
                                      static_cast<int>(BATCH_LDS_MAX)),
                  "batch attr");
    });
}

template <typename V, int NT, bool REG>
int occupancy(size_t lds) {
    set_lds_attr<V, NT, REG>();
    int occ = 0;
    hip_check(hipOccupancyMaxActiveBlocksPerMultiprocessor(
                  &occ, reinterpret_cast<const void *>(k_batch<V, NT, REG>), NT, lds),
              "occupancy");
    return std::max(occ, 1);
}

// register programs need one thread per 16 amplitudes of a tile of at most
// 2^13 amplitudes: 256 or 512 threads
void check_shape(uint32_t threads, bool reg) {
    if (threads != 256 && threads != 512 && threads != 1024)
        fail(TUSQ_EINVAL, "batch workgroups have 256, 512 or 1024 threads");
    if (reg && threads == 1024) fail(TUSQ_EINVAL, "register-blocked batch sweeps take 256 or 512 threads");
}

template <typename V>
int occupancy_for(uint32_t threads, bool reg, size_t lds) {
    check_shape(threads, reg);
    if (reg) return threads == 256 ? occupancy<V, 256, true>(lds) : occupancy<V, 512, true>(lds);
    switch (threads) {
    case 256: return occupancy<V, 256, false>(lds);
    case 512: return occupancy<V, 512, false>(lds);
    default: return occupancy<V, 1024, false>(lds);
    }
}

template <typename V, int NT, bool REG>
void launch_class_nt(dim3 grid, size_t lds, hipStream_t s, BatchCache &bc, uint32_t ci, uint64_t slot_elems,
                     bool want_dist, uint32_t lds_elems) {
    set_lds_attr<V, NT, REG>();
    hipLaunchKernelGGL((k_batch<V, NT, REG>), grid, dim3(NT), lds, s, bc.units.ptr<BUnit>(),
                       bc.range.ptr<uint32_t>() + 2 * ci, bc.queues.ptr<uint32_t>() + ci, bc.steps.ptr<BStep>(),
                       bc.passes.ptr<BPass>(), bc.dops.ptr<DOp>(), bc.mats.ptr<V>(), bc.leaves.ptr<BLeaf>(),
                       bc.scratch.ptr<V>(), slot_elems, want_dist ? bc.partial.ptr<double>() : nullptr,
                       bc.samples.ptr<uint64_t>(), bc.norms.ptr<double>(), lds_elems,
                       bc.prog.ptr<const Instr2>());
}

template <typename V>
void launch_class(uint32_t threads, bool reg, dim3 grid, size_t lds, hipStream_t s, BatchCache &bc,
                  uint32_t ci, uint64_t slot_elems, bool want_dist, uint32_t lds_elems) {
    check_shape(threads, reg);
    if (reg) {
        if (threads == 256) launch_class_nt<V, 256, true>(grid, lds, s, bc, ci, slot_elems, want_dist, lds_elems);
        else launch_class_nt<V, 512, true>(grid, lds, s, bc, ci, slot_elems, want_dist, lds_elems);
        return;
    }
    switch (threads) {
    case 256: launch_class_nt<V, 256, false>(grid, lds, s, bc, ci, slot_elems, want_dist, lds_elems); break;
    case 512: launch_class_nt<V, 512, false>(grid, lds, s, bc, ci, slot_elems, want_dist, lds_elems); break;
    default: launch_class_nt<V, 1024, false>(grid, lds, s, bc, ci, slot_elems, want_dist, lds_elems); break;
    }
}

struct ClassInfo {
    uint32_t n;
    BatchShape shape;
    uint32_t unit_begin = 0, unit_end = 0;
    uint32_t grid = 0, lds_elems = 0;
    size_t lds_bytes = 0;
    uint64_t slot_elems = 0;
};

// force: one shape for every job (the autotuner's probes)
template <typename V>
void batch_typed(Ctx &ctx, const std::vector<const Circuit *> &circs, const tusq_opts &o,
                 std::vector<Result> &out, const BatchShape *force) {
    const size_t J = circs.size();
    const bool c64 = std::is_same<V, float2>::value;
    const uint32_t KL = resident_max(c64);
    for (const Circuit *c : circs)
        if (c->n > 16 || c->n < 1) fail(TUSQ_EUNSUPPORTED, "batched jobs need 1..16 qubits");
    if (o.traversal == TUSQ_CHECKPOINT || o.traversal == TUSQ_CACHING)
        fail(TUSQ_EUNSUPPORTED, "the batched path has no checkpoint or caching traversal");
    if (J == 0) { out.clear(); return; }
    if (J > (1u << 30)) fail(TUSQ_EUNSUPPORTED, "too many jobs in one batch");
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

    // launch shape per qubit count: forced, tuned, or the default
    std::map<uint32_t, BatchShape> shapes;
    for (const Circuit *c : circs) {
        if (shapes.count(c->n)) continue;
        BatchShape b = default_shape(c->n, c64);
        if (force) {
            b = *force;
            if (c->n <= KL) { b.tile_qubits = c->n; b.low_qubits = 0; }
        } else {
            std::lock_guard<std::mutex> g(ctx.mu);
            auto it = ctx.batch_tuned.find(shape_key(c->n, o.precision));
            if (it != ctx.batch_tuned.end()) b = it->second;
        }
        if (!force && o.fusion_max_ops && c->n > KL) b.max_ops = o.fusion_max_ops;
        // a register-blocked launch holds one tile per workgroup in LDS
        if (c->n > KL && b.reg &&
            (b.tile_qubits < BATCH_REG_QUBITS + 6 || b.tile_qubits > 13 ||
             b.threads != (1u << (b.tile_qubits - BATCH_REG_QUBITS))))
            fail(TUSQ_EINVAL, "register-blocked batch shapes take 2^(tile qubits - 4) threads");
        shapes[c->n] = b;
    }

    // 2. work units: leaf ranges of similar cost; one plan per unit
    std::vector<BUnit> units_h;
    std::vector<BStep> steps_h;
    std::vector<BPass> passes_h;
    std::vector<DOp> dops_h;
    std::vector<V> mats_h;
    std::vector<BLeaf> leaves_h;
    std::vector<Instr2> prog_h;
    std::vector<uint32_t> leaf_job;
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
        const BatchShape &b = shapes.at(c.n);
        tusq_opts ou = o;
        ou.seed = o.seed + up.job;
        ou.leaf_begin = up.lb;
        ou.leaf_end = up.le;
        ou.fusion_max_qubits = c.n <= KL ? c.n : b.tile_qubits;
        ou.fusion_low_qubits = c.n <= KL ? 0 : b.low_qubits;
        if (b.max_ops) ou.fusion_max_ops = b.max_ops;
        // slot states: programs that start and end in the initial layout,
        // 16 amplitudes per thread
        ou.sweep_kernel = 1;
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
                                                     unit_opts(ups[x]), false,
                                                     circs[ups[x].job]->n > KL &&
                                                         shapes.at(circs[ups[x].job]->n).reg);
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
        U.step_begin = static_cast<uint32_t>(steps_h.size());
        U.partial_off = partial_elems;
        U.sample_base = job_sample_off[up.job];
        U.seed = o.seed + up.job;
        if (want_dist) partial_elems += 1ull << c.n;
        unit_poff.push_back(U.partial_off);
        const uint32_t pass0 = static_cast<uint32_t>(passes_h.size());
        const uint32_t op0 = static_cast<uint32_t>(dops_h.size());
        const uint32_t mat0 = static_cast<uint32_t>(mats_h.size());
        const uint32_t prog0 = static_cast<uint32_t>(prog_h.size());
        for (const Instr &in : p.prog) {
            // op instructions name a matrix of this unit's pool
            const uint32_t type = in.w0 & 3u;
            prog_h.push_back(Instr2{in.w0, (type == 1u || type == 2u) ? in.mat + mat0 : in.mat});
        }
        for (const Pass &pp : p.passes) {
            BPass bp{};
            bp.k = pp.k;
            bp.low = 0;
            while (bp.low < pp.k && pp.q[bp.low] == bp.low) ++bp.low;
            bp.op_begin = op0 + pp.op_begin;
            bp.op_end = op0 + pp.op_end;
            if (!p.prog.empty() && pp.fwd_end > pp.fwd_begin) {
                bp.prog_fwd_begin = prog0 + pp.fwd_begin;
                bp.prog_fwd_end = prog0 + pp.fwd_end;
                bp.prog_inv_begin = prog0 + pp.inv_begin;
                bp.prog_inv_end = prog0 + pp.inv_end;
            }
            // the register-blocked launch runs every sweep of a slot state as
            // a program on whole thread groups: check what it relies on
            if (c.n > KL && shapes.at(c.n).reg &&
                (pp.k < BATCH_REG_QUBITS || pp.k > shapes.at(c.n).tile_qubits ||
                 pp.fwd_end <= pp.fwd_begin || pp.inv_end <= pp.inv_begin))
                fail(TUSQ_EINVAL, "internal: a batched sweep has no register program for its tile");
            for (uint32_t j2 = 0; j2 < pp.k; ++j2) bp.q[j2] = static_cast<uint8_t>(pp.q[j2]);
            passes_h.push_back(bp);
        }
        for (const Op &op : p.ops)
            dops_h.push_back(DOp{static_cast<uint32_t>(op.a) | (static_cast<uint32_t>(op.b) << 8), mat0 + op.mat});
        // nearest rounding for complex64: batched jobs have no recompute, and
        // the norm-keeping rounding of the single-job path would add a serial
        // host pass over every matrix; each job reports its norm drift
        for (const cd &m : p.mats) {
            using R = decltype(V{}.x);
            mats_h.push_back(V{static_cast<R>(m.real()), static_cast<R>(m.imag())});
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
                b.arg = static_cast<uint32_t>(leaves_h.size());
                leaves_h.push_back(L);
                leaf_job.push_back(static_cast<uint32_t>(up.job));
                work += static_cast<double>(1ull << c.n);
            }
            steps_h.push_back(b);
        }
        U.step_end = static_cast<uint32_t>(steps_h.size());
        U.work = work;
        units_h.push_back(U);
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

    // 3. one persistent launch per qubit count (largest states first), its
    // units largest first
    std::vector<ClassInfo> classes;
    for (auto it = shapes.rbegin(); it != shapes.rend(); ++it) {
        ClassInfo ci;
        ci.n = it->first;
        ci.shape = it->second;
        classes.push_back(ci);
    }
    {
        std::vector<uint32_t> order(units_h.size());
        std::iota(order.begin(), order.end(), 0);
        std::vector<uint32_t> cls_of(17, 0);
        for (uint32_t c = 0; c < classes.size(); ++c) cls_of[classes[c].n] = c;
        std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
            const uint32_t ca = cls_of[units_h[a].n], cb = cls_of[units_h[b].n];
            if (ca != cb) return ca < cb;
            return units_h[a].work > units_h[b].work;
        });
        std::vector<BUnit> sorted(units_h.size());
        for (size_t i = 0; i < order.size(); ++i) sorted[i] = units_h[order[i]];
        units_h.swap(sorted);
        for (uint32_t c = 0, u = 0; c < classes.size(); ++c) {
            classes[c].unit_begin = u;
            while (u < units_h.size() && units_h[u].n == classes[c].n) ++u;
            classes[c].unit_end = u;
        }
    }
    int cus = 0;
    hip_check(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx.device), "attr");
    uint64_t scratch_elems = 1;
    std::vector<uint32_t> range_h;
    std::vector<uint64_t> sig = {o.precision, want_dist ? 1u : 0u, classes.size()};
    for (ClassInfo &ci : classes) {
        const bool res = ci.n <= KL;
        ci.lds_elems = 1u << (res ? ci.n : ci.shape.tile_qubits);
        ci.lds_bytes = sizeof(V) * ci.lds_elems + 8 * BATCH_MAX_CHUNKS;
        ci.slot_elems = res ? 0 : (1ull << ci.n);
        const bool reg = !res && ci.shape.reg;
        const int occ = occupancy_for<V>(ci.shape.threads, reg, ci.lds_bytes);
        ci.grid = static_cast<uint32_t>(std::max(1, cus) * occ);
        scratch_elems = std::max<uint64_t>(scratch_elems, ci.slot_elems * ci.grid);
        range_h.push_back(ci.unit_begin);
        range_h.push_back(ci.unit_end);
        sig.insert(sig.end(), {ci.n, ci.shape.threads, ci.grid, ci.lds_bytes, ci.slot_elems, reg ? 1u : 0u});
    }

    // 4. buffers (kept in the context, grown when a call needs more), the
    // graph (replayed when the launch shapes and buffer addresses match)
    std::lock_guard<std::mutex> bg(ctx.batch_mu);
    if (!ctx.batch) ctx.batch = new BatchCache;
    BatchCache &bc = *ctx.batch;
    bool moved = false;
    const BDesc desc_h{partial_elems, J};
    upload(bc.units, units_h, s, moved);
    upload(bc.range, range_h, s, moved);
    upload(bc.steps, steps_h, s, moved);
    upload(bc.passes, passes_h, s, moved);
    upload(bc.dops, dops_h, s, moved);
    upload(bc.mats, mats_h, s, moved);
    upload(bc.leaves, leaves_h, s, moved);
    upload(bc.prog, prog_h, s, moved);
    upload(bc.juo, job_unit_off, s, moved);
    upload(bc.upo, unit_poff, s, moved);
    upload(bc.jdo, job_dist_off, s, moved);
    upload(bc.jn, job_n, s, moved);
    upload(bc.desc, std::vector<BDesc>{desc_h}, s, moved);
    moved |= bc.scratch.ensure(scratch_elems * sizeof(V));
    if (want_dist) {
        moved |= bc.partial.ensure(std::max<uint64_t>(partial_elems, 1) * 8);
        moved |= bc.dist.ensure(std::max<uint64_t>(job_dist_off[J], 1) * 8);
    }
    moved |= bc.samples.ensure(std::max<uint64_t>(job_sample_off[J], 1) * 8);
    moved |= bc.norms.ensure(std::max<size_t>(leaves_h.size(), 1) * 8);
    moved |= bc.queues.ensure(classes.size() * 4);
    hip_check(hipStreamSynchronize(s), "sync");

    const bool reuse = !moved && bc.exec && bc.sig == sig;
    if (!reuse) {
        bc.drop_graph();
        hip_check(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "capture");
        hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, bc.queues.ptr<uint32_t>(),
                           static_cast<uint32_t>(classes.size()));
        if (want_dist)
            hipLaunchKernelGGL(k_fill_batch, dim3(static_cast<unsigned>(4 * std::max(1, cus))), dim3(256), 0, s,
                               bc.partial.ptr<double>(), bc.desc.ptr<const BDesc>());
        for (uint32_t c = 0; c < classes.size(); ++c) {
            const ClassInfo &ci = classes[c];
            launch_class<V>(ci.shape.threads, ci.n > KL && ci.shape.reg, dim3(ci.grid), ci.lds_bytes, s, bc, c,
                            ci.slot_elems, want_dist, ci.lds_elems);
        }
        if (want_dist)
            hipLaunchKernelGGL(k_batch_combine, dim3(static_cast<unsigned>(2 * std::max(1, cus))), dim3(256), 0, s,
                               bc.partial.ptr<const double>(), bc.juo.ptr<const uint64_t>(),
                               bc.upo.ptr<const uint64_t>(), bc.jdo.ptr<const uint64_t>(),
                               bc.jn.ptr<const uint32_t>(), bc.desc.ptr<const BDesc>(), bc.dist.ptr<double>());
        hipError_t ce = hipStreamEndCapture(s, &bc.graph);
        hip_check(ce, "end capture");
        hip_check(hipGetLastError(), "batch launch");
        hip_check(hipGraphInstantiate(&bc.exec, bc.graph, nullptr, nullptr, 0), "graph instantiate");
        bc.sig = sig;
    }
    const double t2 = now_seconds();
    hip_check(hipGraphLaunch(bc.exec, s), "graph launch");
    hip_check(hipStreamSynchronize(s), "sync");
    const double t_dev = now_seconds() - t2;

    // 5. results
    std::vector<double> hdist(want_dist ? job_dist_off[J] : 0);
    std::vector<uint64_t> hs(job_sample_off[J]);
    std::vector<double> hn(leaves_h.size());
    if (want_dist && !hdist.empty())
        hip_check(hipMemcpy(hdist.data(), bc.dist.d.p, hdist.size() * 8, hipMemcpyDeviceToHost), "dist");
    if (!hs.empty()) hip_check(hipMemcpy(hs.data(), bc.samples.d.p, hs.size() * 8, hipMemcpyDeviceToHost), "samples");
    if (!hn.empty()) hip_check(hipMemcpy(hn.data(), bc.norms.d.p, hn.size() * 8, hipMemcpyDeviceToHost), "norms");
    std::vector<double> drift(J, 0.0);
    for (size_t i = 0; i < hn.size(); ++i) drift[leaf_job[i]] = std::max(drift[leaf_job[i]], std::fabs(hn[i] - 1.0));
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
        r.counters.max_norm_drift = drift[j];
        r.counters.batch_graph_reused = reuse ? 1 : 0;
    }
}

void run_batch_shape(Ctx &ctx, const std::vector<const Circuit *> &circs, const tusq_opts &o,
                     std::vector<Result> &out, const BatchShape *force) {
    if (o.precision == TUSQ_C64) batch_typed<float2>(ctx, circs, o, out, force);
    else if (o.precision == TUSQ_C128) batch_typed<double2>(ctx, circs, o, out, force);
    else fail(TUSQ_EINVAL, "unknown precision");
}

}  // namespace

void run_batch(Ctx &ctx, const std::vector<const Circuit *> &circs, const tusq_opts &o,
               std::vector<Result> &out) {
    run_batch_shape(ctx, circs, o, out, nullptr);
}

BatchShape batch_shape(Ctx &ctx, uint32_t n, uint32_t precision, bool *tuned) {
    std::lock_guard<std::mutex> g(ctx.mu);
    auto it = ctx.batch_tuned.find(shape_key(n, precision));
    if (tuned) *tuned = it != ctx.batch_tuned.end();
    if (it != ctx.batch_tuned.end()) return it->second;
    return default_shape(n, precision == TUSQ_C64);
}

void batch_autotune(Ctx &ctx, const std::vector<const Circuit *> &circs, const tusq_opts &o,
                    uint32_t probe_jobs) {
    const bool c64 = o.precision == TUSQ_C64;
    if (o.precision != TUSQ_C64 && o.precision != TUSQ_C128) fail(TUSQ_EINVAL, "unknown precision");
    // probes: the jobs with the most gates of each qubit count (they carry
    // most of the work)
    std::map<uint32_t, std::vector<const Circuit *>> by_n;
    for (const Circuit *c : circs) {
        if (c->n > 16 || c->n < 1) fail(TUSQ_EUNSUPPORTED, "batched jobs need 1..16 qubits");
        by_n[c->n].push_back(c);
    }
    for (auto &kv : by_n) {
        auto &v = kv.second;
        std::stable_sort(v.begin(), v.end(), [](const Circuit *a, const Circuit *b) {
            return a->gates.size() > b->gates.size();
        });
        v.resize(std::min<size_t>(v.size(), std::max<uint32_t>(probe_jobs, 1)));
    }
    // probes at the call's shot count (at most 10^4): the tree's leaf count
    // decides how many units a launch has, and a probe with a fifth of the
    // shots picked op lists for 15-qubit complex64 jobs that ran the real
    // jobs 2.2x slower than the register programs
    tusq_opts po = o;
    po.shots = std::min<uint64_t>(o.shots, 10000);
    po.want = TUSQ_WANT_SAMPLES;
    po.fusion_max_ops = 0;
    for (auto &kv : by_n) {
        const uint32_t n = kv.first;
        {
            std::lock_guard<std::mutex> g(ctx.mu);
            if (ctx.batch_tuned.count(shape_key(n, o.precision))) continue;
        }
        std::vector<BatchShape> cand;
        if (n <= resident_max(c64)) {
            for (uint32_t th : {256u, 512u, 1024u}) cand.push_back(BatchShape{th, n, 0, 0});
        } else {
            // op lists in LDS over tiles of 2^kt and 2^(kt+1) amplitudes
            // (the larger, 128 KiB, leaves room for one workgroup per CU),
            // and register-blocked programs over tiles of 2^12 / 2^13 (the
            // default is timed first and not repeated here)
            const uint32_t kt = tile_default(c64);
            cand.push_back(BatchShape{256, kt, 5, 32, 0});
            cand.push_back(BatchShape{256, kt + 1, 5, 32, 0});
            cand.push_back(BatchShape{1024, kt + 1, 5, 32, 0});
            cand.push_back(BatchShape{256, 12, 5, 0, 1});
            cand.push_back(BatchShape{512, 13, 4, 0, 1});
            cand.push_back(BatchShape{512, 13, 5, 16, 1});
        }
        // each candidate timed twice (the faster run counts); the default
        // shape is kept unless a candidate beats it by 3 %
        auto timed = [&](const BatchShape &b) {
            double t = 1e300;
            for (int rep = 0; rep < 2; ++rep) {
                std::vector<Result> out;
                run_batch_shape(ctx, kv.second, po, out, &b);
                if (!out.empty()) t = std::min(t, out[0].counters.device_seconds);
            }
            return t;
        };
        // TUSQ_TUNE_LOG set: each candidate's time on stderr
        const bool log = std::getenv("TUSQ_TUNE_LOG") != nullptr;
        auto say = [&](const BatchShape &b, double t) {
            if (log)
                std::fprintf(stderr, "[tusq] batch tune %s n=%u: threads %u tile %u low %u ops %u reg %u: %.3f ms\n",
                             c64 ? "c64" : "c128", n, b.threads, b.tile_qubits, b.low_qubits, b.max_ops, b.reg,
                             t * 1e3);
        };
        BatchShape pick = default_shape(n, c64);
        const double t_default = timed(pick);
        say(pick, t_default);
        double best = t_default;
        for (const BatchShape &b : cand) {
            const double t = timed(b);
            say(b, t);
            if (t < best) {
                best = t;
                pick = b;
            }
        }
        if (best > 0.97 * t_default) pick = default_shape(n, c64);
        std::lock_guard<std::mutex> g(ctx.mu);
        ctx.batch_tuned[shape_key(n, o.precision)] = pick;
    }
}

}  // namespace tusq
