// capi.cpp -- the extern "C" boundary: argument validation, ownership and
// status codes; no exception crosses it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "engine.hpp"
#include "exec.hpp"
#include "serve.hpp"
#include "sha256.hpp"

using namespace tusq;

namespace {
thread_local std::string g_last_error;

template <class F>
int guarded(F &&f) {
    try {
        f();
        return TUSQ_OK;
    } catch (const Error &e) {
        g_last_error = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        g_last_error = "host allocation failed";
        return TUSQ_ENOMEM;
    } catch (const std::exception &e) {
        g_last_error = e.what();
        return TUSQ_EINVAL;
    } catch (...) {
        g_last_error = "unknown failure";
        return TUSQ_EINVAL;
    }
}

void need(bool ok, const char *msg) {
    if (!ok) fail(TUSQ_EINVAL, msg);
}

void check_opts(const tusq_opts *o) {
    need(o != nullptr, "opts is NULL");
    need(o->shots >= 1 && o->shots <= 0xFFFFFFFFull, "shots must be in [1, 2^32)");
    need(o->alpha_den > 0, "alpha_den must be positive");
    need(o->precision == TUSQ_C128 || o->precision == TUSQ_C64, "unknown precision");
    need(o->traversal <= TUSQ_CACHING, "unknown traversal");
    need(!(o->leaf_begin > o->leaf_end && o->leaf_end != 0), "leaf_begin > leaf_end");
    need(o->drift_bound >= 0.0, "drift_bound must be >= 0");
    need(o->fusion_search <= 2, "unknown fusion_search");
}
}  // namespace

extern "C" {

const char *tusq_last_error(void) { return g_last_error.c_str(); }
uint32_t tusq_abi_version(void) { return TUSQ_ABI_VERSION; }

void tusq_opts_default(tusq_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->shots = 1000;
    o->seed = 1;
    o->alpha_num = 1;
    o->alpha_den = 100;
    o->beta = 100;
    o->precision = TUSQ_C128;
    o->traversal = TUSQ_DFTT;
    o->commute = 1;
    o->prune = 1;
    o->drift_bound = 1e-6;
    o->max_passes_between_recompute = 0;
    o->want = TUSQ_WANT_DIST | TUSQ_WANT_SAMPLES;
    o->debug_fail_at_step = -1;
    o->cache_capacity = 4;
}

int tusq_circuit_create(uint32_t n, tusq_circuit **out) {
    return guarded([&] {
        need(out != nullptr, "out is NULL");
        need(n >= 1 && n <= 34, "n_qubits must be in [1, 34]");
        auto *c = new tusq_circuit;
        c->c.n = n;
        *out = c;
    });
}

int tusq_circuit_gate(tusq_circuit *c, uint32_t kind, const uint32_t *qubits, const double *params,
                      uint32_t *gate_index_out) {
    return guarded([&] {
        need(c && qubits, "circuit or qubits is NULL");
        const bool user = kind == TUSQ_UNITARY1 || kind == TUSQ_UNITARY2;
        need(kind < TUSQ_NUM_KINDS || user, "unknown gate kind");
        Gate g{};
        g.kind = static_cast<uint8_t>(kind);
        g.q[0] = qubits[0];
        g.q[1] = is_two_qubit(g.kind) ? qubits[1] : 0;
        need(g.q[0] < c->c.n, "qubit out of range");
        if (is_two_qubit(g.kind))
            need(g.q[1] < c->c.n && g.q[1] != g.q[0], "2-qubit gate qubits out of range or equal");
        std::vector<cd> u;
        if (user) {
            // the matrix, checked finite and unitary: max |(U^H U - I)_ij| <= 1e-10
            const int d = kind == TUSQ_UNITARY1 ? 2 : 4;
            need(params != nullptr, "a unitary gate needs its matrix in params");
            u.resize(d * d);
            for (int i = 0; i < d * d; ++i) {
                u[i] = cd(params[2 * i], params[2 * i + 1]);
                need(std::isfinite(params[2 * i]) && std::isfinite(params[2 * i + 1]),
                     "non-finite matrix entry");
            }
            double dev = 0.0;
            for (int r = 0; r < d; ++r)
                for (int k = 0; k < d; ++k) {
                    cd s = 0.0;
                    for (int j = 0; j < d; ++j) s += std::conj(u[j * d + r]) * u[j * d + k];
                    dev = std::max(dev, std::abs(s - (r == k ? 1.0 : 0.0)));
                }
            need(dev <= 1e-10, "matrix is not unitary");
        } else {
            for (int i = 0; i < 3; ++i) {
                g.p[i] = params ? params[i] : 0.0;
                need(std::isfinite(g.p[i]), "non-finite gate parameter");
            }
        }
        g.chan = -1;
        need(c->c.gates.size() < 0xFFFFFFF0u, "too many gates");
        if (user) {
            g.umat = static_cast<uint32_t>(c->c.umats.size());
            c->c.umats.insert(c->c.umats.end(), u.begin(), u.end());
        }
        c->c.gates.push_back(g);
        c->c.dirty = true;
        if (gate_index_out) *gate_index_out = static_cast<uint32_t>(c->c.gates.size() - 1);
    });
}

int tusq_circuit_pauli_noise(tusq_circuit *c, uint32_t gate_index, const double *probs,
                             uint32_t n_probs) {
    return guarded([&] {
        need(c && probs, "circuit or probs is NULL");
        need(gate_index < c->c.gates.size(), "gate index out of range");
        Gate &g = c->c.gates[gate_index];
        need(!is_measure(g.kind), "a measurement layer takes no noise channel");
        need(g.chan < 0, "gate already has a channel");
        need(n_probs == (is_two_qubit(g.kind) ? 15u : 3u), "wrong number of probabilities for the gate");
        double s = 0.0;
        Channel ch{};
        ch.m = static_cast<uint8_t>(n_probs);
        for (uint32_t k = 0; k < n_probs; ++k) {
            need(probs[k] >= 0.0 && std::isfinite(probs[k]), "probability negative or not finite");
            ch.prob[k] = probs[k];
            s += probs[k];
        }
        need(s <= 1.0 + 1e-12, "probabilities sum above 1");
        g.chan = static_cast<int32_t>(c->c.chans.size());
        c->c.chans.push_back(ch);
        c->c.dirty = true;
    });
}

static void thermal_probs(double t, double t1, double t2, double out[3]) {
    need(std::isfinite(t) && std::isfinite(t1) && std::isfinite(t2), "times must be finite");
    need(t >= 0.0 && t1 > 0.0 && t2 > 0.0, "need t >= 0, T1 > 0, T2 > 0");
    need(t2 <= 2.0 * t1, "need T2 <= 2 T1");
    const double a = -std::expm1(-t / t1);  // 1 - exp(-t/T1)
    const double b = -std::expm1(-t / t2);  // 1 - exp(-t/T2)
    out[0] = out[1] = a / 4.0;
    out[2] = std::max(0.0, b / 2.0 - a / 4.0);
}

int tusq_thermal_pauli_probs(double t, double t1, double t2, double *probs) {
    return guarded([&] {
        need(probs != nullptr, "probs is NULL");
        thermal_probs(t, t1, t2, probs);
    });
}

int tusq_circuit_thermal_noise(tusq_circuit *c, uint32_t gate_index, double t, double t1,
                               double t2) {
    double p1[3];
    double p[15];
    uint32_t m = 3;
    const int rc = guarded([&] {
        need(c != nullptr, "circuit is NULL");
        need(gate_index < c->c.gates.size(), "gate index out of range");
        thermal_probs(t, t1, t2, p1);
        if (is_two_qubit(c->c.gates[gate_index].kind)) {
            // independent channels on the first (a) and second (b) qubit: outcome 4a + b
            const double q[4] = {1.0 - p1[0] - p1[1] - p1[2], p1[0], p1[1], p1[2]};
            m = 15;
            for (int k = 1; k < 16; ++k) p[k - 1] = q[k >> 2] * q[k & 3];
        } else {
            std::copy(p1, p1 + 3, p);
        }
    });
    if (rc != TUSQ_OK) return rc;
    return tusq_circuit_pauli_noise(c, gate_index, p, m);
}

int tusq_circuit_readout_noise(tusq_circuit *c, uint32_t qubit, double p,
                               uint32_t *gate_index_out) {
    const int rc = guarded([&] {
        need(c != nullptr, "circuit is NULL");
        need(qubit < c->c.n, "qubit out of range");
        need(std::isfinite(p) && p >= 0.0 && p <= 1.0, "read-out flip probability outside [0, 1]");
    });
    if (rc != TUSQ_OK) return rc;
    uint32_t g = 0;
    const double angle[3] = {0.0, 0.0, 0.0};
    int r = tusq_circuit_gate(c, TUSQ_RZ, &qubit, angle, &g);
    if (r != TUSQ_OK) return r;
    const double probs[3] = {p, 0.0, 0.0};
    r = tusq_circuit_pauli_noise(c, g, probs, 3);
    if (r != TUSQ_OK) {  // take the gate back: the call appends both or nothing
        c->c.gates.pop_back();
        c->c.dirty = true;
        return r;
    }
    if (gate_index_out) *gate_index_out = g;
    return r;
}

int tusq_circuit_measure(tusq_circuit *c, const uint32_t *qubits, uint32_t count, int reset,
                         uint32_t *gate_index_out) {
    return guarded([&] {
        need(c && qubits, "circuit or qubits is NULL");
        need(count >= 1 && count <= TUSQ_MAX_MEASURED, "a measurement layer takes 1..8 qubits");
        uint64_t mk = 0;
        for (uint32_t i = 0; i < count; ++i) {
            need(qubits[i] < c->c.n, "qubit out of range");
            need(!((mk >> qubits[i]) & 1), "measured qubit repeated");
            mk |= 1ull << qubits[i];
        }
        Gate g{};
        g.kind = static_cast<uint8_t>(reset ? TUSQ_MEASURE_RESET : TUSQ_MEASURE);
        g.q[0] = static_cast<uint32_t>(mk);
        g.q[1] = static_cast<uint32_t>(mk >> 32);
        g.chan = -1;
        need(c->c.gates.size() < 0xFFFFFFF0u, "too many gates");
        c->c.gates.push_back(g);
        c->c.dirty = true;
        if (gate_index_out) *gate_index_out = static_cast<uint32_t>(c->c.gates.size() - 1);
    });
}

int tusq_circuit_destroy(tusq_circuit *c) {
    delete c;
    return TUSQ_OK;
}

int tusq_ecm_build(const tusq_circuit *c, const tusq_opts *o, tusq_tree **out) {
    return guarded([&] {
        need(c && out, "circuit or out is NULL");
        check_opts(o);
        auto *cc = const_cast<tusq_circuit *>(c);
        cc->c.finalize();
        auto *t = new tusq_tree;
        try {
            t->t = build_tree(cc->c, *o);
        } catch (...) {
            delete t;
            throw;
        }
        *out = t;
    });
}

int tusq_tree_get_info(const tusq_tree *t, tusq_tree_info *out) {
    return guarded([&] {
        need(t && out, "tree or out is NULL");
        *out = t->t.info;
    });
}

int tusq_tree_serialize(const tusq_tree *t, uint8_t *buf, size_t cap, size_t *len_out) {
    return guarded([&] {
        need(t && len_out, "tree or len_out is NULL");
        const auto b = serialize_tree(t->t);
        *len_out = b.size();
        if (buf) {
            need(cap >= b.size(), "buffer too small");
            std::memcpy(buf, b.data(), b.size());
        }
    });
}

int tusq_tree_raw_events(const tusq_tree *t, uint32_t *shot, uint32_t *channel, uint8_t *outcome,
                         uint64_t cap, uint64_t *n_out) {
    return guarded([&] {
        need(t && n_out, "tree or n_out is NULL");
        const uint64_t n = t->t.raw_shot.size();
        *n_out = n;
        if (shot || channel || outcome) {
            need(cap >= n, "buffer too small");
            if (shot) std::memcpy(shot, t->t.raw_shot.data(), n * 4);
            if (channel) std::memcpy(channel, t->t.raw_chan.data(), n * 4);
            if (outcome) std::memcpy(outcome, t->t.raw_out.data(), n);
        }
    });
}

int tusq_raw_er_hash(const tusq_tree *t, uint8_t *sha256_out) {
    return guarded([&] {
        need(t && sha256_out, "tree or output is NULL");
        Sha256 h;
        const uint64_t n = t->t.raw_shot.size();
        uint8_t rec[9 * 512];
        size_t fill = 0;
        for (uint64_t i = 0; i < n; ++i) {
            const uint32_t s = t->t.raw_shot[i], ch = t->t.raw_chan[i];
            for (int b = 0; b < 4; ++b) {
                rec[fill + b] = static_cast<uint8_t>(s >> (8 * b));
                rec[fill + 4 + b] = static_cast<uint8_t>(ch >> (8 * b));
            }
            rec[fill + 8] = t->t.raw_out[i];
            fill += 9;
            if (fill == sizeof(rec)) {
                h.update(rec, fill);
                fill = 0;
            }
        }
        h.update(rec, fill);
        h.finish(sha256_out);
    });
}

int tusq_tree_destroy(tusq_tree *t) {
    delete t;
    return TUSQ_OK;
}

int tusq_plan_counters(const tusq_circuit *c, const tusq_tree *t, const tusq_opts *o,
                       tusq_counters *out) {
    return guarded([&] {
        need(c && t && out, "NULL argument");
        check_opts(o);
        auto *cc = const_cast<tusq_circuit *>(c);
        cc->c.finalize();
        need(t->t.n == cc->c.n && t->t.G == cc->c.gates.size(), "tree was built for another circuit");
        const double t0 = now_seconds();
        Plan p = build_plan(cc->c, t->t, *o, false, false);
        p.counters.host_plan_seconds = now_seconds() - t0;
        *out = p.counters;
    });
}

int tusq_plan_dump(const tusq_circuit *c, const tusq_tree *t, const tusq_opts *o, uint64_t *n_steps,
                   int64_t *steps, uint64_t *n_passes, uint32_t *qubits, uint64_t *op_range,
                   uint64_t *n_ops, uint32_t *ops, uint64_t *n_mats, double *mats) {
    return guarded([&] {
        need(c && t && n_steps && n_passes && n_ops && n_mats, "NULL argument");
        check_opts(o);
        auto *cc = const_cast<tusq_circuit *>(c);
        cc->c.finalize();
        need(t->t.n == cc->c.n && t->t.G == cc->c.gates.size(), "tree was built for another circuit");
        Plan p = build_plan(cc->c, t->t, *o, false);
        *n_steps = p.steps.size();
        *n_passes = p.passes.size();
        *n_ops = p.ops.size();
        *n_mats = p.mats.size();
        if (steps)
            for (size_t i = 0; i < p.steps.size(); ++i) {
                steps[2 * i] = p.steps[i].kind;
                steps[2 * i + 1] = static_cast<int64_t>(p.steps[i].id);
            }
        if (qubits)
            for (size_t i = 0; i < p.passes.size(); ++i)
                for (int j = 0; j < 16; ++j) qubits[16 * i + j] = j < static_cast<int>(p.passes[i].k) ? p.passes[i].q[j] : 0xFFFFFFFFu;
        if (op_range)
            for (size_t i = 0; i < p.passes.size(); ++i) {
                op_range[2 * i] = p.passes[i].op_begin;
                op_range[2 * i + 1] = p.passes[i].op_end - p.passes[i].op_begin;
            }
        if (ops)
            for (size_t i = 0; i < p.ops.size(); ++i) {
                ops[3 * i] = p.ops[i].a;
                ops[3 * i + 1] = p.ops[i].b;
                ops[3 * i + 2] = p.ops[i].mat;
            }
        if (mats)
            for (size_t i = 0; i < p.mats.size(); ++i) {
                mats[2 * i] = p.mats[i].real();
                mats[2 * i + 1] = p.mats[i].imag();
            }
    });
}

int tusq_plan_dump_programs(const tusq_circuit *c, const tusq_tree *t, const tusq_opts *o,
                            uint64_t *n_instr, uint32_t *instr, uint64_t *n_passes, uint32_t *ranges,
                            uint32_t *reg_qubits) {
    return guarded([&] {
        need(c && t && n_instr && n_passes && reg_qubits, "NULL argument");
        check_opts(o);
        auto *cc = const_cast<tusq_circuit *>(c);
        cc->c.finalize();
        need(t->t.n == cc->c.n && t->t.G == cc->c.gates.size(), "tree was built for another circuit");
        Plan p = build_plan(cc->c, t->t, *o, false);
        *n_instr = p.prog.size();
        *n_passes = p.passes.size();
        *reg_qubits = p.reg_qubits;
        if (instr)
            for (size_t i = 0; i < p.prog.size(); ++i) {
                instr[2 * i] = p.prog[i].w0;
                instr[2 * i + 1] = p.prog[i].mat;
            }
        if (ranges)
            for (size_t i = 0; i < p.passes.size(); ++i) {
                uint32_t *r = ranges + 12 * i;
                r[0] = p.passes[i].fwd_begin;
                r[1] = p.passes[i].fwd_end;
                r[2] = p.passes[i].inv_begin;
                r[3] = p.passes[i].inv_end;
                for (int d = 0; d < 2; ++d)
                    for (int w = 0; w < 4; ++w) r[4 + 4 * d + w] = p.passes[i].lay[d][w];
            }
    });
}

int tusq_ctx_create(int hip_device, uint64_t hbm_budget_bytes, tusq_ctx **out) {
    return guarded([&] {
        need(out != nullptr, "out is NULL");
        auto *c = new tusq_ctx;
        try {
            c->c = new Ctx(hip_device, hbm_budget_bytes);
        } catch (...) {
            delete c;
            throw;
        }
        *out = c;
    });
}

int tusq_ctx_destroy(tusq_ctx *ctx) {
    if (!ctx) return TUSQ_OK;
    return guarded([&] {
        serving_shutdown(*ctx->c);
        delete ctx->c;
        delete ctx;
    });
}

static void run_common(tusq_ctx *ctx, const tusq_circuit *c, const tusq_tree *given,
                       const tusq_opts *o, void *stream, tusq_result **out) {
    need(ctx && c && out, "NULL argument");
    check_opts(o);
    auto *cc = const_cast<tusq_circuit *>(c);
    cc->c.finalize();
    const uint64_t need_b = job_device_bytes(cc->c.n, o->precision, o->shots, o->want & TUSQ_WANT_DIST);
    if (need_b > ctx->c->budget) fail(TUSQ_ENOMEM, "job needs more device memory than the budget");
    const bool mcm = has_measure(cc->c);
    if (mcm) {
        if (o->traversal != TUSQ_CACHING)
            fail(TUSQ_EUNSUPPORTED, "the circuit has measurement layers: run it with TUSQ_CACHING");
        if (o->prune) fail(TUSQ_EUNSUPPORTED, "measurement layers need prune = 0");
    }
    auto *r = new tusq_result;
    try {
        double t0 = now_seconds();
        Tree local;
        const Tree *t = given ? &given->t : nullptr;
        double ecm_s = 0.0;
        if (!given) {
            local = build_tree(cc->c, *o);
            t = &local;
            ecm_s = now_seconds() - t0;
        } else {
            need(given->t.n == cc->c.n && given->t.G == cc->c.gates.size(),
                 "tree was built for another circuit");
        }
        t0 = now_seconds();
        if (mcm) {
            McmPlan mp = build_mcm_plan(cc->c, *t, *o);
            const double plan_s = now_seconds() - t0;
            if (need_b + mcm_bytes(cc->c.n, o->precision, mp.K) > ctx->c->budget)
                fail(TUSQ_ENOMEM, "cached states exceed the device memory budget");
            execute_mcm(*ctx->c, *t, mp, *o, static_cast<hipStream_t>(stream), r->r);
            r->r.counters.host_ecm_seconds = ecm_s;
            r->r.counters.host_plan_seconds = plan_s;
            *out = r;
            return;
        }
        Plan p = build_plan(cc->c, *t, *o, o->precision == TUSQ_C64);
        const double plan_s = now_seconds() - t0;
        if (need_b + checkpoint_bytes(cc->c.n, o->precision, p.checkpoint_slots) > ctx->c->budget)
            fail(TUSQ_ENOMEM, "checkpoints exceed the device memory budget");
        execute_plan(*ctx->c, *t, p, *o, static_cast<hipStream_t>(stream), r->r);
        r->r.counters.host_ecm_seconds = ecm_s;
        r->r.counters.host_plan_seconds = plan_s;
    } catch (...) {
        delete r;
        throw;
    }
    *out = r;
}

int tusq_run(tusq_ctx *ctx, const tusq_circuit *c, const tusq_opts *o, void *stream,
             tusq_result **out) {
    return guarded([&] { run_common(ctx, c, nullptr, o, stream, out); });
}

int tusq_run_tree(tusq_ctx *ctx, const tusq_circuit *c, const tusq_tree *t, const tusq_opts *o,
                  void *stream, tusq_result **out) {
    return guarded([&] {
        need(t != nullptr, "tree is NULL");
        run_common(ctx, c, t, o, stream, out);
    });
}

int tusq_run_tree_noalloc(tusq_ctx *ctx, const tusq_circuit *c, const tusq_tree *t,
                          const tusq_opts *o, void *stream, double *dist_dev, uint64_t *samples_dev,
                          uint64_t samples_len, tusq_counters *counters_out) {
    return guarded([&] {
        need(ctx && c && t, "NULL argument");
        check_opts(o);
        auto *cc = const_cast<tusq_circuit *>(c);
        cc->c.finalize();
        need(t->t.n == cc->c.n && t->t.G == cc->c.gates.size(), "tree was built for another circuit");
        if (has_measure(cc->c))
            fail(TUSQ_EUNSUPPORTED, "the no-allocation run takes circuits without measurement layers");
        const double t0 = now_seconds();
        Plan p = build_plan(cc->c, t->t, *o, o->precision == TUSQ_C64);
        const double plan_s = now_seconds() - t0;
        Result r;
        execute_plan_static(*ctx->c, t->t, p, *o, static_cast<hipStream_t>(stream), r, dist_dev,
                            samples_dev, samples_len);
        r.counters.host_plan_seconds = plan_s;
        if (counters_out) *counters_out = r.counters;
    });
}

int tusq_autotune(tusq_ctx *ctx, const tusq_circuit *c, const tusq_tree *t, const tusq_opts *o,
                  uint32_t probe_leaves, tusq_opts *tuned) {
    return guarded([&] {
        need(ctx && c && t && o && tuned, "NULL argument");
        check_opts(o);
        auto *cc = const_cast<tusq_circuit *>(c);
        cc->c.finalize();
        need(t->t.n == cc->c.n && t->t.G == cc->c.gates.size(), "tree was built for another circuit");
        *tuned = *o;
        if (has_measure(cc->c))
            fail(TUSQ_EUNSUPPORTED, "the autotuner runs circuits without measurement layers");
        const uint32_t n = cc->c.n;
        if (n <= 12) return;  // one tile holds the state
        const uint64_t key = (static_cast<uint64_t>(n) << 48) | (static_cast<uint64_t>(o->precision) << 40) |
                             cc->c.gates.size();
        {
            std::lock_guard<std::mutex> g(ctx->c->mu);
            auto it = ctx->c->tuned.find(key);
            if (it != ctx->c->tuned.end()) {
                tuned->fusion_max_qubits = it->second[0];
                tuned->fusion_low_qubits = it->second[1];
                tuned->fusion_max_ops = it->second[2];
                tuned->sweep_kernel = it->second[3];
                return;
            }
        }
        // (tile qubits, low qubits, ops per sweep, kernel): kernel 1 = one tile
        // per workgroup, 4 = persistent with register prefetch (16 amplitudes
        // per thread), 5 = persistent with 8 per thread
        static const uint32_t cand[][4] = {{12, 4, 32, 4}, {12, 4, 24, 4}, {13, 4, 32, 4},
                                           {13, 5, 32, 4}, {12, 4, 32, 1}, {11, 4, 24, 5}};
        const uint64_t L = t->t.leaves();
        const uint64_t lb = std::min<uint64_t>(o->leaf_begin, L ? L - 1 : 0);
        const uint64_t le = std::min<uint64_t>(L, lb + std::max<uint32_t>(1, probe_leaves));
        double best = 1e300;
        uint32_t pick[4] = {0, 0, 0, 0};
        for (const auto &cd : cand) {
            if (cd[0] > n) continue;
            tusq_opts tr = *o;
            tr.fusion_max_qubits = cd[0];
            tr.fusion_low_qubits = cd[1];
            tr.fusion_max_ops = cd[2];
            tr.sweep_kernel = cd[3];
            tr.leaf_begin = lb;
            tr.leaf_end = le;
            tr.want = 0;
            tr.profile = 0;
            // the probe plan keeps no recompute paths: no recompute of
            // either kind may come due
            tr.drift_bound = 1e300;
            tr.max_passes_between_recompute = 0;
            Plan p = build_plan(cc->c, t->t, tr, false);
            Result r;
            execute_plan(*ctx->c, t->t, p, tr, nullptr, r);
            if (r.counters.device_seconds < best) {
                best = r.counters.device_seconds;
                std::copy(cd, cd + 4, pick);
            }
        }
        tuned->fusion_max_qubits = pick[0];
        tuned->fusion_low_qubits = pick[1];
        tuned->fusion_max_ops = pick[2];
        tuned->sweep_kernel = pick[3];
        std::lock_guard<std::mutex> g(ctx->c->mu);
        ctx->c->tuned[key] = {pick[0], pick[1], pick[2], pick[3]};
    });
}

int tusq_submit(tusq_ctx *ctx, const tusq_circuit *c, const tusq_opts *o, uint64_t *job_id) {
    return guarded([&] {
        need(ctx && c && job_id, "NULL argument");
        check_opts(o);
        if (has_measure(c->c))
            fail(TUSQ_EUNSUPPORTED, "serving runs circuits without measurement layers; use tusq_run");
        *job_id = serving_submit(*ctx->c, c->c, *o);
    });
}

int tusq_poll(tusq_ctx *ctx, uint64_t job_id, int *state_out) {
    return guarded([&] {
        need(ctx && state_out, "NULL argument");
        *state_out = serving_poll(*ctx->c, job_id);
    });
}

int tusq_wait(tusq_ctx *ctx, uint64_t job_id, tusq_result **out) {
    return guarded([&] {
        need(ctx && out, "NULL argument");
        auto *r = new tusq_result;
        try {
            serving_wait(*ctx->c, job_id, r->r);
        } catch (...) {
            delete r;
            throw;
        }
        *out = r;
    });
}

int tusq_cancel(tusq_ctx *ctx, uint64_t job_id) {
    return guarded([&] {
        need(ctx != nullptr, "NULL argument");
        serving_cancel(*ctx->c, job_id);
    });
}

int tusq_job_times(tusq_ctx *ctx, uint64_t job_id, double *submitted, double *admitted,
                   double *finished) {
    return guarded([&] {
        need(ctx && submitted && admitted && finished, "NULL argument");
        serving_times(*ctx->c, job_id, submitted, admitted, finished);
    });
}

int tusq_run_batch(tusq_ctx *ctx, const tusq_circuit *const *circs, const tusq_opts *o,
                   size_t n_jobs, tusq_result **outs) {
    return guarded([&] {
        need(ctx && circs && outs, "NULL argument");
        check_opts(o);
        std::vector<const Circuit *> cs(n_jobs);
        for (size_t i = 0; i < n_jobs; ++i) {
            need(circs[i] != nullptr, "NULL circuit in batch");
            auto *cc = const_cast<tusq_circuit *>(circs[i]);
            if (has_measure(cc->c))
                fail(TUSQ_EUNSUPPORTED, "the batched path runs circuits without measurement layers");
            cc->c.finalize();
            cs[i] = &cc->c;
        }
        std::vector<Result> rs;
        run_batch(*ctx->c, cs, *o, rs);
        size_t made = 0;
        try {
            for (; made < n_jobs; ++made) {
                outs[made] = new tusq_result;
                outs[made]->r = std::move(rs[made]);
            }
        } catch (...) {
            for (size_t i = 0; i < made; ++i) delete outs[i];
            throw;
        }
    });
}

int tusq_batch_autotune(tusq_ctx *ctx, const tusq_circuit *const *circs, const tusq_opts *o,
                        size_t n_jobs, uint32_t probe_jobs) {
    return guarded([&] {
        need(ctx && circs, "NULL argument");
        check_opts(o);
        std::vector<const Circuit *> cs(n_jobs);
        for (size_t i = 0; i < n_jobs; ++i) {
            need(circs[i] != nullptr, "NULL circuit in batch");
            auto *cc = const_cast<tusq_circuit *>(circs[i]);
            if (has_measure(cc->c))
                fail(TUSQ_EUNSUPPORTED, "the batched path runs circuits without measurement layers");
            cc->c.finalize();
            cs[i] = &cc->c;
        }
        batch_autotune(*ctx->c, cs, *o, probe_jobs);
    });
}

int tusq_batch_shape(tusq_ctx *ctx, uint32_t n_qubits, uint32_t precision, uint32_t shape[5],
                     int *tuned) {
    return guarded([&] {
        need(ctx && shape, "NULL argument");
        need(n_qubits >= 1 && n_qubits <= 16, "batched jobs have 1..16 qubits");
        need(precision == TUSQ_C64 || precision == TUSQ_C128, "unknown precision");
        bool t = false;
        const BatchShape b = batch_shape(*ctx->c, n_qubits, precision, &t);
        shape[0] = b.threads;
        shape[1] = b.tile_qubits;
        shape[2] = b.low_qubits;
        shape[3] = b.max_ops;
        shape[4] = b.reg;
        if (tuned) *tuned = t ? 1 : 0;
    });
}

int tusq_result_distribution(const tusq_result *r, double *out, uint64_t len) {
    return guarded([&] {
        need(r && out, "NULL argument");
        need(r->r.has_dist(), "result holds no distribution");
        need(len == (1ull << r->r.n), "len must be 2^n");
        r->r.dist_copy(out);
    });
}

int tusq_result_distribution_device(const tusq_result *r, void *dptr, void *hip_stream) {
    return guarded([&] {
        need(r && dptr, "NULL argument");
        need(r->r.has_dist(), "result holds no distribution");
        const auto s = static_cast<hipStream_t>(hip_stream);
        const size_t bytes = (1ull << r->r.n) * 8;
        if (r->r.dist.empty()) {
            hip_check(hipSetDevice(r->r.device), "hipSetDevice");
            hip_check(hipMemcpyAsync(dptr, r->r.dist_dev->p, bytes, hipMemcpyDeviceToDevice, s),
                      "distribution to device");
        } else {
            hip_check(hipMemcpyAsync(dptr, r->r.dist.data(), bytes, hipMemcpyHostToDevice, s),
                      "distribution to device");
        }
        hip_check(hipStreamSynchronize(s), "sync");
    });
}

int tusq_result_samples(const tusq_result *r, uint64_t *out, uint64_t len) {
    return guarded([&] {
        need(r && out, "NULL argument");
        need(len == r->r.samples.size(), "len must equal the number of samples");
        if (len) std::memcpy(out, r->r.samples.data(), len * 8);
    });
}

int tusq_result_num_samples(const tusq_result *r, uint64_t *out) {
    return guarded([&] {
        need(r && out, "NULL argument");
        *out = r->r.samples.size();
    });
}

int tusq_result_norms(const tusq_result *r, double *out, uint64_t len) {
    return guarded([&] {
        need(r && out, "NULL argument");
        need(len == r->r.norms.size(), "len must equal the number of leaves run");
        if (len) std::memcpy(out, r->r.norms.data(), len * 8);
    });
}

int tusq_result_counters(const tusq_result *r, tusq_counters *out) {
    return guarded([&] {
        need(r && out, "NULL argument");
        *out = r->r.counters;
    });
}

int tusq_result_destroy(tusq_result *r) {
    delete r;
    return TUSQ_OK;
}

}  // extern "C"
