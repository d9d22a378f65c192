// host_ecm.cpp -- circuit intake and the Error Characterisation Module
// (TUSQ Sec. III-A) on the host: error-realisation sampling, tallying,
// commutation, pruning and the depth-first leaf order.  Integer work only,
// bit-for-bit reproducible for a given seed, multi-threaded over shots and
// over unique ERs.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>
#include <queue>
#include <thread>

#include "engine.hpp"
#include "rng.hpp"

namespace tusq {

[[noreturn]] void fail(int code, const std::string &msg) { throw Error{code, msg}; }

double now_seconds() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

unsigned host_threads(const tusq_opts &o) {
    unsigned t = o.host_threads ? o.host_threads : std::thread::hardware_concurrency();
    return t ? t : 1;
}

bool is_cx(uint8_t kind) { return kind == TUSQ_CX; }
bool is_two_qubit(uint8_t kind) { return kind == TUSQ_CX || kind == TUSQ_UNITARY2; }
bool is_measure(uint8_t kind) { return kind == TUSQ_MEASURE || kind == TUSQ_MEASURE_RESET; }
bool has_measure(const Circuit &c) {
    for (const Gate &g : c.gates)
        if (is_measure(g.kind)) return true;
    return false;
}

void gate_matrix(const Circuit &circ, const Gate &g, cd m[4]) {
    const cd i(0.0, 1.0);
    const double h = g.p[0] * 0.5;
    switch (g.kind) {
    case TUSQ_UNITARY1: std::copy(circ.umats.begin() + g.umat, circ.umats.begin() + g.umat + 4, m); return;
    case TUSQ_U3: {
        const double c = std::cos(g.p[0] * 0.5), s = std::sin(g.p[0] * 0.5);
        m[0] = c;
        m[1] = -std::polar(1.0, g.p[2]) * s;
        m[2] = std::polar(1.0, g.p[1]) * s;
        m[3] = std::polar(1.0, g.p[1] + g.p[2]) * c;
        return;
    }
    case TUSQ_RX: m[0] = std::cos(h); m[1] = -i * std::sin(h); m[2] = m[1]; m[3] = m[0]; return;
    case TUSQ_RY: m[0] = std::cos(h); m[1] = -std::sin(h); m[2] = std::sin(h); m[3] = m[0]; return;
    case TUSQ_RZ: m[0] = std::polar(1.0, -h); m[1] = 0.0; m[2] = 0.0; m[3] = std::polar(1.0, h); return;
    case TUSQ_H: {
        const double r = 0.70710678118654752440;
        m[0] = r; m[1] = r; m[2] = r; m[3] = -r;
        return;
    }
    case TUSQ_S: m[0] = 1.0; m[1] = 0.0; m[2] = 0.0; m[3] = i; return;
    case TUSQ_SDG: m[0] = 1.0; m[1] = 0.0; m[2] = 0.0; m[3] = -i; return;
    case TUSQ_T: m[0] = 1.0; m[1] = 0.0; m[2] = 0.0; m[3] = std::polar(1.0, M_PI / 4); return;
    case TUSQ_TDG: m[0] = 1.0; m[1] = 0.0; m[2] = 0.0; m[3] = std::polar(1.0, -M_PI / 4); return;
    case TUSQ_X: m[0] = 0.0; m[1] = 1.0; m[2] = 1.0; m[3] = 0.0; return;
    case TUSQ_Y: m[0] = 0.0; m[1] = -i; m[2] = i; m[3] = 0.0; return;
    case TUSQ_Z: m[0] = 1.0; m[1] = 0.0; m[2] = 0.0; m[3] = -1.0; return;
    default: fail(TUSQ_EINVAL, "gate_matrix: not a 1-qubit gate");
    }
}

// Integer thresholds: T_k = floor(2^64 * (p_1 + ... + p_k)) with the partial
// sums formed left to right in double precision, saturated at 2^64 - 1.
static void channel_thresholds(Channel &ch) {
    double acc = 0.0;
    for (int k = 0; k < ch.m; ++k) {
        acc += ch.prob[k];
        ch.thr[k] = acc >= 1.0 ? ~0ull : static_cast<uint64_t>(std::ldexp(acc, 64));
    }
}

void Circuit::finalize() {
    if (!dirty) return;
    std::vector<Channel> out;
    for (uint32_t g = 0; g < gates.size(); ++g) {
        if (gates[g].chan < 0) continue;
        Channel ch = chans[gates[g].chan];
        ch.gate = g;
        gates[g].chan = static_cast<int32_t>(out.size());
        channel_thresholds(ch);
        out.push_back(ch);
    }
    chans.swap(out);
    dirty = false;
}

// ---------------------------------------------------------------------------
// Symplectic Pauli bits used by the commutation sweep: bit 0 = X part, bit 1
// = Z part, so X = 1, Z = 2, Y = 3 and products (up to phase) are XOR.  The
// paper's outcome codes are I=0 X=1 Y=2 Z=3.
static inline uint8_t code_to_sym(uint8_t p) { return static_cast<uint8_t>(p == 1 ? 1 : p == 2 ? 3 : p == 3 ? 2 : 0); }
static inline uint8_t sym_to_code(uint8_t s) { return static_cast<uint8_t>(s == 1 ? 1 : s == 3 ? 2 : s == 2 ? 3 : 0); }

// Rules 2 and 3: a noiseless Pauli gate lets every Pauli through; RX, RY, RZ
// let through the Pauli of their own axis.  Every other 1-qubit gate stops it.
static inline bool passes(uint8_t kind, uint8_t sym) {
    switch (kind) {
    case TUSQ_X: case TUSQ_Y: case TUSQ_Z: return true;
    case TUSQ_RX: return sym == 1;
    case TUSQ_RY: return sym == 3;
    case TUSQ_RZ: return sym == 2;
    default: return false;
    }
}

namespace {

constexpr uint32_t NONE = 0xFFFFFFFFu;

// Sparse form of the paper's per-qubit stack algorithm: the only movable
// item on a qubit's stack is its top noisy Pauli, so one pending Pauli per
// qubit suffices; gates are visited only where a pending Pauli or a new
// error meets them (min-heap on the next gate index of each pending qubit).
struct Commuter {
    const Circuit &c;
    const std::vector<std::vector<uint32_t>> &qg;  // gate indices per qubit
    std::vector<uint8_t> pend;
    std::vector<uint32_t> next;
    std::vector<uint32_t> touched;
    std::vector<std::pair<uint32_t, uint32_t>> heap;  // (gate, qubit), min-heap

    Commuter(const Circuit &cc, const std::vector<std::vector<uint32_t>> &q)
        : c(cc), qg(q), pend(cc.n, 0), next(cc.n, NONE) {}

    void schedule(uint32_t q, uint32_t after) {
        const auto &v = qg[q];
        auto it = std::upper_bound(v.begin(), v.end(), after);
        next[q] = it == v.end() ? NONE : *it;
        if (next[q] != NONE) {
            heap.emplace_back(next[q], q);
            std::push_heap(heap.begin(), heap.end(), std::greater<>());
        }
    }
    void set(uint32_t q, uint8_t s) {
        if (!pend[q] && s) touched.push_back(q);
        pend[q] = s;
    }

    // codes: (channel << 4) | outcome, ascending channel
    void run(const uint32_t *codes, size_t n, std::vector<Ev> &out) {
        out.clear();
        heap.clear();
        size_t pos = 0;
        const uint32_t G = static_cast<uint32_t>(c.gates.size());
        while (true) {
            while (!heap.empty()) {
                auto [g, q] = heap.front();
                if (pend[q] && next[q] == g) break;
                std::pop_heap(heap.begin(), heap.end(), std::greater<>());
                heap.pop_back();
            }
            const uint32_t g_ev = pos < n ? c.chans[codes[pos] >> 4].gate : NONE;
            const uint32_t g_pe = heap.empty() ? NONE : heap.front().first;
            const uint32_t g = std::min(g_ev, g_pe);
            if (g == NONE) break;
            while (!heap.empty() && heap.front().first == g) {
                std::pop_heap(heap.begin(), heap.end(), std::greater<>());
                heap.pop_back();
            }
            const Gate &gt = c.gates[g];
            if (is_measure(gt.kind)) {
                // a measurement stops every pending Pauli on its qubits (it
                // is reported just before the layer); a layer has no channel
                const uint64_t mk = measure_mask(gt);
                for (uint32_t q = 0; q < c.n; ++q)
                    if (((mk >> q) & 1) && pend[q]) {
                        out.push_back(Ev{g, q, sym_to_code(pend[q])});
                        pend[q] = 0;
                    }
                continue;
            }
            if (gt.kind == TUSQ_UNITARY2) {
                // a general 2-qubit unitary stops the Paulis on both qubits
                for (int j = 0; j < 2; ++j)
                    if (pend[gt.q[j]]) {
                        out.push_back(Ev{g, gt.q[j], sym_to_code(pend[gt.q[j]])});
                        pend[gt.q[j]] = 0;
                    }
            } else if (is_cx(gt.kind)) {
                const uint32_t qc = gt.q[0], qt = gt.q[1];
                uint8_t sc = pend[qc], st = pend[qt];
                if (sc | st) {
                    // rules 4-6: X_c -> X_c X_t, Z_t -> Z_c Z_t
                    st = static_cast<uint8_t>(st ^ (sc & 1));
                    sc = static_cast<uint8_t>(sc ^ (st & 2));
                    set(qc, sc);
                    set(qt, st);
                }
            } else {
                const uint32_t q = gt.q[0];
                if (pend[q] && !passes(gt.kind, pend[q])) {
                    out.push_back(Ev{g, q, sym_to_code(pend[q])});
                    pend[q] = 0;
                }
            }
            if (g_ev == g) {
                const uint8_t o = static_cast<uint8_t>(codes[pos] & 15);
                ++pos;
                if (is_two_qubit(gt.kind)) {
                    set(gt.q[0], pend[gt.q[0]] ^ code_to_sym(o >> 2));
                    set(gt.q[1], pend[gt.q[1]] ^ code_to_sym(o & 3));
                } else {
                    set(gt.q[0], pend[gt.q[0]] ^ code_to_sym(o));
                }
            }
            for (int j = 0; j < (is_two_qubit(gt.kind) ? 2 : 1); ++j)
                if (pend[gt.q[j]]) schedule(gt.q[j], g);
        }
        for (uint32_t q : touched)
            if (pend[q]) {
                out.push_back(Ev{G, q, sym_to_code(pend[q])});
                pend[q] = 0;
            }
        touched.clear();
        std::sort(out.begin(), out.end(), ev_less);
    }
};

// Without commutation an error stays right after its gate (slot g + 1).
void place_uncommuted(const Circuit &c, const uint32_t *codes, size_t n, std::vector<Ev> &out) {
    out.clear();
    for (size_t i = 0; i < n; ++i) {
        const Channel &ch = c.chans[codes[i] >> 4];
        const Gate &gt = c.gates[ch.gate];
        const uint8_t o = static_cast<uint8_t>(codes[i] & 15);
        if (is_two_qubit(gt.kind)) {
            if (o >> 2) out.push_back(Ev{ch.gate + 1, gt.q[0], static_cast<uint8_t>(o >> 2)});
            if (o & 3) out.push_back(Ev{ch.gate + 1, gt.q[1], static_cast<uint8_t>(o & 3)});
        } else {
            out.push_back(Ev{ch.gate + 1, gt.q[0], o});
        }
    }
    std::sort(out.begin(), out.end(), ev_less);
}

// Depth-first leaf order: lexicographic on events, a finished list ranks
// after any event (at one position an error token precedes the gate token).
bool leaf_less(const Ev *a, size_t na, const Ev *b, size_t nb) {
    const size_t m = std::min(na, nb);
    for (size_t i = 0; i < m; ++i)
        if (!ev_eq(a[i], b[i])) return ev_less(a[i], b[i]);
    return na > nb;
}

uint64_t mix64(uint64_t h, uint64_t v) {
    h ^= v + 0x9E3779B97F4A7C15ull + (h << 6) + (h >> 2);
    h ^= h >> 31;
    h *= 0xBF58476D1CE4E5B9ull;
    return h ^ (h >> 29);
}

template <class F>
void parallel_for(unsigned nt, uint64_t n, F &&f) {
    if (nt <= 1 || n < 2) {
        f(0u, uint64_t{0}, n);
        return;
    }
    nt = static_cast<unsigned>(std::min<uint64_t>(nt, n));
    std::vector<std::thread> th;
    for (unsigned t = 0; t < nt; ++t)
        th.emplace_back([&, t] { f(t, n * t / nt, n * (t + 1) / nt); });
    for (auto &x : th) x.join();
}

// uniform integer in [0, m) by rejection on stream 1, counter (t, attempt)
uint64_t uniform_below(uint64_t seed, uint32_t t, uint64_t m) {
    const uint64_t cut = (0 - m) % m;  // 2^64 mod m
    for (uint32_t attempt = 0;; ++attempt) {
        const uint64_t v = philox_pair(seed, t, attempt, 0, STREAM_PRUNE).lo;
        if (cut == 0 || v < 0 - cut) return v % m;
    }
}

}  // namespace

Tree build_tree(const Circuit &cin, const tusq_opts &o) {
    if (o.shots == 0 || o.shots > 0xFFFFFFFFull) fail(TUSQ_EINVAL, "shots must be in [1, 2^32)");
    if (o.alpha_den == 0) fail(TUSQ_EINVAL, "alpha_den must be positive");
    const Circuit &c = cin;
    const uint64_t S = o.shots;
    const uint32_t C = static_cast<uint32_t>(c.chans.size());
    const unsigned nt = host_threads(o);
    Tree T;
    T.n = c.n;
    T.G = static_cast<uint32_t>(c.gates.size());
    T.S = S;

    // 1. error realisations: one Philox block per (shot, channel pair)
    std::vector<std::vector<uint32_t>> tcodes(nt);
    std::vector<uint32_t> cnt(S);
    std::vector<uint64_t> hash(S);
    // compact per-channel total error threshold: the hot loop only needs
    // "u < T_m" (an error happened) before looking at the channel itself
    std::vector<uint64_t> any_err(C + 1, 0);
    for (uint32_t ci = 0; ci < C; ++ci) any_err[ci] = c.chans[ci].thr[c.chans[ci].m - 1];
    parallel_for(nt, S, [&](unsigned t, uint64_t lo, uint64_t hi) {
        auto &buf = tcodes[t];
        for (uint64_t j = lo; j < hi; ++j) {
            uint32_t k = 0;
            uint64_t h = 0x243F6A8885A308D3ull;
            for (uint32_t cp = 0; cp < C; cp += 2) {
                const Pair64 r = philox_pair(o.seed, cp >> 1, static_cast<uint32_t>(j), 0, STREAM_ERRORS);
                const bool e0 = r.lo < any_err[cp];
                const bool e1 = cp + 1 < C && r.hi < any_err[cp + 1];
                if (!(e0 | e1)) continue;
                for (uint32_t half = 0; half < 2 && cp + half < C; ++half) {
                    const uint64_t u = half ? r.hi : r.lo;
                    if (u >= any_err[cp + half]) continue;  // identity
                    const Channel &ch = c.chans[cp + half];
                    uint32_t out = 0;
                    while (u >= ch.thr[out]) ++out;
                    const uint32_t code = ((cp + half) << 4) | (out + 1);
                    buf.push_back(code);
                    h = mix64(h, code);
                    ++k;
                }
            }
            cnt[j] = k;
            hash[j] = mix64(h, k);
        }
    });
    std::vector<uint64_t> roff(S + 1, 0);
    for (uint64_t j = 0; j < S; ++j) roff[j + 1] = roff[j] + cnt[j];
    std::vector<uint32_t> codes(roff[S]);
    {
        uint64_t at = 0;
        for (auto &b : tcodes) {
            std::copy(b.begin(), b.end(), codes.begin() + at);
            at += b.size();
            std::vector<uint32_t>().swap(b);
        }
    }
    T.raw_shot.resize(codes.size());
    T.raw_chan.resize(codes.size());
    T.raw_out.resize(codes.size());
    for (uint64_t j = 0; j < S; ++j)
        for (uint64_t i = roff[j]; i < roff[j + 1]; ++i) {
            T.raw_shot[i] = static_cast<uint32_t>(j);
            T.raw_chan[i] = codes[i] >> 4;
            T.raw_out[i] = static_cast<uint8_t>(codes[i] & 15);
        }

    // 2. ER tallying: group shots with identical raw ERs (hash, then exact)
    auto same_raw = [&](uint64_t a, uint64_t b) {
        return cnt[a] == cnt[b] &&
               std::equal(codes.begin() + roff[a], codes.begin() + roff[a + 1], codes.begin() + roff[b]);
    };
    std::vector<uint64_t> order(S);
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(), [&](uint64_t a, uint64_t b) {
        if (hash[a] != hash[b]) return hash[a] < hash[b];
        if (cnt[a] != cnt[b]) return cnt[a] < cnt[b];
        const int r = std::memcmp(codes.data() + roff[a], codes.data() + roff[b], 4 * cnt[a]);
        if (r) {
            for (uint32_t i = 0; i < cnt[a]; ++i)
                if (codes[roff[a] + i] != codes[roff[b] + i]) return codes[roff[a] + i] < codes[roff[b] + i];
        }
        return a < b;
    });
    std::vector<uint64_t> rep, rcount;
    for (uint64_t i = 0; i < S; ++i) {
        const uint64_t j = order[i];
        if (!rep.empty() && hash[rep.back()] == hash[j] && same_raw(rep.back(), j)) {
            ++rcount.back();
        } else {
            rep.push_back(j);
            rcount.push_back(1);
        }
    }
    std::vector<uint64_t>().swap(order);
    const uint64_t U = rep.size();
    T.info.raw_unique = U;

    // 3. ER commutation of every unique raw ER
    std::vector<std::vector<uint32_t>> qg(c.n);
    for (uint32_t g = 0; g < T.G; ++g) {
        if (is_measure(c.gates[g].kind)) {
            const uint64_t mk = measure_mask(c.gates[g]);
            for (uint32_t q = 0; q < c.n; ++q)
                if ((mk >> q) & 1) qg[q].push_back(g);
            continue;
        }
        qg[c.gates[g].q[0]].push_back(g);
        if (is_two_qubit(c.gates[g].kind)) qg[c.gates[g].q[1]].push_back(g);
    }
    std::vector<std::vector<Ev>> can(U);
    parallel_for(nt, U, [&](unsigned, uint64_t lo, uint64_t hi) {
        Commuter cm(c, qg);
        std::vector<Ev> out;
        for (uint64_t u = lo; u < hi; ++u) {
            const uint64_t j = rep[u];
            if (o.commute) cm.run(codes.data() + roff[j], cnt[j], out);
            else place_uncommuted(c, codes.data() + roff[j], cnt[j], out);
            can[u] = out;
        }
    });

    // 4. re-tally canonical ERs, in depth-first leaf order
    std::vector<uint64_t> lo_(U);
    std::iota(lo_.begin(), lo_.end(), 0);
    std::sort(lo_.begin(), lo_.end(), [&](uint64_t a, uint64_t b) {
        if (leaf_less(can[a].data(), can[a].size(), can[b].data(), can[b].size())) return true;
        if (leaf_less(can[b].data(), can[b].size(), can[a].data(), can[a].size())) return false;
        return a < b;
    });
    std::vector<uint64_t> lrep, lcount;
    for (uint64_t u : lo_) {
        if (!lrep.empty()) {
            const auto &x = can[lrep.back()];
            const auto &y = can[u];
            if (x.size() == y.size() && std::equal(x.begin(), x.end(), y.begin(), ev_eq)) {
                lcount.back() += rcount[u];
                continue;
            }
        }
        lrep.push_back(u);
        lcount.push_back(rcount[u]);
    }
    const uint64_t L = lrep.size();
    T.info.canonical_unique = L;

    // 5. pruning: significant iff alpha_den * s >= alpha_num * s_max; when
    //    more than beta are insignificant, keep beta of them chosen uniformly
    //    without replacement, standing in for all of their shots.
    std::vector<uint8_t> keep(L, 0);
    std::vector<uint64_t> shots(L, 0), wnum(L, 0), wden(L, 0);
    const uint64_t smax = L ? *std::max_element(lcount.begin(), lcount.end()) : 0;
    T.info.s_max = smax;
    std::vector<uint64_t> insig;
    for (uint64_t i = 0; i < L; ++i) {
        const bool sig = !o.prune || uint64_t(o.alpha_den) * lcount[i] >= uint64_t(o.alpha_num) * smax;
        if (sig) {
            keep[i] = 1;
            shots[i] = wnum[i] = lcount[i];
            wden[i] = S;
        } else {
            insig.push_back(i);
        }
    }
    T.info.significant = L - insig.size();
    T.info.insignificant = insig.size();
    uint64_t s_ins = 0;
    for (uint64_t i : insig) s_ins += lcount[i];
    T.info.s_insig = s_ins;
    if (insig.size() <= o.beta) {
        for (uint64_t i : insig) {
            keep[i] = 1;
            shots[i] = wnum[i] = lcount[i];
            wden[i] = S;
        }
        T.info.d_selected = s_ins;
    } else {
        std::vector<uint64_t> perm(insig.size());
        std::iota(perm.begin(), perm.end(), 0);
        for (uint32_t t = 0; t < o.beta; ++t) {
            const uint64_t r = uniform_below(o.seed, t, perm.size() - t);
            std::swap(perm[t], perm[t + r]);
        }
        perm.resize(o.beta);
        std::sort(perm.begin(), perm.end());
        uint64_t D = 0;
        for (uint64_t p : perm) D += lcount[insig[p]];
        T.info.d_selected = D;
        // shots by largest remainder of s_I * s_j / D (ties: earlier leaf)
        std::vector<uint64_t> rem(perm.size());
        uint64_t given = 0;
        for (size_t t = 0; t < perm.size(); ++t) {
            const uint64_t i = insig[perm[t]];
            const uint64_t num = s_ins * lcount[i];
            keep[i] = 1;
            wnum[i] = num;
            wden[i] = D * S;
            shots[i] = num / D;
            rem[t] = num % D;
            given += shots[i];
        }
        std::vector<size_t> by(perm.size());
        std::iota(by.begin(), by.end(), 0);
        std::stable_sort(by.begin(), by.end(), [&](size_t a, size_t b) { return rem[a] > rem[b]; });
        for (uint64_t u = 0; u < s_ins - given; ++u) shots[insig[perm[by[u]]]] += 1;
    }

    T.off.push_back(0);
    for (uint64_t i = 0; i < L; ++i) {
        if (!keep[i]) continue;
        const auto &e = can[lrep[i]];
        T.ev.insert(T.ev.end(), e.begin(), e.end());
        T.off.push_back(T.ev.size());
        T.count.push_back(lcount[i]);
        T.shots.push_back(shots[i]);
        T.wnum.push_back(wnum[i]);
        T.wden.push_back(wden[i]);
    }
    T.info.n_leaves = T.count.size();
    T.info.n_events = T.ev.size();
    T.info.n_raw_events = codes.size();
    return T;
}

std::vector<uint8_t> serialize_tree(const Tree &t) {
    std::vector<uint8_t> b;
    auto put = [&](const void *p, size_t k) {
        const uint8_t *c = static_cast<const uint8_t *>(p);
        b.insert(b.end(), c, c + k);
    };
    const uint32_t hdr[4] = {0x51535554u, 1u, t.n, t.G};
    put(hdr, 16);
    put(&t.S, 8);
    const uint64_t L = t.leaves();
    put(&L, 8);
    for (uint64_t l = 0; l < L; ++l) {
        put(&t.count[l], 8);
        put(&t.shots[l], 8);
        put(&t.wnum[l], 8);
        put(&t.wden[l], 8);
        const uint32_t ne = static_cast<uint32_t>(t.nev(l));
        put(&ne, 4);
        for (uint32_t e = 0; e < ne; ++e) {
            const Ev &v = t.evs(l)[e];
            put(&v.slot, 4);
            put(&v.qubit, 4);
            put(&v.pauli, 1);
        }
    }
    return b;
}

}  // namespace tusq
