/*
 * tusq_oracle.c -- plain CPU oracle for noisy statevector simulation with
 * error tallying, error commutation, pruning and depth-first tree traversal.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no source,
 * header, table or helper with the GPU engine; both read the same circuit
 * description and nothing else.
 *
 * Everything is deliberately simple: complex128 amplitudes, one gate at a
 * time, left-to-right FP64 sums, and the error-commutation stage implemented
 * literally with one stack per qubit.  Where the paper (TUSQ, arXiv
 * 2508.04880) leaves a choice open, the reading taken is stated next to the
 * code; the list of readings is kept with the project's design notes.
 *
 * Paper map for the citations below:
 *   Sec. II, Eq. (1)        statevector update psi' = U psi
 *   Sec. II (depolarising)  rho' = (1-p) rho + p/3 (X rho X + Y rho Y + Z rho Z);
 *                           read as a weighted mixture of fixed-Pauli circuits
 *   Sec. III-A.1            error realisations (ERs): sample every channel
 *                           per shot; tally identical ERs
 *   Sec. III-A.2/3          ER commutation rules 1-6 and the per-qubit stack
 *                           greedy algorithm
 *   Sec. III-A.4, Eq. (2)   pruning with alpha, beta; S_final
 *   Sec. III-B              DFTT: forward = U, backtrack = U^-1
 *   Sec. III-B.1            T_dftt = 2|E|, T_naive = N_l * h
 *   Sec. III-B.2, Eq. (3)   non-invertible edges (mid-circuit measurement
 *                           layers), DFTT+Caching with a LIFO cache of
 *                           capacity K, alpha(K)
 *
 * Parity status: every function here is pinned by tests against values
 * that do not come from this file (published Philox vectors, density-matrix
 * simulation, closed forms, brute-force operator identities).  The pruning
 * selection follows a reading of the paper's "randomly sample" (uniform
 * without replacement) and is pinned by what that reading fixes: every
 * beta-subset equally likely (chi-square over thousands of seeds), uniform
 * bounded draws where a modulo bias would be gross, and the largest-remainder
 * shots against hand-worked cases and a brute-force closest apportionment.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Gate kinds (the oracle's own numbering; the Python wrapper maps names).   */
enum { OK_U3 = 0, OK_RX, OK_RY, OK_RZ, OK_H, OK_S, OK_SDG, OK_T, OK_TDG,
       OK_X, OK_Y, OK_Z, OK_CX, OK_M, OK_MR, OK_U1M, OK_U2M, OK_NKINDS };
/* OK_U1M / OK_U2M: a caller's 2x2 / 4x4 unitary, read from mats at
 * mat_off[g] as row-major (re, im) pairs; the 4x4's basis index is
 * 2 * bit(q0) + bit(q1).  No Pauli moves through either. */
/* OK_M / OK_MR: a layer of concurrent Z-basis measurements (MR: the measured
 * qubits are reset to |0> afterwards).  Its qubit set is a 64-bit mask held
 * as q0 (low word) and q1 (high word); at most 8 qubits, no noise channel. */
#define MAX_MEASURED 8

/* Pauli codes: I=0, X=1, Y=2, Z=3. */

typedef struct {
    uint32_t n, G;
    const uint8_t *kind;
    const uint32_t *q0, *q1;
    const double *params;   /* 3 per gate */
    const uint8_t *nprob;   /* 0, 3 or 15 per gate */
    const double *probs;    /* concatenated channel probabilities */
    const double *mats;     /* matrices of OK_U1M / OK_U2M gates */
    const uint64_t *mat_off;/* per gate: offset into mats (doubles) */
} oc_circuit;

static int oracle_threads = 1;
void oc_set_threads(int t) { oracle_threads = t > 0 ? t : 1; }
int oc_get_threads(void) { return oracle_threads; }

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, from Salmon, Moraes, Dror and Shaw, "Parallel random       */
/* numbers: as easy as 1, 2, 3" (SC'11): ten rounds of two 32x32->64        */
/* multiplies with the key bumped by the Weyl constants between rounds.      */
void oc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* One 64-bit value: counter (sub, primary, aux, stream), key = seed; half 0
 * is words 0|1<<32, half 1 is words 2|3<<32.  Streams: 0 error sampling,
 * 1 pruning selection, 2 shot sampling. */
static uint64_t draw64(uint64_t seed, uint32_t sub, uint32_t primary, uint32_t aux,
                       uint32_t stream, int half)
{
    uint32_t ctr[4] = {sub, primary, aux, stream};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t o[4];
    oc_philox(ctr, key, o);
    if (half == 0) return (uint64_t)o[0] | ((uint64_t)o[1] << 32);
    return (uint64_t)o[2] | ((uint64_t)o[3] << 32);
}

/* Pauli-twirled thermal relaxation, Sec. VI-A Eq. (4): over a duration t with
 * relaxation time T1 and dephasing time T2,
 *   pX = pY = (1 - e^{-t/T1}) / 4,   pZ = (1 - e^{-t/T2}) / 2 - (1 - e^{-t/T1}) / 4
 * (1 - e^{-x} evaluated as -expm1(-x)).  Returns -1 unless t >= 0, T1 > 0 and
 * 0 < T2 <= 2 T1. */
int oc_thermal_probs(double t, double t1, double t2, double out[3])
{
    if (!(t >= 0.0 && t1 > 0.0 && t2 > 0.0 && t2 <= 2.0 * t1)) return -1;
    double a = -expm1(-t / t1), b = -expm1(-t / t2);
    out[0] = a / 4.0;
    out[1] = a / 4.0;
    out[2] = b / 2.0 - a / 4.0;
    if (out[2] < 0.0) out[2] = 0.0;
    return 0;
}

/* The same channel acting independently on both qubits of a CX: outcome
 * k = 4a + b (a on the control, b on the target) has probability q_a q_b,
 * q = (1 - pX - pY - pZ, pX, pY, pZ); out[k - 1] for k = 1..15. */
int oc_thermal_probs2(double t, double t1, double t2, double out[15])
{
    double p[3];
    if (oc_thermal_probs(t, t1, t2, p)) return -1;
    double q[4] = {1.0 - p[0] - p[1] - p[2], p[0], p[1], p[2]};
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b)
            if (a || b) out[4 * a + b - 1] = q[a] * q[b];
    return 0;
}

/* Integer cumulative thresholds of a Pauli channel: S_k is the plain
 * left-to-right double sum p_1 + ... + p_k; C_k = floor(S_k * 2^64), or
 * 2^64 - 1 once S_k reaches 1.  A uniform u64 u selects the smallest k with
 * u < C_k, and the identity when u >= C_m. */
void oc_thresholds(const double *p, int m, uint64_t *C)
{
    double s = 0.0;
    for (int k = 0; k < m; ++k) {
        s = s + p[k];
        C[k] = (s >= 1.0) ? UINT64_MAX : (uint64_t)ldexp(s, 64);
    }
}

static int pick_outcome(uint64_t u, const uint64_t *C, int m)
{
    for (int k = 0; k < m; ++k)
        if (u < C[k]) return k + 1;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Prepared circuit: channel table.                                         */
typedef struct {
    const oc_circuit *c;
    uint32_t C;            /* number of channels */
    int32_t *gate_chan;    /* per gate: channel index or -1 */
    uint32_t *chan_gate;   /* per channel: gate index */
    uint8_t *chan_m;       /* 3 or 15 */
    uint64_t *chan_thr;    /* 15 per channel */
} prep_t;

static int is_two_qubit(uint8_t k) { return k == OK_CX || k == OK_U2M; }
static int is_measure(uint8_t k) { return k == OK_M || k == OK_MR; }
static uint64_t meas_mask(const oc_circuit *c, uint32_t g)
{
    return (uint64_t)c->q0[g] | ((uint64_t)c->q1[g] << 32);
}
static int has_measure(const oc_circuit *c)
{
    for (uint32_t g = 0; g < c->G; ++g) if (is_measure(c->kind[g])) return 1;
    return 0;
}

static int validate(const oc_circuit *c)
{
    size_t off = 0;
    for (uint32_t g = 0; g < c->G; ++g) {
        if (c->kind[g] >= OK_NKINDS) return -1;
        if (is_measure(c->kind[g])) {
            uint64_t mk = meas_mask(c, g);
            if (!mk || (c->n < 64 && (mk >> c->n)) || __builtin_popcountll(mk) > MAX_MEASURED ||
                c->nprob[g])
                return -1;
            continue;
        }
        if (c->q0[g] >= c->n) return -1;
        if (is_two_qubit(c->kind[g]) && (c->q1[g] >= c->n || c->q1[g] == c->q0[g])) return -1;
        if ((c->kind[g] == OK_U1M || c->kind[g] == OK_U2M) && !(c->mats && c->mat_off)) return -1;
        int m = c->nprob[g];
        if (m != 0 && m != (is_two_qubit(c->kind[g]) ? 15 : 3)) return -1;
        double s = 0.0;
        for (int k = 0; k < m; ++k) {
            double p = c->probs[off + k];
            if (!(p >= 0.0)) return -1;
            s += p;
        }
        if (s > 1.0 + 1e-12) return -1;
        off += m;
    }
    return 0;
}

static int prep_init(prep_t *P, const oc_circuit *c)
{
    memset(P, 0, sizeof(*P));
    P->c = c;
    if (validate(c)) return -1;
    P->gate_chan = malloc(sizeof(int32_t) * (c->G + 1));
    uint32_t C = 0;
    for (uint32_t g = 0; g < c->G; ++g) C += c->nprob[g] ? 1 : 0;
    P->C = C;
    P->chan_gate = malloc(sizeof(uint32_t) * (C + 1));
    P->chan_m = malloc(C + 1);
    P->chan_thr = malloc(sizeof(uint64_t) * 15 * (C + 1));
    size_t off = 0;
    uint32_t ch = 0;
    for (uint32_t g = 0; g < c->G; ++g) {
        int m = c->nprob[g];
        if (m) {
            P->gate_chan[g] = (int32_t)ch;
            P->chan_gate[ch] = g;
            P->chan_m[ch] = (uint8_t)m;
            oc_thresholds(c->probs + off, m, P->chan_thr + 15 * (size_t)ch);
            ++ch;
        } else {
            P->gate_chan[g] = -1;
        }
        off += m;
    }
    return 0;
}

static void prep_free(prep_t *P)
{
    free(P->gate_chan); free(P->chan_gate); free(P->chan_m); free(P->chan_thr);
}

/* ------------------------------------------------------------------------ */
/* ER sampling (Sec. III-A.1): every channel sampled for every shot.  Shot j,
 * channel c uses counter (c >> 1, j, 0, stream 0), half c & 1.  A raw ER is
 * the list of (channel, outcome) with a non-identity outcome. */
static int sample_shot(const prep_t *P, uint64_t seed, uint32_t shot, uint32_t *chan,
                       uint8_t *out)
{
    int cnt = 0;
    for (uint32_t c = 0; c < P->C; ++c) {
        uint64_t u = draw64(seed, c >> 1, shot, 0, 0, (int)(c & 1));
        int k = pick_outcome(u, P->chan_thr + 15 * (size_t)c, P->chan_m[c]);
        if (k) { chan[cnt] = c; out[cnt] = (uint8_t)k; ++cnt; }
    }
    return cnt;
}

int oc_sample_shot(const oc_circuit *c, uint64_t seed, uint32_t shot, uint32_t *chan,
                   uint8_t *out, uint32_t *n_out)
{
    prep_t P;
    if (prep_init(&P, c)) return -1;
    *n_out = (uint32_t)sample_shot(&P, seed, shot, chan, out);
    prep_free(&P);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* ER commutation (Sec. III-A.2/3), implemented literally: one stack per
 * qubit holding noiseless gates (value >= 0: the gate index) and noisy Pauli
 * gates (value < 0: -code).  A noisy Pauli on a stack top moves past a
 * noiseless gate when the paper's rules let it:
 *   rule 2: through a noiseless Pauli gate;
 *   rule 3: X through RX, Y through RY, Z through RZ;
 *   rules 4-6: through CX, becoming its conjugate (X_c -> X_c X_t,
 *              Z_t -> Z_c Z_t, Y_c -> Y_c X_t, Y_t -> Z_c Y_t).
 * Any other gate keeps the noisy gate below it.  A new noisy gate merges with
 * a noisy stack top (rule 1, products taken up to phase); a product equal to
 * the identity disappears.  Reading: gates outside rules 1-6 (U3, H, S, T ...)
 * block, and a Pauli left below gate g is reported at "slot g", i.e. just
 * before g; those still on top at the end are at slot G. */

typedef struct { int32_t *data; uint32_t size; uint32_t cap; } stack_t_;

static int pauli_mul(int a, int b)
{
    /* symplectic (x, z): X=(1,0) Y=(1,1) Z=(0,1); product up to phase */
    int ax = (a == 1 || a == 2), az = (a == 2 || a == 3);
    int bx = (b == 1 || b == 2), bz = (b == 2 || b == 3);
    int x = ax ^ bx, z = az ^ bz;
    if (x && !z) return 1;
    if (x && z) return 2;
    if (!x && z) return 3;
    return 0;
}

/* Conjugate the pair (P on control, Q on target) through CX. */
static void cx_conjugate(int pc, int pt, int *oc, int *ot)
{
    int rc = 0, rt = 0;
    /* X on control -> X_c X_t ; Z on control -> Z_c */
    /* X on target  -> X_t     ; Z on target  -> Z_c Z_t */
    int cx = (pc == 1 || pc == 2), cz = (pc == 2 || pc == 3);
    int tx = (pt == 1 || pt == 2), tz = (pt == 2 || pt == 3);
    if (cx) { rc = pauli_mul(rc, 1); rt = pauli_mul(rt, 1); }
    if (cz) { rc = pauli_mul(rc, 3); }
    if (tx) { rt = pauli_mul(rt, 1); }
    if (tz) { rc = pauli_mul(rc, 3); rt = pauli_mul(rt, 3); }
    *oc = rc; *ot = rt;
}

static int passes_1q(uint8_t kind, int p)
{
    switch (kind) {
    case OK_X: case OK_Y: case OK_Z: return 1;      /* rule 2 */
    case OK_RX: return p == 1;                       /* rule 3 */
    case OK_RY: return p == 2;
    case OK_RZ: return p == 3;
    default: return 0;
    }
}

static void push(stack_t_ *s, int32_t v) { s->data[s->size++] = v; }
static int32_t top(const stack_t_ *s) { return s->size ? s->data[s->size - 1] : INT32_MAX; }

static void noisy_arrive(stack_t_ *s, int p)
{
    if (!p) return;
    int32_t t = top(s);
    if (s->size && t < 0) {
        int r = pauli_mul(-t, p);
        if (r) s->data[s->size - 1] = -r;
        else s->size--;
    } else {
        push(s, -p);
    }
}

/* Event key: (slot << 32) | (qubit << 8) | pauli -- integer order equals
 * (slot, qubit, pauli) order. */
#define EVKEY(slot, q, p) (((uint64_t)(slot) << 32) | ((uint64_t)(q) << 8) | (uint64_t)(p))
#define EV_SLOT(k) ((uint32_t)((k) >> 32))
#define EV_QUBIT(k) ((uint32_t)(((k) >> 8) & 0xFFFFFFu))
#define EV_PAULI(k) ((int)((k) & 0xFFu))

static int cmp_u64(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}

typedef struct {
    stack_t_ *st;  /* n stacks */
    int32_t *pool;
} stacks_t;

static void stacks_alloc(stacks_t *S, const oc_circuit *c)
{
    S->st = calloc(c->n, sizeof(stack_t_));
    size_t *cnt = calloc(c->n, sizeof(size_t));
    for (uint32_t g = 0; g < c->G; ++g) {
        if (is_measure(c->kind[g])) {
            for (uint32_t q = 0; q < c->n; ++q)
                if ((meas_mask(c, g) >> q) & 1) cnt[q]++;
            continue;
        }
        cnt[c->q0[g]]++;
        if (is_two_qubit(c->kind[g])) cnt[c->q1[g]]++;
    }
    size_t tot = 0;
    for (uint32_t q = 0; q < c->n; ++q) tot += 2 * cnt[q] + 2;
    S->pool = malloc(sizeof(int32_t) * tot);
    size_t off = 0;
    for (uint32_t q = 0; q < c->n; ++q) {
        S->st[q].data = S->pool + off;
        S->st[q].cap = (uint32_t)(2 * cnt[q] + 2);
        off += 2 * cnt[q] + 2;
    }
    free(cnt);
}

static void stacks_free(stacks_t *S) { free(S->st); free(S->pool); }

/* Returns the number of canonical events written to keys (capacity n*(G+1)). */
static int commute_one(const prep_t *P, stacks_t *S, int nraw, const uint32_t *chan,
                       const uint8_t *outc, uint64_t *keys)
{
    const oc_circuit *c = P->c;
    for (uint32_t q = 0; q < c->n; ++q) S->st[q].size = 0;
    int ri = 0;
    for (uint32_t g = 0; g < c->G; ++g) {
        uint8_t k = c->kind[g];
        if (is_measure(k)) {
            /* no noisy gate moves through a measurement of its qubit: it
             * stays below and is reported at the measurement's slot */
            for (uint32_t q = 0; q < c->n; ++q)
                if ((meas_mask(c, g) >> q) & 1) push(&S->st[q], (int32_t)g);
            continue;
        }
        if (k == OK_U2M) {
            /* a general 2-qubit unitary stops the Paulis on both qubits */
            push(&S->st[c->q0[g]], (int32_t)g);
            push(&S->st[c->q1[g]], (int32_t)g);
        } else if (is_two_qubit(k)) {
            stack_t_ *sc = &S->st[c->q0[g]], *stt = &S->st[c->q1[g]];
            int pc = 0, pt = 0;
            if (sc->size && top(sc) < 0) { pc = -top(sc); sc->size--; }
            if (stt->size && top(stt) < 0) { pt = -top(stt); stt->size--; }
            push(sc, (int32_t)g);
            push(stt, (int32_t)g);
            int oc, ot;
            cx_conjugate(pc, pt, &oc, &ot);
            if (oc) push(sc, -oc);
            if (ot) push(stt, -ot);
        } else {
            stack_t_ *s = &S->st[c->q0[g]];
            if (s->size && top(s) < 0 && passes_1q(k, -top(s))) {
                int32_t p = top(s);
                s->size--;
                push(s, (int32_t)g);
                push(s, p);
            } else {
                push(s, (int32_t)g);
            }
        }
        /* noisy gate that follows gate g */
        int32_t ch = P->gate_chan[g];
        if (ch >= 0 && ri < nraw && chan[ri] == (uint32_t)ch) {
            int o = outc[ri++];
            if (is_two_qubit(k)) {
                noisy_arrive(&S->st[c->q0[g]], o >> 2);
                noisy_arrive(&S->st[c->q1[g]], o & 3);
            } else {
                noisy_arrive(&S->st[c->q0[g]], o);
            }
        }
    }
    int ne = 0;
    for (uint32_t q = 0; q < c->n; ++q) {
        stack_t_ *s = &S->st[q];
        for (uint32_t i = 0; i < s->size; ++i) {
            if (s->data[i] < 0) {
                uint32_t slot = c->G;
                for (uint32_t j = i + 1; j < s->size; ++j)
                    if (s->data[j] >= 0) { slot = (uint32_t)s->data[j]; break; }
                keys[ne++] = EVKEY(slot, q, -s->data[i]);
            }
        }
    }
    qsort(keys, (size_t)ne, sizeof(uint64_t), cmp_u64);
    return ne;
}

/* Without commutation, a raw ER's Paulis sit right after their gate, i.e.
 * at slot g + 1 (before the next gate in circuit order); several on one
 * qubit at one slot are impossible because each gate has one channel. */
static int no_commute_one(const prep_t *P, int nraw, const uint32_t *chan,
                          const uint8_t *outc, uint64_t *keys)
{
    const oc_circuit *c = P->c;
    int ne = 0;
    for (int i = 0; i < nraw; ++i) {
        uint32_t g = P->chan_gate[chan[i]];
        int o = outc[i];
        if (is_two_qubit(c->kind[g])) {
            if (o >> 2) keys[ne++] = EVKEY(g + 1, c->q0[g], o >> 2);
            if (o & 3) keys[ne++] = EVKEY(g + 1, c->q1[g], o & 3);
        } else {
            keys[ne++] = EVKEY(g + 1, c->q0[g], o);
        }
    }
    qsort(keys, (size_t)ne, sizeof(uint64_t), cmp_u64);
    return ne;
}

int oc_commute(const oc_circuit *c, uint32_t nraw, const uint32_t *chan, const uint8_t *outc,
               int commute, uint32_t *slot, uint32_t *qubit, uint8_t *pauli, uint32_t *n_out)
{
    prep_t P;
    if (prep_init(&P, c)) return -1;
    uint64_t *keys = malloc(sizeof(uint64_t) * ((size_t)c->n * (c->G + 2) + 2 * nraw + 1));
    int ne;
    if (commute) {
        stacks_t S;
        stacks_alloc(&S, c);
        ne = commute_one(&P, &S, (int)nraw, chan, outc, keys);
        stacks_free(&S);
    } else {
        ne = no_commute_one(&P, (int)nraw, chan, outc, keys);
    }
    for (int i = 0; i < ne; ++i) {
        slot[i] = EV_SLOT(keys[i]); qubit[i] = EV_QUBIT(keys[i]); pauli[i] = (uint8_t)EV_PAULI(keys[i]);
    }
    *n_out = (uint32_t)ne;
    free(keys);
    prep_free(&P);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Leaf order: lexicographic over event keys, an exhausted list ranking above
 * every event (so the noiseless leaf is last).  This is a depth-first order
 * of the token trie, because at a given position an event token comes
 * before the gate token of the same slot. */
static int leaf_cmp(const uint64_t *a, uint64_t na, const uint64_t *b, uint64_t nb)
{
    uint64_t i = 0;
    for (;; ++i) {
        if (i == na && i == nb) return 0;
        if (i == na) return 1;
        if (i == nb) return -1;
        if (a[i] != b[i]) return a[i] < b[i] ? -1 : 1;
    }
}

typedef struct {
    uint32_t n, G;
    uint64_t S;
    uint64_t n_leaves;
    uint64_t *ev_off;
    uint64_t *ev_key;
    uint64_t *count, *shots, *wnum, *wden;
    uint64_t stats[8]; /* raw unique, canonical unique, sig, insig, s_I, D, s_max, kept */
    uint64_t n_raw;
    uint32_t *raw_shot, *raw_chan;
    uint8_t *raw_out;
} oc_tree;

/* sort contexts (sorting is single threaded) */
static const uint64_t *g_off;
static const uint64_t *g_key;
static const uint64_t *g_raw_off;
static const uint64_t *g_raw_code;

static int cmp_raw(const void *pa, const void *pb)
{
    uint64_t a = *(const uint64_t *)pa, b = *(const uint64_t *)pb;
    uint64_t na = g_raw_off[a + 1] - g_raw_off[a], nb = g_raw_off[b + 1] - g_raw_off[b];
    const uint64_t *x = g_raw_code + g_raw_off[a], *y = g_raw_code + g_raw_off[b];
    for (uint64_t i = 0; i < na && i < nb; ++i)
        if (x[i] != y[i]) return x[i] < y[i] ? -1 : 1;
    if (na != nb) return na < nb ? -1 : 1;
    return (a > b) - (a < b);
}

static int cmp_leaf_idx(const void *pa, const void *pb)
{
    uint64_t a = *(const uint64_t *)pa, b = *(const uint64_t *)pb;
    int r = leaf_cmp(g_key + g_off[a], g_off[a + 1] - g_off[a], g_key + g_off[b],
                     g_off[b + 1] - g_off[b]);
    if (r) return r;
    return (a > b) - (a < b);
}

/* Uniform integer in [0, m) from stream 1 by rejection: draw with counter
 * (t, attempt, 0, 1), half 0; accept when below 2^64 - (2^64 mod m). */
static uint64_t bounded(uint64_t seed, uint32_t t, uint64_t m)
{
    uint64_t rem = (0 - m) % m;  /* 2^64 mod m */
    for (uint32_t attempt = 0;; ++attempt) {
        uint64_t v = draw64(seed, t, attempt, 0, 1, 0);
        if (rem == 0 || v < (0 - rem)) return v % m;
    }
}

/* Pruning selection (Sec. III-A.4 says only that beta of the insignificant
 * circuits are sampled at random; read as uniformly without replacement):
 * a partial Fisher-Yates shuffle of the positions 0 .. nins-1 whose step t
 * swaps position t with t + bounded(seed, t, nins - t).  out[0 .. beta)
 * receives the chosen positions in ascending order; out holds nins entries
 * (scratch beyond beta).  Requires beta <= nins. */
void oc_prune_select(uint64_t seed, uint64_t nins, uint32_t beta, uint64_t *out)
{
    for (uint64_t t = 0; t < nins; ++t) out[t] = t;
    for (uint32_t t = 0; t < beta; ++t) {
        uint64_t r = bounded(seed, t, nins - t);
        uint64_t tmp = out[t]; out[t] = out[t + r]; out[t + r] = tmp;
    }
    qsort(out, beta, sizeof(uint64_t), cmp_u64);
}

/* Integer shots of the beta selected circuits (Eq. (2): the insignificant
 * shots sI shared in proportion to the selected counts cnt, D = their sum):
 * the quota sI * cnt[t] / D is floored, and the sI - sum(floors) units left
 * go one each to the largest remainders (sI * cnt[t]) mod D, a tie to the
 * earlier circuit (Hamilton's largest-remainder method). */
void oc_apportion(uint64_t sI, const uint64_t *cnt, uint32_t beta, uint64_t *out)
{
    uint64_t D = 0, given = 0;
    for (uint32_t t = 0; t < beta; ++t) D += cnt[t];
    uint64_t *rem = malloc(sizeof(uint64_t) * (beta + 1));
    uint8_t *got = calloc(beta + 1, 1);
    for (uint32_t t = 0; t < beta; ++t) {
        uint64_t num = sI * cnt[t];
        out[t] = num / D; rem[t] = num % D; given += out[t];
    }
    uint64_t left = sI - given;
    for (uint64_t u = 0; u < left; ++u) {
        int64_t best = -1;
        for (uint32_t t = 0; t < beta; ++t)
            if (!got[t] && (best < 0 || rem[t] > rem[best])) best = t;
        got[best] = 1;
        out[best] += 1;
    }
    free(got); free(rem);
}

/* bounded() for tests of the rejection rule */
uint64_t oc_bounded(uint64_t seed, uint32_t t, uint64_t m) { return bounded(seed, t, m); }

void oc_tree_free(oc_tree *t)
{
    if (!t) return;
    free(t->ev_off); free(t->ev_key); free(t->count); free(t->shots); free(t->wnum);
    free(t->wden); free(t->raw_shot); free(t->raw_chan); free(t->raw_out);
    free(t);
}

/* Build the tree of circuits to simulate: sample, tally, commute, re-tally,
 * prune (Sec. III-A), then order the leaves depth-first. */
oc_tree *oc_ecm(const oc_circuit *c, uint64_t S, uint64_t seed, int commute, int prune,
                uint32_t a_num, uint32_t a_den, uint32_t beta)
{
    if (S == 0 || S > 0xFFFFFFFFull || a_den == 0) return NULL;
    prep_t P;
    if (prep_init(&P, c)) return NULL;
    oc_tree *T = calloc(1, sizeof(oc_tree));
    T->n = c->n; T->G = c->G; T->S = S;

    /* 1. raw ERs, per shot (blocks of shots per thread, concatenated in
     *    shot order) */
    int nth = oracle_threads;
    uint64_t *cnt = calloc(S + 1, sizeof(uint64_t));
    uint64_t **buf = calloc((size_t)nth, sizeof(uint64_t *));
    uint64_t *bufn = calloc((size_t)nth, sizeof(uint64_t));
#pragma omp parallel num_threads(nth)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        uint64_t lo = S * (uint64_t)tid / (uint64_t)nth, hi = S * (uint64_t)(tid + 1) / (uint64_t)nth;
        uint64_t cap = 1024, len = 0;
        uint64_t *b = malloc(sizeof(uint64_t) * cap);
        uint32_t *ch = malloc(sizeof(uint32_t) * (P.C + 1));
        uint8_t *oo = malloc(P.C + 1);
        for (uint64_t j = lo; j < hi; ++j) {
            int k = sample_shot(&P, seed, (uint32_t)j, ch, oo);
            cnt[j] = (uint64_t)k;
            if (len + (uint64_t)k > cap) {
                while (len + (uint64_t)k > cap) cap *= 2;
                b = realloc(b, sizeof(uint64_t) * cap);
            }
            for (int i = 0; i < k; ++i) b[len++] = ((uint64_t)ch[i] << 8) | oo[i];
        }
        buf[tid] = b; bufn[tid] = len;
        free(ch); free(oo);
    }
    uint64_t *raw_off = malloc(sizeof(uint64_t) * (S + 1));
    raw_off[0] = 0;
    for (uint64_t j = 0; j < S; ++j) raw_off[j + 1] = raw_off[j] + cnt[j];
    uint64_t nraw = raw_off[S];
    uint64_t *raw_code = malloc(sizeof(uint64_t) * (nraw + 1));
    {
        uint64_t o = 0;
        for (int t = 0; t < nth; ++t) {
            memcpy(raw_code + o, buf[t], sizeof(uint64_t) * bufn[t]);
            o += bufn[t];
            free(buf[t]);
        }
    }
    free(buf); free(bufn); free(cnt);
    T->n_raw = nraw;
    T->raw_shot = malloc(sizeof(uint32_t) * (nraw + 1));
    T->raw_chan = malloc(sizeof(uint32_t) * (nraw + 1));
    T->raw_out = malloc(nraw + 1);
    for (uint64_t j = 0; j < S; ++j)
        for (uint64_t i = raw_off[j]; i < raw_off[j + 1]; ++i) {
            T->raw_shot[i] = (uint32_t)j;
            T->raw_chan[i] = (uint32_t)(raw_code[i] >> 8);
            T->raw_out[i] = (uint8_t)(raw_code[i] & 0xFF);
        }

    /* 2. tally raw ERs: sort shots by their ER, count runs */
    uint64_t *ord = malloc(sizeof(uint64_t) * S);
    for (uint64_t j = 0; j < S; ++j) ord[j] = j;
    g_raw_off = raw_off; g_raw_code = raw_code;
    qsort(ord, S, sizeof(uint64_t), cmp_raw);
    uint64_t U = 0;
    uint64_t *urep = malloc(sizeof(uint64_t) * S), *ucount = malloc(sizeof(uint64_t) * S);
    for (uint64_t i = 0; i < S; ++i) {
        uint64_t j = ord[i];
        int same = 0;
        if (U) {
            uint64_t r = urep[U - 1];
            uint64_t na = raw_off[j + 1] - raw_off[j], nb = raw_off[r + 1] - raw_off[r];
            same = (na == nb) && !memcmp(raw_code + raw_off[j], raw_code + raw_off[r], na * 8);
        }
        if (same) ucount[U - 1]++;
        else { urep[U] = j; ucount[U] = 1; ++U; }
    }
    free(ord);
    T->stats[0] = U;

    /* 3. canonical ER of every unique raw ER */
    uint64_t *cn = calloc(U + 1, sizeof(uint64_t));
    uint64_t **ck = calloc(U + 1, sizeof(uint64_t *));
#pragma omp parallel num_threads(nth)
    {
        stacks_t St;
        if (commute) stacks_alloc(&St, c);
        uint64_t *keys = malloc(sizeof(uint64_t) * ((size_t)c->n * (c->G + 2) + 2 * P.C + 2));
        uint32_t *ch = malloc(sizeof(uint32_t) * (P.C + 1));
        uint8_t *oo = malloc(P.C + 1);
#pragma omp for schedule(dynamic, 256)
        for (uint64_t u = 0; u < U; ++u) {
            uint64_t r = urep[u];
            int k = (int)(raw_off[r + 1] - raw_off[r]);
            for (int i = 0; i < k; ++i) {
                ch[i] = (uint32_t)(raw_code[raw_off[r] + i] >> 8);
                oo[i] = (uint8_t)(raw_code[raw_off[r] + i] & 0xFF);
            }
            int ne = commute ? commute_one(&P, &St, k, ch, oo, keys)
                             : no_commute_one(&P, k, ch, oo, keys);
            cn[u] = (uint64_t)ne;
            ck[u] = malloc(sizeof(uint64_t) * (ne + 1));
            memcpy(ck[u], keys, sizeof(uint64_t) * ne);
        }
        if (commute) stacks_free(&St);
        free(keys); free(ch); free(oo);
    }
    free(raw_off); free(raw_code); free(urep);

    /* 4. re-tally canonical ERs, in leaf order */
    uint64_t *coff = malloc(sizeof(uint64_t) * (U + 1));
    coff[0] = 0;
    for (uint64_t u = 0; u < U; ++u) coff[u + 1] = coff[u] + cn[u];
    uint64_t *ckey = malloc(sizeof(uint64_t) * (coff[U] + 1));
    for (uint64_t u = 0; u < U; ++u) { memcpy(ckey + coff[u], ck[u], cn[u] * 8); free(ck[u]); }
    free(ck); free(cn);
    uint64_t *lord = malloc(sizeof(uint64_t) * (U + 1));
    for (uint64_t u = 0; u < U; ++u) lord[u] = u;
    g_off = coff; g_key = ckey;
    qsort(lord, U, sizeof(uint64_t), cmp_leaf_idx);
    uint64_t L = 0;
    uint64_t *lrep = malloc(sizeof(uint64_t) * (U + 1)), *lcnt = malloc(sizeof(uint64_t) * (U + 1));
    for (uint64_t i = 0; i < U; ++i) {
        uint64_t u = lord[i];
        if (L && leaf_cmp(ckey + coff[u], coff[u + 1] - coff[u], ckey + coff[lrep[L - 1]],
                          coff[lrep[L - 1] + 1] - coff[lrep[L - 1]]) == 0) {
            lcnt[L - 1] += ucount[u];
        } else {
            lrep[L] = u; lcnt[L] = ucount[u]; ++L;
        }
    }
    free(lord); free(ucount);
    T->stats[1] = L;

    /* 5. pruning (Sec. III-A.4).  Significant iff a_den*s >= a_num*s_max.
     *    If more than beta leaves are insignificant, beta of them are drawn
     *    uniformly without replacement (partial Fisher-Yates on stream 1) and
     *    given the insignificant shots s_I in proportion to their counts. */
    uint8_t *keep = calloc(L + 1, 1);
    uint64_t *shots = calloc(L + 1, sizeof(uint64_t)), *wnum = calloc(L + 1, sizeof(uint64_t)),
             *wden = calloc(L + 1, sizeof(uint64_t));
    uint64_t smax = 0;
    for (uint64_t i = 0; i < L; ++i) if (lcnt[i] > smax) smax = lcnt[i];
    T->stats[6] = smax;
    uint64_t nsig = 0, nins = 0;
    uint64_t *ins = malloc(sizeof(uint64_t) * (L + 1));
    for (uint64_t i = 0; i < L; ++i) {
        int sig = !prune || ((uint64_t)a_den * lcnt[i] >= (uint64_t)a_num * smax);
        if (sig) { keep[i] = 1; shots[i] = lcnt[i]; wnum[i] = lcnt[i]; wden[i] = S; ++nsig; }
        else ins[nins++] = i;
    }
    T->stats[2] = nsig; T->stats[3] = nins;
    if (nins <= beta) {
        for (uint64_t t = 0; t < nins; ++t) {
            uint64_t i = ins[t];
            keep[i] = 1; shots[i] = lcnt[i]; wnum[i] = lcnt[i]; wden[i] = S;
        }
        uint64_t sI = 0;
        for (uint64_t t = 0; t < nins; ++t) sI += lcnt[ins[t]];
        T->stats[4] = sI; T->stats[5] = sI;
    } else {
        uint64_t *a = malloc(sizeof(uint64_t) * nins);
        oc_prune_select(seed, nins, beta, a);
        uint64_t sI = 0, D = 0;
        for (uint64_t t = 0; t < nins; ++t) sI += lcnt[ins[t]];
        uint64_t *cnt = malloc(sizeof(uint64_t) * beta), *got = malloc(sizeof(uint64_t) * beta);
        for (uint32_t t = 0; t < beta; ++t) { cnt[t] = lcnt[ins[a[t]]]; D += cnt[t]; }
        T->stats[4] = sI; T->stats[5] = D;
        oc_apportion(sI, cnt, beta, got);
        for (uint32_t t = 0; t < beta; ++t) {
            uint64_t i = ins[a[t]];
            keep[i] = 1; wnum[i] = sI * cnt[t]; wden[i] = D * S; shots[i] = got[t];
        }
        free(cnt); free(got); free(a);
    }
    free(ins);

    uint64_t nk = 0, nev = 0;
    for (uint64_t i = 0; i < L; ++i) if (keep[i]) { ++nk; nev += coff[lrep[i] + 1] - coff[lrep[i]]; }
    T->stats[7] = nk;
    T->n_leaves = nk;
    T->ev_off = malloc(sizeof(uint64_t) * (nk + 1));
    T->ev_key = malloc(sizeof(uint64_t) * (nev + 1));
    T->count = malloc(sizeof(uint64_t) * (nk + 1));
    T->shots = malloc(sizeof(uint64_t) * (nk + 1));
    T->wnum = malloc(sizeof(uint64_t) * (nk + 1));
    T->wden = malloc(sizeof(uint64_t) * (nk + 1));
    uint64_t li = 0, eo = 0;
    T->ev_off[0] = 0;
    for (uint64_t i = 0; i < L; ++i) {
        if (!keep[i]) continue;
        uint64_t u = lrep[i], ne = coff[u + 1] - coff[u];
        memcpy(T->ev_key + eo, ckey + coff[u], ne * 8);
        eo += ne;
        T->ev_off[li + 1] = eo;
        T->count[li] = lcnt[i]; T->shots[li] = shots[i]; T->wnum[li] = wnum[i]; T->wden[li] = wden[i];
        ++li;
    }
    free(keep); free(shots); free(wnum); free(wden); free(lrep); free(lcnt); free(coff); free(ckey);
    prep_free(&P);
    return T;
}

uint64_t oc_tree_num_leaves(const oc_tree *t) { return t->n_leaves; }
uint64_t oc_tree_num_events(const oc_tree *t) { return t->ev_off[t->n_leaves]; }
uint64_t oc_tree_num_raw(const oc_tree *t) { return t->n_raw; }
void oc_tree_stats(const oc_tree *t, uint64_t out[8]) { memcpy(out, t->stats, sizeof(t->stats)); }

void oc_tree_leaves(const oc_tree *t, uint64_t *ev_off, uint32_t *slot, uint32_t *qubit,
                    uint8_t *pauli, uint64_t *count, uint64_t *shots, uint64_t *wnum, uint64_t *wden)
{
    memcpy(ev_off, t->ev_off, sizeof(uint64_t) * (t->n_leaves + 1));
    uint64_t ne = t->ev_off[t->n_leaves];
    for (uint64_t i = 0; i < ne; ++i) {
        slot[i] = EV_SLOT(t->ev_key[i]); qubit[i] = EV_QUBIT(t->ev_key[i]);
        pauli[i] = (uint8_t)EV_PAULI(t->ev_key[i]);
    }
    memcpy(count, t->count, sizeof(uint64_t) * t->n_leaves);
    memcpy(shots, t->shots, sizeof(uint64_t) * t->n_leaves);
    memcpy(wnum, t->wnum, sizeof(uint64_t) * t->n_leaves);
    memcpy(wden, t->wden, sizeof(uint64_t) * t->n_leaves);
}

void oc_tree_raw(const oc_tree *t, uint32_t *shot, uint32_t *chan, uint8_t *outc)
{
    memcpy(shot, t->raw_shot, sizeof(uint32_t) * t->n_raw);
    memcpy(chan, t->raw_chan, sizeof(uint32_t) * t->n_raw);
    memcpy(outc, t->raw_out, t->n_raw);
}

/* Tree byte format (little endian):
 *   u32 magic 0x51535554, u32 version 1, u32 n, u32 G, u64 shots, u64 leaves,
 *   per leaf: u64 count, u64 shots, u64 wnum, u64 wden, u32 n_events,
 *             n_events x (u32 slot, u32 qubit, u8 pauli). */
static size_t put(uint8_t *b, size_t cap, size_t at, const void *v, size_t k)
{
    if (b && at + k <= cap) memcpy(b + at, v, k);
    return at + k;
}

size_t oc_tree_serialize(const oc_tree *t, uint8_t *buf, size_t cap)
{
    size_t at = 0;
    uint32_t h[4] = {0x51535554u, 1u, t->n, t->G};
    at = put(buf, cap, at, h, 16);
    at = put(buf, cap, at, &t->S, 8);
    at = put(buf, cap, at, &t->n_leaves, 8);
    for (uint64_t i = 0; i < t->n_leaves; ++i) {
        at = put(buf, cap, at, &t->count[i], 8);
        at = put(buf, cap, at, &t->shots[i], 8);
        at = put(buf, cap, at, &t->wnum[i], 8);
        at = put(buf, cap, at, &t->wden[i], 8);
        uint32_t ne = (uint32_t)(t->ev_off[i + 1] - t->ev_off[i]);
        at = put(buf, cap, at, &ne, 4);
        for (uint64_t e = t->ev_off[i]; e < t->ev_off[i + 1]; ++e) {
            uint32_t s = EV_SLOT(t->ev_key[e]), q = EV_QUBIT(t->ev_key[e]);
            uint8_t p = (uint8_t)EV_PAULI(t->ev_key[e]);
            at = put(buf, cap, at, &s, 4);
            at = put(buf, cap, at, &q, 4);
            at = put(buf, cap, at, &p, 1);
        }
    }
    return at;
}

/* ------------------------------------------------------------------------ */
/* Statevector simulation (Sec. II, Eq. (1)), complex128.  Gate matrices:    */
/*   U3(t,f,l) = [[cos t/2, -e^{il} sin t/2], [e^{if} sin t/2, e^{i(f+l)} cos t/2]]
 *   RX(t) = exp(-i t X / 2), RY(t) = exp(-i t Y / 2), RZ(t) = exp(-i t Z / 2)
 *   H, S = diag(1, i), T = diag(1, e^{i pi/4}), their daggers, X, Y, Z.
 * Bit q of a basis index is qubit q.  CX(c, t) flips t where c is 1.        */
typedef double complex cplx;

static void gate_matrix(uint8_t kind, const double *pr, cplx m[4])
{
    double t = pr ? pr[0] : 0.0;
    switch (kind) {
    case OK_U3: {
        double ct = cos(pr[0] / 2), st = sin(pr[0] / 2);
        m[0] = ct; m[1] = -cexp(I * pr[2]) * st;
        m[2] = cexp(I * pr[1]) * st; m[3] = cexp(I * (pr[1] + pr[2])) * ct;
        break;
    }
    case OK_RX: m[0] = cos(t / 2); m[1] = -I * sin(t / 2); m[2] = -I * sin(t / 2); m[3] = cos(t / 2); break;
    case OK_RY: m[0] = cos(t / 2); m[1] = -sin(t / 2); m[2] = sin(t / 2); m[3] = cos(t / 2); break;
    case OK_RZ: m[0] = cexp(-I * t / 2); m[1] = 0; m[2] = 0; m[3] = cexp(I * t / 2); break;
    case OK_H: m[0] = M_SQRT1_2; m[1] = M_SQRT1_2; m[2] = M_SQRT1_2; m[3] = -M_SQRT1_2; break;
    case OK_S: m[0] = 1; m[1] = 0; m[2] = 0; m[3] = I; break;
    case OK_SDG: m[0] = 1; m[1] = 0; m[2] = 0; m[3] = -I; break;
    case OK_T: m[0] = 1; m[1] = 0; m[2] = 0; m[3] = cexp(I * M_PI / 4); break;
    case OK_TDG: m[0] = 1; m[1] = 0; m[2] = 0; m[3] = cexp(-I * M_PI / 4); break;
    case OK_X: m[0] = 0; m[1] = 1; m[2] = 1; m[3] = 0; break;
    case OK_Y: m[0] = 0; m[1] = -I; m[2] = I; m[3] = 0; break;
    case OK_Z: m[0] = 1; m[1] = 0; m[2] = 0; m[3] = -1; break;
    default: m[0] = 1; m[1] = 0; m[2] = 0; m[3] = 1; break;
    }
}

static void apply_1q(cplx *psi, uint32_t n, uint32_t q, const cplx m[4])
{
    uint64_t N = 1ull << n, bit = 1ull << q;
#pragma omp parallel for num_threads(oracle_threads) schedule(static) if (N >= (1ull << 16))
    for (uint64_t i = 0; i < N; ++i) {
        if (i & bit) continue;
        cplx a0 = psi[i], a1 = psi[i | bit];
        psi[i] = m[0] * a0 + m[1] * a1;
        psi[i | bit] = m[2] * a0 + m[3] * a1;
    }
}

static void apply_cx(cplx *psi, uint32_t n, uint32_t qc, uint32_t qt)
{
    uint64_t N = 1ull << n, bc = 1ull << qc, bt = 1ull << qt;
#pragma omp parallel for num_threads(oracle_threads) schedule(static) if (N >= (1ull << 16))
    for (uint64_t i = 0; i < N; ++i) {
        if (!(i & bc) || (i & bt)) continue;
        cplx tmp = psi[i]; psi[i] = psi[i | bt]; psi[i | bt] = tmp;
    }
}

/* Pauli error gates; exact in floating point (swaps, negations, *i). */
static void apply_pauli(cplx *psi, uint32_t n, uint32_t q, int p)
{
    uint64_t N = 1ull << n, bit = 1ull << q;
#pragma omp parallel for num_threads(oracle_threads) schedule(static) if (N >= (1ull << 16))
    for (uint64_t i = 0; i < N; ++i) {
        if (i & bit) continue;
        cplx a0 = psi[i], a1 = psi[i | bit];
        if (p == 1) { psi[i] = a1; psi[i | bit] = a0; }
        else if (p == 2) { psi[i] = -I * a1; psi[i | bit] = I * a0; }
        else { psi[i | bit] = -a1; }
    }
}

/* A 4x4 on qubits (qa, qb): amplitude index 2 * bit(qa) + bit(qb). */
static void apply_2q(cplx *psi, uint32_t n, uint32_t qa, uint32_t qb, const cplx m[16])
{
    uint64_t N = 1ull << n, ba = 1ull << qa, bb = 1ull << qb;
#pragma omp parallel for num_threads(oracle_threads) schedule(static) if (N >= (1ull << 16))
    for (uint64_t i = 0; i < N; ++i) {
        if (i & (ba | bb)) continue;
        uint64_t idx[4] = {i, i | bb, i | ba, i | ba | bb};
        cplx a[4], r[4];
        for (int k = 0; k < 4; ++k) a[k] = psi[idx[k]];
        for (int r_ = 0; r_ < 4; ++r_) {
            r[r_] = 0;
            for (int k = 0; k < 4; ++k) r[r_] += m[4 * r_ + k] * a[k];
        }
        for (int k = 0; k < 4; ++k) psi[idx[k]] = r[k];
    }
}

static void apply_gate(const oc_circuit *c, uint32_t g, cplx *psi, int inverse)
{
    if (c->kind[g] == OK_CX) { apply_cx(psi, c->n, c->q0[g], c->q1[g]); return; }
    if (c->kind[g] == OK_U2M) {
        const double *d = c->mats + c->mat_off[g];
        cplx m[16];
        for (int r = 0; r < 4; ++r)
            for (int k = 0; k < 4; ++k) {
                /* the inverse is the conjugate transpose */
                int s = inverse ? 4 * k + r : 4 * r + k;
                cplx v = d[2 * s] + I * d[2 * s + 1];
                m[4 * r + k] = inverse ? conj(v) : v;
            }
        apply_2q(psi, c->n, c->q0[g], c->q1[g], m);
        return;
    }
    cplx m[4];
    if (c->kind[g] == OK_U1M) {
        const double *d = c->mats + c->mat_off[g];
        for (int k = 0; k < 4; ++k) m[k] = d[2 * k] + I * d[2 * k + 1];
    } else {
        gate_matrix(c->kind[g], c->params + 3 * (size_t)g, m);
    }
    if (inverse) {
        cplx d[4] = {conj(m[0]), conj(m[2]), conj(m[1]), conj(m[3])};
        apply_1q(psi, c->n, c->q0[g], d);
    } else {
        apply_1q(psi, c->n, c->q0[g], m);
    }
}

static void reset_state(cplx *psi, uint32_t n)
{
    uint64_t N = 1ull << n;
    for (uint64_t i = 0; i < N; ++i) psi[i] = 0;
    psi[0] = 1;
}

/* Token list of a leaf: for s = 0..G, its events at slot s (qubit order),
 * then gate s.  Token t >= 0 is gate t; t < 0 is event (-t - 1). */
static uint64_t leaf_tokens(const oc_circuit *c, const uint64_t *keys, uint64_t ne, int64_t *tok)
{
    uint64_t k = 0, e = 0;
    for (uint32_t s = 0; s <= c->G; ++s) {
        while (e < ne && EV_SLOT(keys[e]) == s) { tok[k++] = -(int64_t)e - 1; ++e; }
        if (s < c->G) tok[k++] = (int64_t)s;
    }
    return k;
}

/* ops: the paper's operation count (Sec. III-B.2): 1 per 1-qubit matrix
 * (gate or Pauli), 4 per 2-qubit matrix, 1 per forward measurement edge. */
typedef struct { uint64_t fwd_gates, inv_gates, fwd_paulis, inv_paulis, resets, leaves, draws,
                          ret_gates, ret_paulis, saves, restores, mcm, ops; } counters_t;

static void apply_token(const oc_circuit *c, const uint64_t *keys, int64_t t, cplx *psi,
                        int inverse, counters_t *ct)
{
    if (t >= 0) {
        apply_gate(c, (uint32_t)t, psi, inverse);
        if (inverse) ct->inv_gates++; else ct->fwd_gates++;
        ct->ops += is_two_qubit(c->kind[t]) ? 4 : 1;
    } else {
        uint64_t k = keys[-t - 1];
        apply_pauli(psi, c->n, EV_QUBIT(k), EV_PAULI(k));
        if (inverse) ct->inv_paulis++; else ct->fwd_paulis++;
        ct->ops += 1;
    }
}

/* Depth (in tokens) of the deepest node shared by two leaves: with j the
 * first differing event index and b the smaller slot of the two events there
 * (an exhausted list has none), the shared prefix is gates [0, b) plus the
 * first j events: b + j tokens. */
static uint64_t shared_depth(const oc_circuit *c, const uint64_t *a, uint64_t na, const uint64_t *b,
                             uint64_t nb)
{
    uint64_t j = 0;
    while (j < na && j < nb && a[j] == b[j]) ++j;
    uint64_t sa = j < na ? EV_SLOT(a[j]) : (uint64_t)c->G + 1;
    uint64_t sb = j < nb ? EV_SLOT(b[j]) : (uint64_t)c->G + 1;
    uint64_t bslot = sa < sb ? sa : sb;
    if (bslot > c->G) bslot = c->G;
    return bslot + j;
}

int oc_trajectory(const oc_circuit *c, uint32_t ne, const uint32_t *slot, const uint32_t *qubit,
                  const uint8_t *pauli, uint64_t max_tokens, double *state_out)
{
    if (validate(c) || has_measure(c)) return -1;
    uint64_t *keys = malloc(sizeof(uint64_t) * (ne + 1));
    for (uint32_t i = 0; i < ne; ++i) keys[i] = EVKEY(slot[i], qubit[i], pauli[i]);
    for (uint32_t i = 1; i < ne; ++i) if (keys[i] <= keys[i - 1]) { free(keys); return -1; }
    int64_t *tok = malloc(sizeof(int64_t) * (c->G + ne + 1));
    uint64_t nt = leaf_tokens(c, keys, ne, tok);
    if (max_tokens && max_tokens < nt) nt = max_tokens;
    cplx *psi = (cplx *)state_out;
    reset_state(psi, c->n);
    counters_t ct = {0};
    for (uint64_t i = 0; i < nt; ++i) apply_token(c, keys, tok[i], psi, 0, &ct);
    free(tok); free(keys);
    return 0;
}

/* Compute to depth d, keep that state, continue to the leaf, then undo back
 * to depth d with inverse gates in reverse order; report max |difference|. */
int oc_roundtrip(const oc_circuit *c, uint32_t ne, const uint32_t *slot, const uint32_t *qubit,
                 const uint8_t *pauli, uint64_t depth, double *maxdiff)
{
    if (validate(c) || has_measure(c)) return -1;
    uint64_t N = 1ull << c->n;
    uint64_t *keys = malloc(sizeof(uint64_t) * (ne + 1));
    for (uint32_t i = 0; i < ne; ++i) keys[i] = EVKEY(slot[i], qubit[i], pauli[i]);
    int64_t *tok = malloc(sizeof(int64_t) * (c->G + ne + 1));
    uint64_t nt = leaf_tokens(c, keys, ne, tok);
    if (depth > nt) depth = nt;
    cplx *psi = malloc(sizeof(cplx) * N), *saved = malloc(sizeof(cplx) * N);
    reset_state(psi, c->n);
    counters_t ct = {0};
    for (uint64_t i = 0; i < depth; ++i) apply_token(c, keys, tok[i], psi, 0, &ct);
    memcpy(saved, psi, sizeof(cplx) * N);
    for (uint64_t i = depth; i < nt; ++i) apply_token(c, keys, tok[i], psi, 0, &ct);
    for (uint64_t i = nt; i > depth; --i) apply_token(c, keys, tok[i - 1], psi, 1, &ct);
    double m = 0;
    for (uint64_t i = 0; i < N; ++i) { double d = cabs(psi[i] - saved[i]); if (d > m) m = d; }
    *maxdiff = m;
    free(psi); free(saved); free(tok); free(keys);
    return 0;
}

/* Index drawn for uniform target x in [0, norm): the smallest i whose
 * left-to-right prefix sum cdf[i] exceeds x (binary search over the
 * monotone prefix array); if rounding leaves none, the last index with
 * non-zero probability. */
static uint64_t draw_index(const double *cdf, uint64_t N, double x)
{
    uint64_t lo = 0, hi = N;
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo) / 2;
        if (cdf[mid] > x) hi = mid; else lo = mid + 1;
    }
    if (lo < N) return lo;
    uint64_t i = N - 1;
    while (i > 0 && cdf[i] == cdf[i - 1]) --i;
    return i;
}

/* Traversal policies: 0 = plain DFTT (undo the previous leaf to the shared
 * node with inverse gates, then go down; Sec. III-B), 1 = naive (every leaf
 * from |0...0>), 2 = hybrid (undo only when that costs strictly fewer tokens
 * than recomputing the leaf from the root).
 * Leaf l draws shots[l] samples: draw d uses stream 2, counter
 * (d >> 1, l, 0), half d & 1; u = (v >> 11) * 2^-53; target u * norm.
 * counters: fwd gates, inv gates, fwd paulis, inv paulis, resets, leaves,
 * draws, then the gates and paulis a final return to the root would undo. */
/* Checkpoint traversal with at most `slots` kept states (0 = no limit):
 * when a save finds the stack full, the state farthest from the leaves (the
 * bottom of the stack) is dropped; a leaf whose branch depth is no longer
 * kept undoes the previous leaf back to it instead (the hybrid of
 * checkpointing and uncomputation). */
static uint64_t ckpt_slots_limit = 0;
void oc_set_checkpoint_slots(uint64_t slots) { ckpt_slots_limit = slots; }

/* oc_run_margins: oc_run that also writes, per draw, the distance of its
 * target to the nearer CDF boundary of the drawn index (the margin
 * oc_leaf_margins gives), so that tests can excuse draws a different
 * summation order may move without recomputing the leaf. */
int oc_run_margins(const oc_circuit *c, const oc_tree *t, uint64_t seed, int traversal,
                   uint64_t lb, uint64_t le, double *dist, uint64_t *samples, double *margins,
                   uint64_t *counters, double *norms);

int oc_run(const oc_circuit *c, const oc_tree *t, uint64_t seed, int traversal, uint64_t lb,
           uint64_t le, double *dist, uint64_t *samples, uint64_t *counters, double *norms)
{
    return oc_run_margins(c, t, seed, traversal, lb, le, dist, samples, NULL, counters, norms);
}

int oc_run_margins(const oc_circuit *c, const oc_tree *t, uint64_t seed, int traversal,
                   uint64_t lb, uint64_t le, double *dist, uint64_t *samples, double *margins,
                   uint64_t *counters, double *norms)
{
    if (validate(c)) return -1;
    if (has_measure(c)) return -3;  /* non-invertible edges: oc_run_mcm */
    if (le == 0 && lb == 0) le = t->n_leaves;
    if (lb > le || le > t->n_leaves) return -1;
    uint64_t N = 1ull << c->n;
    cplx *psi = malloc(sizeof(cplx) * N);
    double *cdf = samples ? malloc(sizeof(double) * N) : NULL;
    size_t cap = (size_t)c->G + (size_t)c->n * ((size_t)c->G + 1) + 1;
    int64_t *ta = malloc(sizeof(int64_t) * cap);
    int64_t *tb = malloc(sizeof(int64_t) * cap);
    counters_t ct = {0};
    if (dist) for (uint64_t i = 0; i < N; ++i) dist[i] = 0.0;
    uint64_t so = 0, na = 0, nka = 0;
    const uint64_t *ka = NULL;
    /* Checkpoint traversal (3): plain DFTT, except that the state at every
     * depth where a later leaf branches off the current path is kept, and a
     * leaf starts from the kept state at its branch depth instead of undoing
     * the previous leaf.  bd[l - lb] = branch depth of leaf l (shared with
     * leaf l - 1); a depth x is kept while leaf l runs forward through it if
     * some later leaf m branches at x and no leaf in between branches
     * shallower than x. */
    uint64_t *bd = NULL, *kdepth = NULL, nk = 0;
    cplx **kstate = NULL;
    if (traversal == 3 && le > lb) {
        bd = calloc(le - lb, sizeof(uint64_t));
        for (uint64_t l = lb + 1; l < le; ++l) {
            const uint64_t *k0 = t->ev_key + t->ev_off[l - 1], *k1 = t->ev_key + t->ev_off[l];
            bd[l - lb] = shared_depth(c, k0, t->ev_off[l] - t->ev_off[l - 1], k1,
                                      t->ev_off[l + 1] - t->ev_off[l]);
        }
        kdepth = malloc(sizeof(uint64_t) * (c->G + c->n * (size_t)c->G + 2));
        kstate = malloc(sizeof(cplx *) * (c->G + c->n * (size_t)c->G + 2));
    }
    for (uint64_t l = lb; l < le; ++l) {
        const uint64_t *kb = t->ev_key + t->ev_off[l];
        uint64_t nkb = t->ev_off[l + 1] - t->ev_off[l];
        uint64_t nb = leaf_tokens(c, kb, nkb, tb);
        uint64_t from = 0;
        int reset = 1;
        if (l > lb && traversal == 3) {
            uint64_t d = bd[l - lb];
            while (nk > 0 && kdepth[nk - 1] > d) free(kstate[--nk]);
            if (d > 0) {
                if (nk > 0 && kdepth[nk - 1] == d) {
                    memcpy(psi, kstate[nk - 1], sizeof(cplx) * N);
                    ct.restores++;
                } else {
                    /* its state was dropped (slot limit): undo back to it */
                    if (!ckpt_slots_limit) return -2;  /* unreachable without a limit */
                    for (uint64_t i = na; i > d; --i) apply_token(c, ka, ta[i - 1], psi, 1, &ct);
                }
                from = d;
                reset = 0;
            } else {
                while (nk > 0) free(kstate[--nk]);
            }
        } else if (l > lb && traversal != 1) {
            uint64_t d = shared_depth(c, ka, nka, kb, nkb);
            if (traversal == 0 || (na - d) + (nb - d) < nb) {
                for (uint64_t i = na; i > d; --i) apply_token(c, ka, ta[i - 1], psi, 1, &ct);
                from = d;
                reset = 0;
            }
        }
        if (reset) { reset_state(psi, c->n); ct.resets++; }
        for (uint64_t i = from; i < nb; ++i) {
            if (traversal == 3 && i > from) {
                /* keep depth i if a later leaf branches here (running minimum) */
                int keep = 0;
                uint64_t r = UINT64_MAX;
                for (uint64_t m = l + 1; m < le; ++m) {
                    uint64_t dm = bd[m - lb];
                    if (dm < r) r = dm;
                    if (r < i) break;
                    if (dm == i) { keep = 1; break; }
                }
                if (keep) {
                    if (ckpt_slots_limit && nk == ckpt_slots_limit) {
                        /* full: drop the state farthest from the leaves */
                        free(kstate[0]);
                        memmove(kdepth, kdepth + 1, sizeof(uint64_t) * (nk - 1));
                        memmove(kstate, kstate + 1, sizeof(cplx *) * (nk - 1));
                        --nk;
                    }
                    kdepth[nk] = i;
                    kstate[nk] = malloc(sizeof(cplx) * N);
                    memcpy(kstate[nk], psi, sizeof(cplx) * N);
                    ++nk;
                    ct.saves++;
                }
            }
            apply_token(c, kb, tb[i], psi, 0, &ct);
        }
        ct.leaves++;
        double w = (double)t->wnum[l] / (double)t->wden[l];
        double nrm = 0.0;
        for (uint64_t i = 0; i < N; ++i) {
            double pr = creal(psi[i]) * creal(psi[i]) + cimag(psi[i]) * cimag(psi[i]);
            nrm = nrm + pr;
            if (dist) dist[i] = dist[i] + w * pr;
            if (cdf) cdf[i] = nrm;
        }
        if (norms) norms[l - lb] = nrm;
        if (samples) {
            for (uint64_t d = 0; d < t->shots[l]; ++d) {
                uint64_t v = draw64(seed, (uint32_t)(d >> 1), (uint32_t)l, 0, 2, (int)(d & 1));
                double u = (double)(v >> 11) * 0x1p-53;
                uint64_t i = draw_index(cdf, N, u * nrm);
                if (margins) {
                    double x = u * nrm, lo = i ? cdf[i - 1] : 0.0;
                    double m1 = fabs(x - lo), m2 = fabs(cdf[i] - x);
                    margins[so] = m1 < m2 ? m1 : m2;
                }
                samples[so++] = i;
                ct.draws++;
            }
        }
        int64_t *tmp = ta; ta = tb; tb = tmp;
        na = nb; ka = kb; nka = nkb;
    }
    if (le > lb) { ct.ret_gates = c->G; ct.ret_paulis = nka; }
    while (nk > 0) free(kstate[--nk]);
    free(bd); free(kdepth); free(kstate);
    free(psi); free(cdf); free(ta); free(tb);
    if (counters) memcpy(counters, &ct, sizeof(ct));
    return 0;
}

/* Per-draw margin to the nearest CDF boundary of the drawn index, in the
 * same units as the target (used by tests to excuse draws that rounding in
 * a different summation order could legitimately move). */
int oc_leaf_margins(const oc_circuit *c, const double *state, uint64_t seed, uint64_t leaf,
                    uint64_t shots, uint64_t *idx_out, double *margin_out)
{
    uint64_t N = 1ull << c->n;
    const cplx *psi = (const cplx *)state;
    double *cdf = malloc(sizeof(double) * N);
    double nrm = 0.0;
    for (uint64_t i = 0; i < N; ++i) {
        nrm = nrm + (creal(psi[i]) * creal(psi[i]) + cimag(psi[i]) * cimag(psi[i]));
        cdf[i] = nrm;
    }
    for (uint64_t d = 0; d < shots; ++d) {
        uint64_t v = draw64(seed, (uint32_t)(d >> 1), (uint32_t)leaf, 0, 2, (int)(d & 1));
        double x = (double)(v >> 11) * 0x1p-53 * nrm;
        uint64_t i = draw_index(cdf, N, x);
        double lo = i ? cdf[i - 1] : 0.0;
        double m1 = fabs(x - lo), m2 = fabs(cdf[i] - x);
        idx_out[d] = i;
        margin_out[d] = m1 < m2 ? m1 : m2;
    }
    free(cdf);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Non-invertible edges: mid-circuit measurement layers (Sec. III-B.2).
 *
 * Semantics (readings; the paper fixes the tree structure and the caching
 * protocol, not the trajectory rule):
 *   - a layer of m <= 8 measured qubits q_0 < ... < q_{m-1} is one edge;
 *     outcome o has bit b = the value of q_b, weight P_o = the sum of
 *     |psi_i|^2 over the basis states i of that pattern (left to right);
 *   - every shot picks its own outcome: shot j (0-based within leaf l) at
 *     layer k draws v on stream 3, counter (j, l, k), half 0;
 *     u = (v >> 11) 2^-53, and the outcome is the smallest o with
 *     u T < C_o, C_o = P_0 + ... + P_o, T = C_{2^m-1} (if rounding leaves
 *     none, the last o with P_o > 0);
 *   - the state becomes P_o psi / sqrt(P_o); MR then flips the measured
 *     qubits back to 0 (psi'[i] = psi[i ^ deposit(o)] / sqrt(P_o) on the
 *     all-zero pattern);
 *   - a node's shots thereby split into outcome branches; a final leaf
 *     reached with c shots of tree leaf l weighs c / S (trees without
 *     pruning only).
 *
 * DFTT+Caching with cache capacity K, over stages (stage s = the tokens
 * between layers s-1 and s):
 *   - within a stage the walk is plain DFTT: undo to the node shared with
 *     the next path, then go down;
 *   - a pre-measurement node of layer k is pushed on the LIFO cache when
 *     the walk reaches it if k is one of the K layers closest to the leaves
 *     (k >= M - K), and popped once all of its outcome branches are done;
 *   - crossing a measurement edge backwards fetches the node from the
 *     cache; an uncached node is recomputed from the root (replaying the
 *     recorded outcomes), after which the walk continues with DFTT;
 *   - K = 0 switches DFTT off: every final leaf is computed from the root.
 * Samples: final leaf (l, c shots) draws c indices with the shot-sampling
 * stream, counter (d >> 1, l, 0), half d & 1, d running over the draws of
 * tree leaf l in walk order.
 * The operation counts of Eq. (3): 1 per 1-qubit matrix, 4 per CX, 1 per
 * forward measurement edge, 0 for a fetch; N_1 is the count with K = 0 and
 * N_2 the count with K >= M (every pre-measurement node cached). */

typedef struct {
    uint64_t n;
    uint64_t *leaf;   /* tree leaf of entry i */
    uint64_t *off;    /* shots of entry i: shot[off[i] .. off[i+1]) */
    uint32_t *shot;
} mgroup_t;

typedef struct {
    const oc_circuit *c;
    const oc_tree *t;
    uint64_t seed, N, lb;
    uint32_t M, K;
    int naive;
    uint32_t *lgate;          /* gate index of layer k */
    int64_t **tok;            /* per leaf in range: token list */
    uint64_t *ntok;
    uint64_t **lpos;          /* per leaf: token position of layer k */
    cplx *psi, *tmp;
    cplx **cache;             /* per layer (only cached layers used) */
    uint64_t *rep;            /* per stage: a leaf of the current path */
    uint32_t *out;            /* per layer: outcome of the current path */
    double *dist, *cdf;
    uint64_t *samples, so, *sbase;
    counters_t ct;
    uint64_t max_cached;
    uint64_t cached_now;
} mwalk_t;

static const uint64_t *mw_keys(const mwalk_t *W, uint64_t l) { return W->t->ev_key + W->t->ev_off[l]; }
static uint64_t st_begin(const mwalk_t *W, uint64_t l, uint32_t s)
{
    return s == 0 ? 0 : W->lpos[l - W->lb][s - 1] + 1;
}
static uint64_t st_end(const mwalk_t *W, uint64_t l, uint32_t s)
{
    return s < W->M ? W->lpos[l - W->lb][s] : W->ntok[l - W->lb];
}
static int tok_same(const mwalk_t *W, uint64_t la, int64_t ta, uint64_t lb_, int64_t tb)
{
    if ((ta >= 0) != (tb >= 0)) return 0;
    if (ta >= 0) return ta == tb;
    return mw_keys(W, la)[-ta - 1] == mw_keys(W, lb_)[-tb - 1];
}
/* tokens the stage-s parts of leaves a and b share from the stage start */
static uint64_t stage_lcp(const mwalk_t *W, uint64_t a, uint64_t b, uint32_t s)
{
    uint64_t a0 = st_begin(W, a, s), a1 = st_end(W, a, s);
    uint64_t b0 = st_begin(W, b, s), b1 = st_end(W, b, s);
    uint64_t d = 0;
    while (a0 + d < a1 && b0 + d < b1 &&
           tok_same(W, a, W->tok[a - W->lb][a0 + d], b, W->tok[b - W->lb][b0 + d]))
        ++d;
    return d;
}
static void fwd_range(mwalk_t *W, uint64_t l, uint32_t s, uint64_t from, uint64_t to)
{
    uint64_t b = st_begin(W, l, s);
    for (uint64_t i = from; i < to; ++i)
        apply_token(W->c, mw_keys(W, l), W->tok[l - W->lb][b + i], W->psi, 0, &W->ct);
}
static void inv_range(mwalk_t *W, uint64_t l, uint32_t s, uint64_t from, uint64_t to)
{
    uint64_t b = st_begin(W, l, s);
    for (uint64_t i = from; i > to; --i)
        apply_token(W->c, mw_keys(W, l), W->tok[l - W->lb][b + i - 1], W->psi, 1, &W->ct);
}

/* outcome weights of layer k's qubits over the current state */
static void layer_weights(const mwalk_t *W, uint32_t k, double *P, uint32_t *qs, uint32_t *m)
{
    uint64_t mk = meas_mask(W->c, W->lgate[k]);
    uint32_t mm = 0;
    for (uint32_t q = 0; q < W->c->n; ++q) if ((mk >> q) & 1) qs[mm++] = q;
    *m = mm;
    for (uint32_t o = 0; o < (1u << mm); ++o) P[o] = 0.0;
    for (uint64_t i = 0; i < W->N; ++i) {
        uint32_t o = 0;
        for (uint32_t b = 0; b < mm; ++b) o |= (uint32_t)((i >> qs[b]) & 1) << b;
        P[o] = P[o] + (creal(W->psi[i]) * creal(W->psi[i]) + cimag(W->psi[i]) * cimag(W->psi[i]));
    }
}

static uint32_t pick_branch(const double *P, uint32_t no, double u)
{
    double T = 0.0;
    for (uint32_t o = 0; o < no; ++o) T = T + P[o];
    double x = u * T, C = 0.0;
    for (uint32_t o = 0; o < no; ++o) {
        C = C + P[o];
        if (x < C) return o;
    }
    uint32_t o = no - 1;
    while (o > 0 && P[o] == 0.0) --o;
    return o;
}

/* measurement edge of layer k with outcome o: project, renormalise, reset */
static void apply_mcm(mwalk_t *W, uint32_t k, uint32_t o)
{
    double P[1 << MAX_MEASURED];
    uint32_t qs[MAX_MEASURED], m;
    layer_weights(W, k, P, qs, &m);
    int reset = W->c->kind[W->lgate[k]] == OK_MR;
    uint64_t dep = 0;
    for (uint32_t b = 0; b < m; ++b) if ((o >> b) & 1) dep |= 1ull << qs[b];
    uint32_t want = reset ? 0u : o;
    uint64_t flip = reset ? dep : 0;
    double sc = 1.0 / sqrt(P[o]);
    for (uint64_t i = 0; i < W->N; ++i) {
        uint32_t pat = 0;
        for (uint32_t b = 0; b < m; ++b) pat |= (uint32_t)((i >> qs[b]) & 1) << b;
        W->tmp[i] = pat == want ? W->psi[i ^ flip] * sc : 0.0;
    }
    memcpy(W->psi, W->tmp, sizeof(cplx) * W->N);
    W->ct.mcm++;
    W->ct.ops++;
}

static int layer_cached(const mwalk_t *W, uint32_t k)
{
    return !W->naive && W->K > 0 && k + W->K >= W->M;
}

static void reach_pre(mwalk_t *W, uint32_t k);
/* state := the root of stage s on the current path */
static void reach_root(mwalk_t *W, uint32_t s)
{
    if (s == 0) {
        reset_state(W->psi, W->c->n);
        W->ct.resets++;
        return;
    }
    reach_pre(W, s - 1);
    apply_mcm(W, s - 1, W->out[s - 1]);
}
/* state := the pre-measurement node of layer k on the current path */
static void reach_pre(mwalk_t *W, uint32_t k)
{
    if (layer_cached(W, k)) {
        memcpy(W->psi, W->cache[k], sizeof(cplx) * W->N);
        W->ct.restores++;
        return;
    }
    reach_root(W, k);
    uint64_t l = W->rep[k];
    fwd_range(W, l, k, 0, st_end(W, l, k) - st_begin(W, l, k));
}

static void final_leaf(mwalk_t *W, uint64_t l, uint64_t c)
{
    double w = (double)c / (double)W->t->S, nrm = 0.0;
    for (uint64_t i = 0; i < W->N; ++i) {
        double pr = creal(W->psi[i]) * creal(W->psi[i]) + cimag(W->psi[i]) * cimag(W->psi[i]);
        nrm = nrm + pr;
        if (W->dist) W->dist[i] = W->dist[i] + w * pr;
        if (W->cdf) W->cdf[i] = nrm;
    }
    if (W->samples) {
        for (uint64_t k = 0; k < c; ++k) {
            uint64_t d = W->sbase[l - W->lb] + k;
            uint64_t v = draw64(W->seed, (uint32_t)(d >> 1), (uint32_t)l, 0, 2, (int)(d & 1));
            double u = (double)(v >> 11) * 0x1p-53;
            W->samples[W->so++] = draw_index(W->cdf, W->N, u * nrm);
        }
    }
    W->sbase[l - W->lb] += c;
    W->ct.leaves++;
    W->ct.draws += c;
}

static int mwalk(mwalk_t *W, uint32_t s, const mgroup_t *G)
{
    uint64_t i = 0, prev = UINT64_MAX;
    int valid = 1;
    while (i < G->n) {
        uint64_t l = G->leaf[i], j = i + 1;
        uint64_t len = st_end(W, l, s) - st_begin(W, l, s);
        while (j < G->n) {
            uint64_t l2 = G->leaf[j];
            if (st_end(W, l2, s) - st_begin(W, l2, s) != len || stage_lcp(W, l, l2, s) != len) break;
            ++j;
        }
        if (prev != UINT64_MAX) {
            uint64_t lp = G->leaf[prev];
            uint64_t d = stage_lcp(W, lp, l, s);
            if (valid && !W->naive) {
                inv_range(W, lp, s, st_end(W, lp, s) - st_begin(W, lp, s), d);
            } else {
                reach_root(W, s);
                fwd_range(W, l, s, 0, d);
            }
            fwd_range(W, l, s, d, len);
        } else {
            fwd_range(W, l, s, 0, len);
        }
        if (s == W->M) {
            if (j != i + 1) return -2;  /* distinct leaves differ somewhere */
            final_leaf(W, l, G->off[i + 1] - G->off[i]);
            valid = !W->naive;
        } else {
            W->rep[s] = l;
            double P[1 << MAX_MEASURED];
            uint32_t qs[MAX_MEASURED], m;
            layer_weights(W, s, P, qs, &m);
            uint32_t no = 1u << m;
            /* split the shots of entries i..j-1 by outcome */
            uint64_t tot = G->off[j] - G->off[i];
            uint32_t *oc = malloc(sizeof(uint32_t) * (tot + 1));
            uint64_t *cnt = calloc(no, sizeof(uint64_t));
            for (uint64_t e = i; e < j; ++e)
                for (uint64_t x = G->off[e]; x < G->off[e + 1]; ++x) {
                    uint64_t v = draw64(W->seed, G->shot[x], (uint32_t)G->leaf[e], s, 3, 0);
                    uint32_t o = pick_branch(P, no, (double)(v >> 11) * 0x1p-53);
                    oc[x - G->off[i]] = o;
                    cnt[o]++;
                }
            int cached = layer_cached(W, s);
            if (cached) {
                memcpy(W->cache[s], W->psi, sizeof(cplx) * W->N);
                W->ct.saves++;
                W->cached_now++;
                if (W->cached_now > W->max_cached) W->max_cached = W->cached_now;
            }
            int first = 1;
            for (uint32_t o = 0; o < no; ++o) {
                if (!cnt[o]) continue;
                mgroup_t H;
                H.leaf = malloc(sizeof(uint64_t) * (j - i));
                H.off = malloc(sizeof(uint64_t) * (j - i + 1));
                H.shot = malloc(sizeof(uint32_t) * (cnt[o] + 1));
                H.n = 0;
                H.off[0] = 0;
                uint64_t y = 0;
                for (uint64_t e = i; e < j; ++e) {
                    uint64_t y0 = y;
                    for (uint64_t x = G->off[e]; x < G->off[e + 1]; ++x)
                        if (oc[x - G->off[i]] == o) H.shot[y++] = G->shot[x];
                    if (y > y0) { H.leaf[H.n] = G->leaf[e]; H.off[++H.n] = y; }
                }
                if (!first) reach_pre(W, s);
                W->out[s] = o;
                apply_mcm(W, s, o);
                int rc = mwalk(W, s + 1, &H);
                free(H.leaf); free(H.off); free(H.shot);
                if (rc) { free(oc); free(cnt); return rc; }
                first = 0;
            }
            free(oc); free(cnt);
            if (cached) {
                memcpy(W->psi, W->cache[s], sizeof(cplx) * W->N);
                W->ct.restores++;
                W->cached_now--;
                valid = 1;
            } else {
                valid = 0;
            }
        }
        prev = i;
        i = j;
    }
    return 0;
}

/* counters as oc_run's, then the measurement edges applied and the
 * operation count; stats[0] = most states held in the cache at once. */
int oc_run_mcm(const oc_circuit *c, const oc_tree *t, uint64_t seed, uint32_t K, uint64_t lb,
               uint64_t le, double *dist, uint64_t *samples, uint64_t *counters, uint64_t *stats)
{
    if (validate(c)) return -1;
    if (le == 0 && lb == 0) le = t->n_leaves;
    if (lb > le || le > t->n_leaves) return -1;
    for (uint64_t l = lb; l < le; ++l)
        if (t->shots[l] != t->count[l] || t->wnum[l] != t->count[l] || t->wden[l] != t->S)
            return -4;  /* pruned trees are not split into outcome branches */
    mwalk_t W;
    memset(&W, 0, sizeof(W));
    W.c = c; W.t = t; W.seed = seed; W.N = 1ull << c->n; W.lb = lb;
    W.naive = K == 0;
    uint32_t M = 0;
    for (uint32_t g = 0; g < c->G; ++g) M += is_measure(c->kind[g]) ? 1 : 0;
    W.M = M;
    W.K = K > M ? M : K;
    W.lgate = malloc(sizeof(uint32_t) * (M + 1));
    for (uint32_t g = 0, k = 0; g < c->G; ++g) if (is_measure(c->kind[g])) W.lgate[k++] = g;
    uint64_t L = le - lb;
    W.tok = calloc(L + 1, sizeof(int64_t *));
    W.ntok = calloc(L + 1, sizeof(uint64_t));
    W.lpos = calloc(L + 1, sizeof(uint64_t *));
    for (uint64_t l = lb; l < le; ++l) {
        uint64_t ne = t->ev_off[l + 1] - t->ev_off[l];
        W.tok[l - lb] = malloc(sizeof(int64_t) * (c->G + ne + 1));
        W.ntok[l - lb] = leaf_tokens(c, t->ev_key + t->ev_off[l], ne, W.tok[l - lb]);
        W.lpos[l - lb] = malloc(sizeof(uint64_t) * (M + 1));
        for (uint64_t i = 0, k = 0; i < W.ntok[l - lb]; ++i) {
            int64_t tk = W.tok[l - lb][i];
            if (tk >= 0 && is_measure(c->kind[tk])) W.lpos[l - lb][k++] = i;
        }
    }
    W.psi = malloc(sizeof(cplx) * W.N);
    W.tmp = malloc(sizeof(cplx) * W.N);
    W.cache = calloc(M + 1, sizeof(cplx *));
    for (uint32_t k = 0; k < M; ++k)
        if (layer_cached(&W, k)) W.cache[k] = malloc(sizeof(cplx) * W.N);
    W.rep = calloc(M + 1, sizeof(uint64_t));
    W.out = calloc(M + 1, sizeof(uint32_t));
    W.dist = dist;
    if (dist) for (uint64_t i = 0; i < W.N; ++i) dist[i] = 0.0;
    W.samples = samples;
    W.cdf = samples ? malloc(sizeof(double) * W.N) : NULL;
    W.sbase = calloc(L + 1, sizeof(uint64_t));
    /* the root group: every leaf in range with all of its shots */
    mgroup_t G;
    uint64_t tot = 0;
    for (uint64_t l = lb; l < le; ++l) tot += t->shots[l];
    G.n = L;
    G.leaf = malloc(sizeof(uint64_t) * (L + 1));
    G.off = malloc(sizeof(uint64_t) * (L + 1));
    G.shot = malloc(sizeof(uint32_t) * (tot + 1));
    G.off[0] = 0;
    for (uint64_t l = lb, y = 0; l < le; ++l) {
        G.leaf[l - lb] = l;
        for (uint64_t j = 0; j < t->shots[l]; ++j) G.shot[y++] = (uint32_t)j;
        G.off[l - lb + 1] = G.off[l - lb] + t->shots[l];
    }
    int rc = 0;
    if (L > 0) {
        reset_state(W.psi, c->n);
        W.ct.resets++;
        rc = mwalk(&W, 0, &G);
    }
    if (counters) memcpy(counters, &W.ct, sizeof(W.ct));
    if (stats) stats[0] = W.max_cached;
    for (uint64_t l = 0; l < L; ++l) { free(W.tok[l]); free(W.lpos[l]); }
    for (uint32_t k = 0; k < M; ++k) free(W.cache[k]);
    free(W.tok); free(W.ntok); free(W.lpos); free(W.cache); free(W.rep); free(W.out);
    free(W.psi); free(W.tmp); free(W.cdf); free(W.sbase); free(W.lgate);
    free(G.leaf); free(G.off); free(G.shot);
    return rc;
}

/* One uniform double in [0, 1) of the method's streams: (v >> 11) 2^-53 with
 * v = draw64(seed, counter (sub, primary, aux, stream), half). */
double oc_uniform53(uint64_t seed, uint32_t sub, uint32_t primary, uint32_t aux, uint32_t stream,
                    int half)
{
    return (double)(draw64(seed, sub, primary, aux, stream, half) >> 11) * 0x1p-53;
}
