/*
 * CPU oracle for the state-vector simulator — TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct complex128 implementation of what the GPU
 * path computes.  Only the test-suite, the smoke check and the CPU-baseline leg
 * of the benchmark load it.  It shares no code, header or table with the HIP
 * library; the two meet only through the seeded inputs of the workload module.
 *
 * Conventions (Software description, "Distributed implementation"):
 *   - amplitude i of an n-qubit state, i = sum_q i_q 2^q, qubit 0 is the least
 *     significant bit (eq. 1 and the three-qubit figure's vector ordering);
 *   - a one-qubit gate is the 2x2 matrix U, row = output, acting on pairs
 *     (i, i + 2^q) with i_q = 0 (eq. 3);
 *   - gate matrices arrive as u[8] = {re00, im00, re01, im01, re10, im10, re11, im11}.
 *
 * Element-wise loops may run on several OpenMP threads: each pair or element
 * is updated independently, so the result does not depend on the thread
 * count.  Every reduction is a sequential sum accumulated in long double, in
 * index order; the cut and diagonal expectations over whole registers sum
 * fixed 2^16-term chunks that way and then add the chunk sums in order, so
 * their result does not depend on the thread count either.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;
typedef long double ldbl;

#define EXPORT __attribute__((visibility("default")))

static cplx mat(const double *u, int r, int c) { return u[4 * r + 2 * c] + I * u[4 * r + 2 * c + 1]; }

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11 "Parallel random numbers:
 * as easy as 1, 2, 3"): ten rounds of the 4x32 Philox S-box, with the key
 * bumped by the Weyl constants between rounds.                              */

EXPORT void ref_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += W0; k1 += W1; }
        uint64_t p0 = (uint64_t)M0 * c0;
        uint64_t p1 = (uint64_t)M1 * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Stream tags in counter word 2, so independent uses of one seed never share
 * counters. */
enum { TAG_INIT_RANDOM = 1, TAG_SAMPLE = 2, TAG_TRAJ = 3, TAG_MEASURE = 6, TAG_NOISE = 7 };

static void philox_draw_w3(uint64_t seed, uint32_t w0, uint32_t w1, uint32_t tag, uint32_t w3, uint32_t out[4])
{
    uint32_t ctr[4] = {w0, w1, tag, w3};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    ref_philox4x32_10(ctr, key, out);
}

static void philox_draw(uint64_t seed, uint32_t w0, uint32_t w1, uint32_t tag, uint32_t out[4])
{
    philox_draw_w3(seed, w0, w1, tag, 0u, out);
}

/* 53-bit uniform in [0,1) from two 32-bit words (lo, hi). */
static double u53(uint32_t lo, uint32_t hi)
{
    uint64_t v = ((uint64_t)hi << 32) | lo;
    return (double)(v >> 11) * (1.0 / 9007199254740992.0);
}

/* ------------------------------------------------------------------------ */
/* Gates                                                                     */

/* eq. (3): for every i with bit q clear, j = i + 2^q,
 *   a'_i = U00 a_i + U01 a_j,  a'_j = U10 a_i + U11 a_j. */
EXPORT void ref_apply_1q(cplx *psi, int n, int q, const double *u)
{
    const uint64_t N = 1ull << n, s = 1ull << q;
    const cplx u00 = mat(u, 0, 0), u01 = mat(u, 0, 1), u10 = mat(u, 1, 0), u11 = mat(u, 1, 1);
#pragma omp parallel for schedule(static)
    for (uint64_t i = 0; i < N; ++i) {
        if (i & s) continue;
        const uint64_t j = i | s;
        const cplx a = psi[i], b = psi[j];
        psi[i] = u00 * a + u01 * b;
        psi[j] = u10 * a + u11 * b;
    }
}

/* Controlled one-qubit gate: eq. (3) on target t restricted to the indices
 * whose control bit c is 1 (Software description, two-qubit gates of the
 * controlled form). */
EXPORT void ref_apply_c1q(cplx *psi, int n, int c, int t, const double *u)
{
    const uint64_t N = 1ull << n, sc = 1ull << c, st = 1ull << t;
    const cplx u00 = mat(u, 0, 0), u01 = mat(u, 0, 1), u10 = mat(u, 1, 0), u11 = mat(u, 1, 1);
#pragma omp parallel for schedule(static)
    for (uint64_t i = 0; i < N; ++i) {
        if ((i & st) || !(i & sc)) continue;
        const uint64_t j = i | st;
        const cplx a = psi[i], b = psi[j];
        psi[i] = u00 * a + u01 * b;
        psi[j] = u10 * a + u11 * b;
    }
}

/* Two-qubit diagonal: a_i *= d[2*b(q1) + b(q0)]; d given as 4 interleaved complex. */
EXPORT void ref_apply_diag2(cplx *psi, int n, int q0, int q1, const double *d)
{
    const uint64_t N = 1ull << n;
    cplx dd[4];
    for (int k = 0; k < 4; ++k) dd[k] = d[2 * k] + I * d[2 * k + 1];
#pragma omp parallel for schedule(static)
    for (uint64_t i = 0; i < N; ++i) {
        const int k = (int)(((i >> q1) & 1) * 2 + ((i >> q0) & 1));
        psi[i] *= dd[k];
    }
}

/* SWAP(a, b): exchange the amplitudes whose bits a and b are (1,0) and (0,1). */
EXPORT void ref_apply_swap(cplx *psi, int n, int a, int b)
{
    const uint64_t N = 1ull << n, sa = 1ull << a, sb = 1ull << b;
#pragma omp parallel for schedule(static)
    for (uint64_t i = 0; i < N; ++i) {
        if ((i & sa) && !(i & sb)) {
            const uint64_t j = (i ^ sa) | sb;
            const cplx t = psi[i];
            psi[i] = psi[j];
            psi[j] = t;
        }
    }
}

/* k-qubit gate (1 <= k <= 5): U is 2^k x 2^k, row-major interleaved (re, im),
 * row = output; bit m of a matrix index is the value of qubit qs[m].  For
 * every index i with all k target bits clear, the 2^k amplitudes
 * a_{i + off(j)}, off(j) = sum_m j_m 2^{qs[m]}, are replaced by U times them
 * (the two-qubit case of the Software description's gates, generalised). */
EXPORT int ref_apply_kq(cplx *psi, int n, const int32_t *qs, int k, const double *u)
{
    if (k < 1 || k > 5) return -1;
    const int K = 1 << k;
    uint64_t mask = 0, off[32];
    for (int m = 0; m < k; ++m) mask |= 1ull << qs[m];
    for (int j = 0; j < K; ++j) {
        off[j] = 0;
        for (int m = 0; m < k; ++m)
            if ((j >> m) & 1) off[j] |= 1ull << qs[m];
    }
    const uint64_t N = 1ull << n;
#pragma omp parallel for schedule(static)
    for (uint64_t i = 0; i < N; ++i) {
        if (i & mask) continue;
        cplx in[32];
        for (int j = 0; j < K; ++j) in[j] = psi[i + off[j]];
        for (int r = 0; r < K; ++r) {
            cplx acc = 0;
            for (int j = 0; j < K; ++j) acc += (u[2 * (r * K + j)] + I * u[2 * (r * K + j) + 1]) * in[j];
            psi[i + off[r]] = acc;
        }
    }
    return 0;
}

/* Gate-list record, laid out as the workload module's structured dtype:
 * int32 kind, q0, q1, pad; double u[8]. */
typedef struct { int32_t kind, q0, q1, pad; double u[8]; } ref_gate;
enum { RG_1Q = 1, RG_C1Q = 2, RG_DIAG2 = 3, RG_SWAP = 4, RG_NOISE = 5 };

static void apply_gate(cplx *psi, int n, const ref_gate *g)
{
    switch (g->kind) {
    case RG_1Q: ref_apply_1q(psi, n, g->q0, g->u); break;
    case RG_C1Q: ref_apply_c1q(psi, n, g->q0, g->q1, g->u); break;
    case RG_DIAG2: ref_apply_diag2(psi, n, g->q0, g->q1, g->u); break;
    case RG_SWAP: ref_apply_swap(psi, n, g->q0, g->q1); break;
    default: break;
    }
}

/* Sequential application of a gate list, one gate at a time. */
EXPORT int ref_apply_gates(cplx *psi, int n, const ref_gate *g, int count)
{
    for (int k = 0; k < count; ++k) {
        if (g[k].kind < RG_1Q || g[k].kind > RG_NOISE) return -1;
        if (g[k].kind == RG_NOISE) continue;  /* the noiseless circuit: noise gates are the identity */
        apply_gate(psi, n, &g[k]);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Initialisation                                                            */

/* |index> (Initialize("base", index)). */
EXPORT void ref_init_basis(cplx *psi, int n, uint64_t index)
{
    const uint64_t N = 1ull << n;
    for (uint64_t i = 0; i < N; ++i) psi[i] = 0.0;
    psi[index] = 1.0;
}

/* Balanced superposition H^{(x)n}|0>: Hadamard on every qubit of |0...0>. */
EXPORT void ref_init_uniform(cplx *psi, int n)
{
    const double r = 1.0 / sqrt(2.0);
    const double h[8] = {r, 0, r, 0, r, 0, -r, 0};
    ref_init_basis(psi, n, 0);
    for (int q = 0; q < n; ++q) ref_apply_1q(psi, n, q, h);
}

/* Seeded random state: amplitude i = (2u-1) + i(2v-1) with u, v the 53-bit
 * uniforms of Philox(key = seed, counter = (i_lo, i_hi, TAG_INIT_RANDOM, 0))
 * words (0,1) and (2,3); then divided by the 2-norm. */
static cplx random_amp(uint64_t seed, uint64_t i)
{
    uint32_t x[4];
    philox_draw(seed, (uint32_t)i, (uint32_t)(i >> 32), TAG_INIT_RANDOM, x);
    return (2.0 * u53(x[0], x[1]) - 1.0) + I * (2.0 * u53(x[2], x[3]) - 1.0);
}

/* The amplitudes of indices first .. first + count - 1 before the division by
 * the norm (any index below 2^64, so registers too large to hold here can be
 * checked at chosen indices). */
EXPORT void ref_random_raw(uint64_t seed, uint64_t first, uint64_t count, cplx *out)
{
    for (uint64_t k = 0; k < count; ++k) out[k] = random_amp(seed, first + k);
}

EXPORT void ref_init_random(cplx *psi, int n, uint64_t seed)
{
    const uint64_t N = 1ull << n;
#pragma omp parallel for schedule(static)
    for (uint64_t i = 0; i < N; ++i) psi[i] = random_amp(seed, i);
    ldbl s = 0;
    for (uint64_t i = 0; i < N; ++i) s += (ldbl)creal(psi[i]) * creal(psi[i]) + (ldbl)cimag(psi[i]) * cimag(psi[i]);
    const double inv = (double)(1.0L / sqrtl(s));
#pragma omp parallel for schedule(static)
    for (uint64_t i = 0; i < N; ++i) psi[i] *= inv;
}

/* ------------------------------------------------------------------------ */
/* Max-Cut cost and its phase                                                */

/* C(k) = sum over edges (u,v) of w_uv [k_u != k_v]  (w = 1 when w == NULL). */
static double cut_value(uint64_t k, int E, const int32_t *edges, const double *w)
{
    double c = 0.0;
    for (int e = 0; e < E; ++e) {
        const int bu = (int)((k >> edges[2 * e]) & 1), bv = (int)((k >> edges[2 * e + 1]) & 1);
        if (bu != bv) c += w ? w[e] : 1.0;
    }
    return c;
}

EXPORT double ref_cut_value(uint64_t k, int E, const int32_t *edges, const double *w)
{
    return cut_value(k, E, edges, w);
}

/* E_exact = max over all 2^n bipartitions k of C(k), by enumeration; the
 * smallest k attaining it goes to *argmax.  The approximation ratio of the
 * swarm study divides the best <C> by this value. */
EXPORT double ref_cut_max(int n, int E, const int32_t *edges, const double *w, uint64_t *argmax)
{
    const uint64_t N = 1ull << n;
    double best = -INFINITY;
    uint64_t arg = 0;
#pragma omp parallel
    {
        double tb = -INFINITY;
        uint64_t ta = 0;
#pragma omp for schedule(static)
        for (uint64_t k = 0; k < N; ++k) {
            const double c = cut_value(k, E, edges, w);
            if (c > tb) { tb = c; ta = k; }
        }
#pragma omp critical
        {
            if (tb > best || (tb == best && ta < arg)) { best = tb; arg = ta; }
        }
    }
    if (argmax) *argmax = arg;
    return best;
}

/* a_k <- exp(-i gamma C(k)) a_k: the QAOA cost layer, diagonal in the
 * computational basis. */
EXPORT void ref_apply_cut_phase(cplx *psi, int n, int E, const int32_t *edges, const double *w, double gamma)
{
    const uint64_t N = 1ull << n;
#pragma omp parallel for schedule(static)
    for (uint64_t k = 0; k < N; ++k) {
        const double c = cut_value(k, E, edges, w);
        psi[k] *= cexp(-I * gamma * c);
    }
}

/* ------------------------------------------------------------------------ */
/* Read-outs                                                                 */

EXPORT double ref_norm2(const cplx *psi, int n)
{
    const uint64_t N = 1ull << n;
    ldbl s = 0;
    for (uint64_t i = 0; i < N; ++i) s += (ldbl)creal(psi[i]) * creal(psi[i]) + (ldbl)cimag(psi[i]) * cimag(psi[i]);
    return (double)s;
}

/* GetProbability(q): P(q = 1) = sum over i with i_q = 1 of |a_i|^2. */
EXPORT double ref_prob_one(const cplx *psi, int n, int q)
{
    const uint64_t N = 1ull << n;
    ldbl s = 0;
    for (uint64_t i = 0; i < N; ++i)
        if ((i >> q) & 1) s += (ldbl)creal(psi[i]) * creal(psi[i]) + (ldbl)cimag(psi[i]) * cimag(psi[i]);
    return (double)s;
}

/* Projective measurement of qubit q with a given outcome: P = sum of |a_i|^2
 * over i with bit q = outcome; amplitudes with the other bit value become 0,
 * the rest are divided by sqrt(P) (all become 0 if P = 0).  Returns P. */
EXPORT double ref_collapse(cplx *psi, int n, int q, int outcome)
{
    const uint64_t N = 1ull << n, s = 1ull << q, want = outcome ? s : 0;
    ldbl p = 0;
    for (uint64_t i = 0; i < N; ++i)
        if ((i & s) == want) p += (ldbl)creal(psi[i]) * creal(psi[i]) + (ldbl)cimag(psi[i]) * cimag(psi[i]);
    const double scale = p > 0 ? (double)(1.0L / sqrtl(p)) : 0.0;
    for (uint64_t i = 0; i < N; ++i) psi[i] = (i & s) == want ? psi[i] * scale : 0.0;
    return (double)p;
}

/* Born-rule measurement of qubit q: u = u53(x0, x1) of Philox4x32-10(key =
 * seed, counter = (q, 0, 6, 0)); outcome 1 iff u < P1 / (P0 + P1), then the
 * state collapses onto it.  Returns the outcome; *prob = its probability. */
EXPORT int ref_measure(cplx *psi, int n, int q, uint64_t seed, double *prob)
{
    const uint64_t N = 1ull << n, s = 1ull << q;
    ldbl p0 = 0, p1 = 0;
    for (uint64_t i = 0; i < N; ++i) {
        const ldbl m = (ldbl)creal(psi[i]) * creal(psi[i]) + (ldbl)cimag(psi[i]) * cimag(psi[i]);
        if (i & s) p1 += m; else p0 += m;
    }
    uint32_t x[4];
    philox_draw(seed, (uint32_t)q, 0u, TAG_MEASURE, x);
    const double u = u53(x[0], x[1]);
    const int outcome = u < (double)p1 / ((double)p0 + (double)p1);
    const double p = ref_collapse(psi, n, q, outcome);
    if (prob) *prob = p;
    return outcome;
}

/* <Z_q> = P(0) - P(1) = 1 - 2 P(1) for a normalised state; written as the
 * plain sum of (-1)^{i_q} |a_i|^2 so it holds for any norm. */
EXPORT void ref_expect_z_all(const cplx *psi, int n, double *out)
{
    const uint64_t N = 1ull << n;
    for (int q = 0; q < n; ++q) {
        ldbl s = 0;
        for (uint64_t i = 0; i < N; ++i) {
            const ldbl p = (ldbl)creal(psi[i]) * creal(psi[i]) + (ldbl)cimag(psi[i]) * cimag(psi[i]);
            s += ((i >> q) & 1) ? -p : p;
        }
        out[q] = (double)s;
    }
}

/* <C> = sum_k C(k) |a_k|^2. */
/* Long sums over k are taken in fixed chunks of 2^16 terms: each chunk is a
 * plain sequential long-double sum, and the chunk sums are added in chunk
 * order.  The result does not depend on the thread count, and the chunks may
 * run in parallel. */
#define SUM_CHUNK_BITS 16

EXPORT double ref_expect_cut(const cplx *psi, int n, int E, const int32_t *edges, const double *w)
{
    const uint64_t N = 1ull << n;
    const uint64_t C = N > (1ull << SUM_CHUNK_BITS) ? N >> SUM_CHUNK_BITS : 1, L = N / C;
    ldbl *part = (ldbl *)malloc(C * sizeof(ldbl));
    if (!part) return NAN;
#pragma omp parallel for schedule(static)
    for (uint64_t c = 0; c < C; ++c) {
        ldbl s = 0;
        for (uint64_t k = c * L; k < (c + 1) * L; ++k) {
            const ldbl p = (ldbl)creal(psi[k]) * creal(psi[k]) + (ldbl)cimag(psi[k]) * cimag(psi[k]);
            s += (ldbl)cut_value(k, E, edges, w) * p;
        }
        part[c] = s;
    }
    ldbl s = 0;
    for (uint64_t c = 0; c < C; ++c) s += part[c];
    free(part);
    return (double)s;
}

/* sum_k d_k |a_k|^2 for a real diagonal observable d (chunked as above). */
EXPORT double ref_expect_diag(const cplx *psi, int n, const double *d)
{
    const uint64_t N = 1ull << n;
    const uint64_t C = N > (1ull << SUM_CHUNK_BITS) ? N >> SUM_CHUNK_BITS : 1, L = N / C;
    ldbl *part = (ldbl *)malloc(C * sizeof(ldbl));
    if (!part) return NAN;
#pragma omp parallel for schedule(static)
    for (uint64_t c = 0; c < C; ++c) {
        ldbl s = 0;
        for (uint64_t k = c * L; k < (c + 1) * L; ++k) {
            const ldbl p = (ldbl)creal(psi[k]) * creal(psi[k]) + (ldbl)cimag(psi[k]) * cimag(psi[k]);
            s += (ldbl)d[k] * p;
        }
        part[c] = s;
    }
    ldbl s = 0;
    for (uint64_t c = 0; c < C; ++c) s += part[c];
    free(part);
    return (double)s;
}

/* <psi| P |psi> for the Pauli product with X on xmask-only bits, Z on
 * zmask-only bits and Y on bits in both.  Built by applying the Pauli
 * matrices one qubit at a time to a copy and taking the inner product. */
EXPORT int ref_expect_pauli(const cplx *psi, int n, uint64_t xmask, uint64_t zmask, double *out /*re,im*/)
{
    const uint64_t N = 1ull << n;
    cplx *phi = (cplx *)malloc(N * sizeof(cplx));
    if (!phi) return -1;
    memcpy(phi, psi, N * sizeof(cplx));
    const double X[8] = {0, 0, 1, 0, 1, 0, 0, 0};
    const double Y[8] = {0, 0, 0, -1, 0, 1, 0, 0};
    const double Z[8] = {1, 0, 0, 0, 0, 0, -1, 0};
    for (int q = 0; q < n; ++q) {
        const int x = (int)((xmask >> q) & 1), z = (int)((zmask >> q) & 1);
        if (x && z) ref_apply_1q(phi, n, q, Y);
        else if (x) ref_apply_1q(phi, n, q, X);
        else if (z) ref_apply_1q(phi, n, q, Z);
    }
    ldbl re = 0, im = 0;
    for (uint64_t i = 0; i < N; ++i) {
        const cplx t = conj(psi[i]) * phi[i];
        re += creal(t);
        im += cimag(t);
    }
    free(phi);
    out[0] = (double)re;
    out[1] = (double)im;
    return 0;
}

/* <a|b> = sum_i conj(a_i) b_i. */
EXPORT void ref_inner(const cplx *a, const cplx *b, int n, double *out /*re,im*/)
{
    const uint64_t N = 1ull << n;
    ldbl re = 0, im = 0;
    for (uint64_t i = 0; i < N; ++i) {
        const cplx t = conj(a[i]) * b[i];
        re += creal(t);
        im += cimag(t);
    }
    out[0] = (double)re;
    out[1] = (double)im;
}

/* Sampling: shot s draws u_s = 53-bit uniform of Philox(seed, (s_lo, s_hi,
 * TAG_SAMPLE, 0)) words 0,1 and returns the smallest i with CDF(i) > u_s,
 * CDF(i) = sum_{j<=i} |a_j|^2 summed in index order in long double and
 * rounded to FP64 (so the oracle's CDF is the exact prefix sum to well below
 * 1e-15 also over 2^31 terms).  When u_s is not below CDF(N-1) the last index
 * of nonzero probability is returned.  Also reports, per shot, the distance
 * from u_s to the nearest CDF boundary (so callers can tell which decisions
 * sit within rounding of a boundary). */
EXPORT int ref_sample(const cplx *psi, int n, int64_t shots, uint64_t seed, uint64_t *out, double *margin)
{
    const uint64_t N = 1ull << n;
    double *cdf = (double *)malloc(N * sizeof(double));
    if (!cdf) return -1;
    ldbl acc = 0.0L;
    uint64_t last_nz = 0;
    for (uint64_t i = 0; i < N; ++i) {
        const ldbl p = (ldbl)creal(psi[i]) * creal(psi[i]) + (ldbl)cimag(psi[i]) * cimag(psi[i]);
        acc += p;
        cdf[i] = (double)acc;
        if (p > 0.0L) last_nz = i;
    }
    for (int64_t s = 0; s < shots; ++s) {
        uint32_t x[4];
        philox_draw(seed, (uint32_t)s, (uint32_t)((uint64_t)s >> 32), TAG_SAMPLE, x);
        const double u = u53(x[0], x[1]);
        uint64_t lo = 0, hi = N; /* first index with cdf > u, in [0, N] */
        while (lo < hi) {
            const uint64_t mid = lo + (hi - lo) / 2;
            if (cdf[mid] > u) hi = mid; else lo = mid + 1;
        }
        uint64_t r = lo < N ? lo : last_nz;
        out[s] = r;
        if (margin) {
            double m = fabs(cdf[r] - u);
            if (r > 0) m = fmin(m, fabs(u - cdf[r - 1]));
            margin[s] = m;
        }
    }
    free(cdf);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* QAOA Max-Cut (Particle Swarm / QAOA section)                              */
/*
 * |psi(theta)> = prod_{l=1..p} exp(-i beta_l B) exp(-i gamma_l C) H^{(x)n}|0>,
 * B = sum_j X_j, C = the cut counter above; theta = [gamma_1..gamma_p,
 * beta_1..beta_p]; objective L = <psi|C|psi>.  exp(-i beta B) is the product
 * of RX_j(2 beta) = exp(-i beta X_j) over all qubits.
 */

static void rx_matrix(double theta, double u[8])
{
    const double c = cos(theta / 2.0), s = sin(theta / 2.0);
    u[0] = c; u[1] = 0; u[2] = 0; u[3] = -s;
    u[4] = 0; u[5] = -s; u[6] = c; u[7] = 0;
}

static void qaoa_prepare(cplx *psi, int n, int E, const int32_t *edges, const double *w, int p, const double *theta)
{
    ref_init_uniform(psi, n);
    for (int l = 0; l < p; ++l) {
        ref_apply_cut_phase(psi, n, E, edges, w, theta[l]);
        double u[8];
        rx_matrix(2.0 * theta[p + l], u);
        for (int j = 0; j < n; ++j) ref_apply_1q(psi, n, j, u);
    }
}

/* Prepare |psi(theta)> into psi (caller-owned, 2^n) and return <C>. */
EXPORT double ref_qaoa_state(cplx *psi, int n, int E, const int32_t *edges, const double *w, int p, const double *theta)
{
    qaoa_prepare(psi, n, E, edges, w, p, theta);
    return ref_expect_cut(psi, n, E, edges, w);
}

EXPORT double ref_qaoa_energy(int n, int E, const int32_t *edges, const double *w, int p, const double *theta)
{
    cplx *psi = (cplx *)malloc((1ull << n) * sizeof(cplx));
    if (!psi) return NAN;
    const double e = ref_qaoa_state(psi, n, E, edges, w, p, theta);
    free(psi);
    return e;
}

/* Imaginary part of <a| X_j |b> = sum_i conj(a_i) b_{i xor 2^j}. */
static ldbl im_inner_x(const cplx *a, const cplx *b, int n, int j)
{
    const uint64_t N = 1ull << n, s = 1ull << j;
    ldbl im = 0;
    for (uint64_t i = 0; i < N; ++i) im += cimag(conj(a[i]) * b[i ^ s]);
    return im;
}

/* Imaginary part of <a| C |b> = sum_k C(k) conj(a_k) b_k. */
static ldbl im_inner_cut(const cplx *a, const cplx *b, int n, int E, const int32_t *edges, const double *w)
{
    const uint64_t N = 1ull << n;
    ldbl im = 0;
    for (uint64_t k = 0; k < N; ++k) im += (ldbl)cut_value(k, E, edges, w) * cimag(conj(a[k]) * b[k]);
    return im;
}

/* Adjoint differentiation: with lambda = C psi at the output, walk the gates
 * backwards; for a gate G(t) = exp(-i t K) the derivative contribution is
 * 2 Im <lambda| K |psi> taken right after the gate (both vectors at the same
 * point), after which both vectors are multiplied by G(t)^dagger.  Each
 * RX_j(2 beta_l) contributes to d/d beta_l, each cost layer to d/d gamma_l.
 * Returns <C>, writes grad[2p]. */
EXPORT double ref_qaoa_grad(int n, int E, const int32_t *edges, const double *w, int p, const double *theta, double *grad)
{
    const uint64_t N = 1ull << n;
    cplx *psi = (cplx *)malloc(N * sizeof(cplx));
    cplx *lam = (cplx *)malloc(N * sizeof(cplx));
    if (!psi || !lam) { free(psi); free(lam); return NAN; }
    qaoa_prepare(psi, n, E, edges, w, p, theta);
    const double energy = ref_expect_cut(psi, n, E, edges, w);
    for (uint64_t k = 0; k < N; ++k) lam[k] = cut_value(k, E, edges, w) * psi[k];
    for (int l = p - 1; l >= 0; --l) {
        double uinv[8];
        rx_matrix(-2.0 * theta[p + l], uinv);
        ldbl gb = 0;
        for (int j = n - 1; j >= 0; --j) {
            gb += 2.0L * im_inner_x(lam, psi, n, j);
            ref_apply_1q(psi, n, j, uinv);
            ref_apply_1q(lam, n, j, uinv);
        }
        grad[p + l] = (double)gb;
        grad[l] = (double)(2.0L * im_inner_cut(lam, psi, n, E, edges, w));
        ref_apply_cut_phase(psi, n, E, edges, w, -theta[l]);
        ref_apply_cut_phase(lam, n, E, edges, w, -theta[l]);
    }
    free(psi);
    free(lam);
    return energy;
}

/* Central finite differences of the energy: grad_k = (L(t + h e_k) - L(t - h e_k)) / 2h. */
EXPORT void ref_qaoa_grad_fd(int n, int E, const int32_t *edges, const double *w, int p, const double *theta, double h, double *grad)
{
    double *t = (double *)malloc(2 * p * sizeof(double));
    for (int k = 0; k < 2 * p; ++k) {
        memcpy(t, theta, 2 * p * sizeof(double));
        t[k] = theta[k] + h;
        const double ep = ref_qaoa_energy(n, E, edges, w, p, t);
        t[k] = theta[k] - h;
        const double em = ref_qaoa_energy(n, E, edges, w, p, t);
        grad[k] = (ep - em) / (2.0 * h);
    }
    free(t);
}

/* ------------------------------------------------------------------------ */
/* Noise trajectories: stochastic Pauli insertion                            */
/*
 * The single-qubit depolarizing channel (1-p) rho + (p/3)(X rho X + Y rho Y +
 * Z rho Z) unravelled into pure-state trajectories: after each gate, for each
 * qubit the gate touches (q0 before q1), one Philox draw decides whether a
 * Pauli is inserted and which one.  Draw number `slot` of trajectory `t` is
 * Philox(key = seed, counter = (t, slot, TAG_TRAJ, 0)); insert iff
 * x0 < floor(p 2^32); Pauli = 1 + floor(3 x1 / 2^32) with 1 = X, 2 = Y, 3 = Z.
 */

EXPORT uint32_t ref_depol_threshold(double p)
{
    if (p <= 0.0) return 0u;
    if (p >= 1.0) return 0xFFFFFFFFu;
    return (uint32_t)floor(p * 4294967296.0);
}

/* Stochastic noise gate (Pool of multiple states: one-qubit rotations with
 * random angles whose ensemble average is the decoherence channel).  For a
 * duration d: independent rotations R_X(a_x), then R_Y(a_y), then R_Z(a_z),
 * R_P(a) = exp(-i a P / 2), with normal angles of variances d / T1, d / T1
 * and 2 d / T2 - d / T1 (inv_T1 = 1 / T1, inv_T2 = 1 / T2).  A rotation by a
 * normal angle of variance v averages to the Pauli channel that flips with
 * probability (1 - e^{-v/2}) / 2, so the three together scale the Bloch
 * vector by (e^{-d/T2}, e^{-d/T2}, e^{-d/T1}).  Normals by Box-Muller from
 * Philox(key = seed, counter = (t, gate index, 7, w)): w = 0 gives a_x (cos
 * branch) and a_y (sin branch), w = 1 gives a_z (cos branch). */
static double gauss_pair(uint64_t seed, uint32_t t, uint32_t k, uint32_t w, double *second)
{
    uint32_t x[4];
    philox_draw_w3(seed, t, k, TAG_NOISE, w, x);
    const double u1 = u53(x[0], x[1]), u2 = u53(x[2], x[3]);
    const double r = sqrt(-2.0 * log(1.0 - u1));
    const double ang = 2.0 * M_PI * u2;
    if (second) *second = r * sin(ang);
    return r * cos(ang);
}

static void noise_gate(cplx *psi, int n, int q, double d, double inv_T1, double inv_T2, uint64_t seed, uint32_t t, uint32_t k)
{
    const double vxy = d * inv_T1, vz = 2.0 * d * inv_T2 - d * inv_T1;
    double gy;
    const double gx = gauss_pair(seed, t, k, 0u, &gy);
    const double gz = gauss_pair(seed, t, k, 1u, NULL);
    const double ax = sqrt(vxy) * gx, ay = sqrt(vxy) * gy, az = sqrt(vz > 0 ? vz : 0.0) * gz;
    const double cx = cos(ax / 2), sx = sin(ax / 2), cy = cos(ay / 2), sy = sin(ay / 2), cz = cos(az / 2), sz = sin(az / 2);
    const double RX[8] = {cx, 0, 0, -sx, 0, -sx, cx, 0};
    const double RY[8] = {cy, 0, -sy, 0, sy, 0, cy, 0};
    const double RZ[8] = {cz, -sz, 0, 0, 0, 0, cz, sz};
    ref_apply_1q(psi, n, q, RX);
    ref_apply_1q(psi, n, q, RY);
    ref_apply_1q(psi, n, q, RZ);
}

/* Runs trajectory `t` in place on psi (already initialised).  Writes up to
 * log_cap insertion records (slot << 2 | pauli) and returns the number of
 * insertions.  Noise gates (kind 5, qubit q0, duration u[0]) draw no
 * insertion slots.  With psi == NULL only the draws are made (the insertion
 * decisions do not depend on the state). */
EXPORT int ref_traj_run_one(cplx *psi, int n, const ref_gate *g, int count, double p, uint64_t seed, uint32_t t,
                            uint32_t *log, int log_cap, double inv_T1, double inv_T2)
{
    const double X[8] = {0, 0, 1, 0, 1, 0, 0, 0};
    const double Y[8] = {0, 0, 0, -1, 0, 1, 0, 0};
    const double Z[8] = {1, 0, 0, 0, 0, 0, -1, 0};
    const uint32_t thr = ref_depol_threshold(p);
    uint32_t slot = 0;
    int nins = 0;
    for (int k = 0; k < count; ++k) {
        if (g[k].kind == RG_NOISE) {
            if (psi) noise_gate(psi, n, g[k].q0, g[k].u[0], inv_T1, inv_T2, seed, t, (uint32_t)k);
            continue;
        }
        if (psi) apply_gate(psi, n, &g[k]);
        const int touched[2] = {g[k].q0, g[k].q1};
        const int nt = (g[k].kind == RG_1Q) ? 1 : 2;
        for (int a = 0; a < nt; ++a, ++slot) {
            uint32_t x[4];
            philox_draw(seed, t, slot, TAG_TRAJ, x);
            if (x[0] < thr) {
                const int pauli = 1 + (int)(((uint64_t)x[1] * 3u) >> 32);
                if (psi) ref_apply_1q(psi, n, touched[a], pauli == 1 ? X : (pauli == 2 ? Y : Z));
                if (log && nins < log_cap) log[nins] = (slot << 2) | (uint32_t)pauli;
                ++nins;
            }
        }
    }
    return nins;
}

/* Threads an OpenMP loop of the oracle runs on (reported with CPU timings). */
#ifdef _OPENMP
#include <omp.h>
EXPORT int ref_threads(void) { return omp_get_max_threads(); }
EXPORT void ref_set_threads(int t) { omp_set_num_threads(t > 0 ? t : 1); }
#else
EXPORT int ref_threads(void) { return 1; }
EXPORT void ref_set_threads(int t) { (void)t; }
#endif
