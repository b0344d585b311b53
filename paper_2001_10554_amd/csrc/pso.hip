// Exact Max-Cut values and a particle swarm over a pool of QAOA circuits
// (Particle Swarm / QAOA section; velocity update eq. (4)).
//
// The swarm lives on the device: a round is one pool evaluation of every
// particle's <C> (the pool's captured graph, replayed) followed by one
// kernel that folds the evaluations into the bests and moves the particles,
// so a whole run issues no host synchronisation.  Each graph's swarm is one
// workgroup of the step kernel (thread = particle).
#include <cmath>
#include <vector>

#include "common.h"

#define QS_API extern "C" __attribute__((visibility("default")))

namespace qs {

constexpr u32 kTagPso = 4, kTagPsoInit = 5;
constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr int kPsoMaxParticles = 1024;
constexpr int kPsoMaxDims = 128;

// ------------------------------------------------------------------ exact cut

// C(k) >= C(0) = 0 for the maximum, and non-negative doubles order like their
// bit patterns, so the maximum is an unsigned 64-bit atomic max on the bits;
// a second sweep takes the smallest k attaining it.  Only k with bit n-1 clear
// are visited: C(k) = C(~k), and the smaller of a complementary pair has that
// bit clear.
__global__ void k_cut_init(double *mx, u64 *arg) {
    mx[0] = 0.0;
    if (arg) arg[0] = ~0ull;
}

template <bool WEIGHTED>
__device__ __forceinline__ double cut_of(u64 k, const Graph &g, const Weights &w) {
    if (WEIGHTED) return cut_weighted(k, g, w.w);
    return (double)cut_count(k, g);
}

template <bool WEIGHTED>
__global__ __launch_bounds__(kBlock) void k_cut_max(Graph g, Weights w, u64 half, double *mx) {
    double best = 0.0;
    for (u64 k = (u64)blockIdx.x * kBlock + threadIdx.x; k < half; k += (u64)gridDim.x * kBlock) {
        const double c = cut_of<WEIGHTED>(k, g, w);
        best = c > best ? c : best;
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const double o = __shfl_xor(best, d, 64);
        best = o > best ? o : best;
    }
    if ((threadIdx.x & 63) == 0 && best > 0.0)
        atomicMax((unsigned long long *)mx, (unsigned long long)__double_as_longlong(best));
}

template <bool WEIGHTED>
__global__ __launch_bounds__(kBlock) void k_cut_argmax(Graph g, Weights w, u64 half, const double *mx, u64 *arg) {
    const double target = mx[0];
    u64 first = ~0ull;
    for (u64 k = (u64)blockIdx.x * kBlock + threadIdx.x; k < half; k += (u64)gridDim.x * kBlock) {
        if (k >= first) break;  // this thread's later k cannot be smaller
        if (cut_of<WEIGHTED>(k, g, w) == target) first = k;
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const u64 o = __shfl_xor(first, d, 64);
        first = o < first ? o : first;
    }
    if ((threadIdx.x & 63) == 0 && first != ~0ull) atomicMin((unsigned long long *)arg, (unsigned long long)first);
}

// ------------------------------------------------------------------ swarm

struct SwarmPtrs {
    double *pos, *vel, *pbest, *pbest_val, *gbest, *gbest_val, *E;
};

__global__ void k_pso_init(SwarmPtrs s, int G, int R, int D, u32 k0, u32 k1) {
    const u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    const u64 total = (u64)G * R * D;
    if (i < total) {
        const u32 c = (u32)(i / D), d = (u32)(i % D);
        const Philox4 x = philox4x32_10(c, d, kTagPsoInit, 0u, k0, k1);
        const double p = kTwoPi * u53(x.v[0], x.v[1]);
        s.pos[i] = p;
        s.vel[i] = kTwoPi * u53(x.v[2], x.v[3]);
        s.pbest[i] = p;
        if (d == 0) s.pbest_val[c] = -INFINITY;
    }
    if (i < (u64)G * D) s.gbest[i] = 0.0;
    if (i < (u64)G) s.gbest_val[i] = -INFINITY;
}

// Block g = swarm of graph g, thread k = particle k.  The update keeps the
// operation order of eq. (4) with no fused multiply-adds, so it rounds like
// a plain evaluation of the formula.
__global__ void k_pso_step(SwarmPtrs s, int R, int D, int round, int move, double omega, double phi_p, double phi_g, double attract,
                           u32 k0, u32 k1, double *history) {
#pragma clang fp contract(off)
    __shared__ double sv[kPsoMaxParticles];
    __shared__ int si[kPsoMaxParticles];
    __shared__ int take;
    const int g = blockIdx.x, k = threadIdx.x;
    const u64 c = (u64)g * R + k;
    double *pos = s.pos + c * D, *pb = s.pbest + c * D, *gb = s.gbest + (u64)g * D;
    double pv = -INFINITY;
    if (k < R) {
        pv = s.pbest_val[c];
        const double e = s.E[c];
        if (e > pv) {
            pv = e;
            s.pbest_val[c] = e;
            for (int d = 0; d < D; ++d) pb[d] = pos[d];
        }
    }
    sv[k] = pv;
    si[k] = k;
    __syncthreads();
    // lowest index among the largest personal bests
    for (int h = (int)blockDim.x >> 1; h >= 1; h >>= 1) {
        if (k < h) {
            const double a = sv[k], b = sv[k + h];
            if (b > a || (b == a && si[k + h] < si[k])) {
                sv[k] = b;
                si[k] = si[k + h];
            }
        }
        __syncthreads();
    }
    if (k == 0) {
        take = sv[0] > s.gbest_val[g] ? si[0] : -1;
        if (take >= 0) s.gbest_val[g] = sv[0];
        if (history) history[g] = take >= 0 ? sv[0] : s.gbest_val[g];
    }
    __syncthreads();
    if (take >= 0) {
        const double *src = s.pbest + ((u64)g * R + take) * D;
        for (int d = k; d < D; d += blockDim.x) gb[d] = src[d];
    }
    __syncthreads();
    if (!move || k >= R) return;
    const Philox4 x = philox4x32_10((u32)c, (u32)round, kTagPso, 0u, k0, k1);
    const double rp = u53(x.v[0], x.v[1]), rg = u53(x.v[2], x.v[3]);
    const double cp = phi_p * rp, cg = phi_g * rg;
    double *vel = s.vel + c * D;
    for (int d = 0; d < D; ++d) {
        const double th = pos[d];
        const double to_p = (pb[d] - th) * attract, to_g = (gb[d] - th) * attract;
        const double v = omega * vel[d] + cp * to_p + cg * to_g;
        vel[d] = v;
        pos[d] = th + v;
    }
}

static int check_swarm(const qs_pool_desc *d, const qs_pso_swarm *sw) {
    if (!d || !sw) return fail(QS_ERR_ARG, "null pool descriptor or swarm");
    if (d->num_graphs < 1 || d->sets_per_graph < 1 || d->p < 1) return fail(QS_ERR_ARG, "swarm needs graphs, particles and p >= 1");
    if (d->sets_per_graph > kPsoMaxParticles) return fail(QS_ERR_ARG, "at most 1024 particles per swarm");
    if (2 * d->p > kPsoMaxDims) return fail(QS_ERR_ARG, "swarm positions hold at most 128 coordinates (p <= 64)");
    if ((long long)d->num_graphs * d->sets_per_graph > (1ll << 30)) return fail(QS_ERR_ARG, "too many particles");
    if (!sw->pos || !sw->vel || !sw->pbest || !sw->pbest_val || !sw->gbest || !sw->gbest_val || !sw->E)
        return fail(QS_ERR_ARG, "null swarm array");
    return QS_OK;
}

static SwarmPtrs ptrs(const qs_pso_swarm *sw) {
    return SwarmPtrs{sw->pos, sw->vel, sw->pbest, sw->pbest_val, sw->gbest, sw->gbest_val, sw->E};
}

static int launch_pso_init(const qs_pool_desc *d, u64 seed, const qs_pso_swarm *sw, hipStream_t st) {
    const int G = d->num_graphs, R = d->sets_per_graph, D = 2 * d->p;
    const u64 total = (u64)G * R * D;
    hipLaunchKernelGGL(k_pso_init, dim3(grid_for(total, 256)), dim3(256), 0, st, ptrs(sw), G, R, D, (u32)seed, (u32)(seed >> 32));
    QS_LAUNCH_CHECK("pso_init");
    return QS_OK;
}

static int launch_pso_step(const qs_pool_desc *d, const qs_pso_params *prm, int round, int move, u64 seed, const qs_pso_swarm *sw,
                           double *history, hipStream_t st) {
    const int R = d->sets_per_graph, D = 2 * d->p;
    int threads = 64;
    while (threads < R) threads <<= 1;
    hipLaunchKernelGGL(k_pso_step, dim3(d->num_graphs), dim3(threads), 0, st, ptrs(sw), R, D, round, move, prm->omega, prm->phi_p,
                       prm->phi_g, (double)(prm->attract >= 0 ? 1 : -1), (u32)seed, (u32)(seed >> 32), history);
    QS_LAUNCH_CHECK("pso_step");
    return QS_OK;
}

}  // namespace qs

using namespace qs;

QS_API int qs_cut_max(const qs_pool_desc *d, const double *w, double *max_dev, uint64_t *argmax_dev, void *stream) {
    try {
        if (!d || !d->n_qubits || !d->edge_offset || !d->edges || !max_dev) return fail(QS_ERR_ARG, "null cut-max argument");
        if (d->num_graphs < 1 || d->edge_offset[0] != 0) return fail(QS_ERR_ARG, "cut max needs >= 1 graph and edge_offset[0] = 0");
        hipStream_t st = (hipStream_t)stream;
        for (int gi = 0; gi < d->num_graphs; ++gi) {
            const int n = d->n_qubits[gi];
            if (n < 1 || n > QS_MAX_QUBITS_C128) return fail(QS_ERR_ARG, "cut max: qubit count must be in [1, 34]");
            const int e0 = d->edge_offset[gi], ne = d->edge_offset[gi + 1] - e0;
            if (ne < 0 || ne > kMaxEdges) return fail(QS_ERR_ARG, "cut max: 0..256 edges per graph");
            Graph g{};
            Weights W{};
            g.ne = ne;
            g.weighted = w != nullptr;
            for (int e = 0; e < ne; ++e) {
                const int a = d->edges[2 * (e0 + e)], b = d->edges[2 * (e0 + e) + 1];
                if (a < 0 || b < 0 || a >= n || b >= n || a == b) return fail(QS_ERR_ARG, "cut max: edge out of range or self-loop");
                g.uv[e] = pack_edge(a, b);
                W.w[e] = w ? w[e0 + e] : 1.0;
            }
            const u64 half = 1ull << (n - 1);
            const unsigned blocks = grid_for(half, kBlock) < 16384 ? grid_for(half, kBlock) : 16384;
            double *mx = max_dev + gi;
            u64 *arg = argmax_dev ? argmax_dev + gi : nullptr;
            hipLaunchKernelGGL(k_cut_init, dim3(1), dim3(1), 0, st, mx, arg);
            if (w) {
                hipLaunchKernelGGL(k_cut_max<true>, dim3(blocks), dim3(kBlock), 0, st, g, W, half, mx);
                if (arg) hipLaunchKernelGGL(k_cut_argmax<true>, dim3(blocks), dim3(kBlock), 0, st, g, W, half, mx, arg);
            } else {
                hipLaunchKernelGGL(k_cut_max<false>, dim3(blocks), dim3(kBlock), 0, st, g, W, half, mx);
                if (arg) hipLaunchKernelGGL(k_cut_argmax<false>, dim3(blocks), dim3(kBlock), 0, st, g, W, half, mx, arg);
            }
            QS_LAUNCH_CHECK("cut_max");
        }
        return QS_OK;
    } catch (...) {
        return fail(QS_ERR_UNSUPPORTED, "unexpected internal error");
    }
}

QS_API int qs_pso_init(const qs_pool_desc *d, uint64_t seed, const qs_pso_swarm *sw, void *stream) {
    try {
        if (int rc = check_swarm(d, sw)) return rc;
        return launch_pso_init(d, seed, sw, (hipStream_t)stream);
    } catch (...) {
        return fail(QS_ERR_UNSUPPORTED, "unexpected internal error");
    }
}

QS_API int qs_pso_step(const qs_pool_desc *d, const qs_pso_params *prm, int round, int move, uint64_t seed, const qs_pso_swarm *sw,
                       double *history_dev, void *stream) {
    try {
        if (int rc = check_swarm(d, sw)) return rc;
        if (!prm || round < 0) return fail(QS_ERR_ARG, "null swarm parameters or negative round");
        return launch_pso_step(d, prm, round, move, seed, sw, history_dev, (hipStream_t)stream);
    } catch (...) {
        return fail(QS_ERR_UNSUPPORTED, "unexpected internal error");
    }
}

QS_API int qs_pso_run(const qs_pool_desc *d, const qs_pso_params *prm, int rounds, uint64_t seed, const qs_pso_swarm *sw,
                      double *history_dev, void *ws, size_t ws_bytes, void *stream) {
    try {
        if (int rc = check_swarm(d, sw)) return rc;
        if (!prm || rounds < 1 || !history_dev) return fail(QS_ERR_ARG, "swarm run needs parameters, rounds >= 1 and a history array");
        hipStream_t st = (hipStream_t)stream;
        if (int rc = launch_pso_init(d, seed, sw, st)) return rc;
        for (int r = 0; r < rounds; ++r) {
            if (int rc = qs_pool_run(d, sw->pos, sw->E, nullptr, ws, ws_bytes, stream)) return rc;
            if (int rc = launch_pso_step(d, prm, r, r + 1 < rounds, seed, sw, history_dev + (size_t)r * d->num_graphs, st)) return rc;
        }
        return QS_OK;
    } catch (...) {
        return fail(QS_ERR_UNSUPPORTED, "unexpected internal error");
    }
}
