// Projective measurement of one qubit and dense k-qubit gates.
//
// Measurement: one read pass sums |a_i|^2 separately for bit q = 0 and 1
// (fixed-order two-stage FP64 reduction), a one-block kernel takes the Born
// decision and the normalisation, and one pass over the pairs (i, i + 2^q)
// reads only the kept half and writes both (the other half becomes 0).  The
// decision stays on the device, so nothing waits for the host.
//
// k-qubit gates (k <= 5): thread = one group of 2^k amplitudes (the indices
// that differ only in the target bits), held in registers in FP64; every lane
// of a wave needs the same matrix entry at the same time, so the matrix is
// read through the scalar cache into SGPRs (no LDS traffic).  Rows are
// written back as they are formed, which is safe in place because the
// thread owns its group.  At k <= 3 the pass is HBM-bound (about 2^(k+1) * 4
// flops per 16-byte amplitude read and written against a ridge near 10
// flop/B); at k = 5 it approaches the FP64 vector ridge.  On this chip the
// FP64 matrix cores have the same peak as the vector units, so the
// contraction stays on the vector path.
#include "launch.h"

namespace qs {

constexpr u32 kTagMeasure = 6;

template <typename R>
__global__ __launch_bounds__(kBlock) void k_prob_bits(const cx<R> *__restrict__ psi, u64 chunk, int q, double *__restrict__ partial) {
    __shared__ double sh[2][kBlock / 64];
    const u64 lo = (u64)blockIdx.x * chunk, hi = lo + chunk;
    double p0 = 0.0, p1 = 0.0;
    for (u64 i = lo + threadIdx.x; i < hi; i += kBlock) {
        const double m = norm2d<R>(psi[i]);
        if ((i >> q) & 1)
            p1 += m;
        else
            p0 += m;
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        p0 += __shfl_xor(p0, d, 64);
        p1 += __shfl_xor(p1, d, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        sh[0][threadIdx.x >> 6] = p0;
        sh[1][threadIdx.x >> 6] = p1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        partial[2 * (u64)blockIdx.x] = sh[0][0] + sh[0][1] + sh[0][2] + sh[0][3];
        partial[2 * (u64)blockIdx.x + 1] = sh[1][0] + sh[1][1] + sh[1][2] + sh[1][3];
    }
}

// ctl[0] = 1 / sqrt(P(outcome)) (0 if that probability is 0), ctl[1] = outcome.
// outcome < 0: draw it (Born rule, Philox counter (q, 0, 6, 0)).
__global__ __launch_bounds__(kBlock) void k_measure_decide(const double *__restrict__ partial, int G, int q, int outcome, u32 k0, u32 k1,
                                                           double *__restrict__ ctl, int32_t *__restrict__ outcome_out,
                                                           double *__restrict__ prob_out) {
    __shared__ double sh[2][kBlock];
    double a0 = 0.0, a1 = 0.0;
    for (int b = threadIdx.x; b < G; b += kBlock) {
        a0 += partial[2 * b];
        a1 += partial[2 * b + 1];
    }
    sh[0][threadIdx.x] = a0;
    sh[1][threadIdx.x] = a1;
    __syncthreads();
    for (int h = kBlock / 2; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + h];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double P0 = sh[0][0], P1 = sh[1][0];
    int out = outcome;
    if (out < 0) {
        const Philox4 x = philox4x32_10((u32)q, 0u, kTagMeasure, 0u, k0, k1);
        out = u53(x.v[0], x.v[1]) < P1 / (P0 + P1) ? 1 : 0;
    }
    const double P = out ? P1 : P0;
    ctl[0] = P > 0.0 ? 1.0 / sqrt(P) : 0.0;
    ctl[1] = (double)out;
    if (outcome_out) outcome_out[0] = out;
    if (prob_out) prob_out[0] = P;
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_collapse(cx<R> *__restrict__ psi, u64 pairs, int q, const double *__restrict__ ctl) {
    const double scale = ctl[0];
    const int out = ctl[1] != 0.0;
    const u64 s = 1ull << q;
    for (u64 k = (u64)blockIdx.x * kBlock + threadIdx.x; k < pairs; k += (u64)gridDim.x * kBlock) {
        const u64 i0 = insert0(k, q), keep = out ? i0 | s : i0, drop = keep ^ s;
        cx<R> v = psi[keep];
        v.x = (R)((double)v.x * scale);
        v.y = (R)((double)v.y * scale);
        psi[keep] = v;
        cx<R> z;
        z.x = (R)0;
        z.y = (R)0;
        psi[drop] = z;
    }
}

int launch_measure(qs_state *s, int q, int outcome, u64 seed, int32_t *outcome_dev, double *prob_dev) {
    const int n = s->n;
    const u64 N = 1ull << n;
    const int c = n > 22 ? n - 11 : (n > 11 ? 11 : n);  // chunk 2^c amplitudes, at most 2048 blocks
    const int G = (int)(N >> c);
    double *partial = s->scratch, *ctl = s->scratch + 2 * (size_t)G;
    if (s->dtype == QS_C128)
        hipLaunchKernelGGL(k_prob_bits<double>, dim3(G), dim3(kBlock), 0, s->stream, (const cx<double> *)s->buf, 1ull << c, q, partial);
    else
        hipLaunchKernelGGL(k_prob_bits<float>, dim3(G), dim3(kBlock), 0, s->stream, (const cx<float> *)s->buf, 1ull << c, q, partial);
    hipLaunchKernelGGL(k_measure_decide, dim3(1), dim3(kBlock), 0, s->stream, partial, G, q, outcome, (u32)seed, (u32)(seed >> 32), ctl,
                       outcome_dev, prob_dev);
    const u64 pairs = N >> 1;
    const unsigned grid = grid_for(pairs, (u64)kBlock * 4) < 65536 ? grid_for(pairs, (u64)kBlock * 4) : 65536;
    if (s->dtype == QS_C128)
        hipLaunchKernelGGL(k_collapse<double>, dim3(grid), dim3(kBlock), 0, s->stream, (cx<double> *)s->buf, pairs, q, ctl);
    else
        hipLaunchKernelGGL(k_collapse<float>, dim3(grid), dim3(kBlock), 0, s->stream, (cx<float> *)s->buf, pairs, q, ctl);
    QS_LAUNCH_CHECK("measure");
    return QS_OK;
}

// ------------------------------------------------------------------ k-qubit gates

struct KqArgs {
    u64 off[32];  // off[j] = sum_m j_m 2^{qubit m}
    int sorted[5];  // target positions, ascending
};

template <typename R, int K>
__global__ __launch_bounds__(kBlock) void k_apply_kq(cx<R> *__restrict__ psi, u64 groups, KqArgs a, const d2v *__restrict__ U, u64 blk0) {
    constexpr int D = 1 << K;
    const u64 g = (blk0 + blockIdx.x) * kBlock + threadIdx.x;
    if (g >= groups) return;
    u64 base = g;
#pragma unroll
    for (int m = 0; m < K; ++m) base = insert0(base, a.sorted[m]);
    d2v in[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        const cx<R> v = psi[base + a.off[j]];
        in[j].x = (double)v.x;
        in[j].y = (double)v.y;
    }
    // One row at a time: the row's entries are wave-uniform and arrive through
    // scalar loads, so the inner product takes its matrix operands from SGPRs.
#pragma unroll 1
    for (int r = 0; r < D; ++r) {
        double ar = 0.0, ai = 0.0;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const d2v u = U[r * D + j];
            ar += u.x * in[j].x - u.y * in[j].y;
            ai += u.x * in[j].y + u.y * in[j].x;
        }
        cx<R> o;
        o.x = (R)ar;
        o.y = (R)ai;
        psi[base + a.off[r]] = o;
    }
}

template <typename R>
static void launch_kq_t(qs_state *s, int k, u64 groups, const KqArgs &a, const d2v *U, u64 blocks) {
    cx<R> *psi = (cx<R> *)s->buf;
    for_pieces(blocks, [&](unsigned grid, u64 b0) {
        switch (k) {
        case 1: hipLaunchKernelGGL((k_apply_kq<R, 1>), dim3(grid), dim3(kBlock), 0, s->stream, psi, groups, a, U, b0); break;
        case 2: hipLaunchKernelGGL((k_apply_kq<R, 2>), dim3(grid), dim3(kBlock), 0, s->stream, psi, groups, a, U, b0); break;
        case 3: hipLaunchKernelGGL((k_apply_kq<R, 3>), dim3(grid), dim3(kBlock), 0, s->stream, psi, groups, a, U, b0); break;
        case 4: hipLaunchKernelGGL((k_apply_kq<R, 4>), dim3(grid), dim3(kBlock), 0, s->stream, psi, groups, a, U, b0); break;
        default: hipLaunchKernelGGL((k_apply_kq<R, 5>), dim3(grid), dim3(kBlock), 0, s->stream, psi, groups, a, U, b0); break;
        }
    });
}

int launch_apply_kq(qs_state *s, const int32_t *qubits, int k, const double *U_dev) {
    KqArgs a{};
    for (int j = 0; j < (1 << k); ++j) {
        u64 o = 0;
        for (int m = 0; m < k; ++m)
            if ((j >> m) & 1) o |= 1ull << qubits[m];
        a.off[j] = o;
    }
    for (int m = 0; m < k; ++m) a.sorted[m] = qubits[m];
    for (int i = 1; i < k; ++i)
        for (int j = i; j > 0 && a.sorted[j - 1] > a.sorted[j]; --j) {
            const int t = a.sorted[j];
            a.sorted[j] = a.sorted[j - 1];
            a.sorted[j - 1] = t;
        }
    const u64 groups = 1ull << (s->n - k);
    const u64 grid = (groups + kBlock - 1) / kBlock;  // launched in pieces of at most 2^23 blocks
    if (s->dtype == QS_C128)
        launch_kq_t<double>(s, k, groups, a, (const d2v *)U_dev, grid);
    else
        launch_kq_t<float>(s, k, groups, a, (const d2v *)U_dev, grid);
    QS_LAUNCH_CHECK("apply_kq");
    return QS_OK;
}

}  // namespace qs
