// Read-out kernels: probabilities / <Z_q> of every qubit in one pass,
// diagonal and Pauli expectations, inner products, and sampling.
//
// Every reduction is two-stage and deterministic: stage 1 gives each block a
// fixed contiguous chunk and writes one FP64 partial per output; stage 2 is a
// single block that sums the partials in a fixed order.  Results are therefore
// bit-identical from run to run (for a given n), and always accumulate in
// FP64, also for complex64 states.
#include "launch.h"
#include "vec.h"

namespace qs {

// Sum over the block; every lane of wave 0 returns the total.  Wave level is a
// butterfly over xor-shuffles, then the 4 wave sums are added in order.
__device__ __forceinline__ double block_sum(double v, double *sh) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    double t = 0.0;
    for (int k = 0; k < kBlock / 64; ++k) t += sh[k];
    return t;
}

// ------------------------------------------------------------------ marginals: norm and P(q = 1) for all q
// Block b owns amplitudes [b 2^c, (b+1) 2^c); thread t reads b 2^c + 256 j + t.
// So index bits 0..7 are fixed per thread, bits 8..c-1 run with j and bits >= c
// are fixed per block.  A thread keeps its total and one partial per j-bit:
// the low 4 j-bits are resolved at compile time inside an unrolled group of 16
// loads, the upper ones once per group.  partial layout: [block][1 + n] =
// (sum |a|^2, P(q=1) for q = 0..n-1).

constexpr int kMaxJBits = 24;

template <typename R>
__global__ __launch_bounds__(kBlock) void k_marginals(const cx<R> *__restrict__ psi, int n, int c, double *__restrict__ partial) {
    __shared__ double sh[kBlock / 64];
    const u64 base = ((u64)blockIdx.x << c) + threadIdx.x;
    const int jb = c - 8;
    const u64 groups = 1ull << (jb - 4);
    double tot = 0.0, acc[kMaxJBits];
#pragma unroll
    for (int b = 0; b < kMaxJBits; ++b) acc[b] = 0.0;
    for (u64 jh = 0; jh < groups; ++jh) {
        double p[16];
#pragma unroll
        for (int jl = 0; jl < 16; ++jl) p[jl] = norm2d<R>(ld<true>(psi + base + ((jh * 16 + jl) << 8)));
        double s = 0, s0 = 0, s1 = 0, s2 = 0, s3 = 0;
#pragma unroll
        for (int jl = 0; jl < 16; ++jl) {
            s += p[jl];
            if (jl & 1) s0 += p[jl];
            if (jl & 2) s1 += p[jl];
            if (jl & 4) s2 += p[jl];
            if (jl & 8) s3 += p[jl];
        }
        tot += s;
        acc[0] += s0;
        acc[1] += s1;
        acc[2] += s2;
        acc[3] += s3;
#pragma unroll
        for (int b = 4; b < kMaxJBits; ++b)
            if (b < jb && ((jh >> (b - 4)) & 1)) acc[b] += s;
    }
    double *out = partial + (u64)blockIdx.x * (n + 1);
    const double btot = block_sum(tot, sh);
    if (threadIdx.x == 0) out[0] = btot;
    for (int q = 0; q < 8 && q < n; ++q) {
        const double v = block_sum(((threadIdx.x >> q) & 1) ? tot : 0.0, sh);
        if (threadIdx.x == 0) out[1 + q] = v;
    }
#pragma unroll
    for (int b = 0; b < kMaxJBits; ++b) {
        if (b < jb) {
            const double v = block_sum(acc[b], sh);
            if (threadIdx.x == 0) out[1 + 8 + b] = v;
        }
    }
    if (threadIdx.x == 0)
        for (int q = c; q < n; ++q) out[1 + q] = ((blockIdx.x >> (q - c)) & 1) ? btot : 0.0;
}

// Small states (n < 12): one block, per-amplitude bit tests.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_marginals_small(const cx<R> *__restrict__ psi, int n, double *__restrict__ partial) {
    __shared__ double sh[kBlock / 64];
    const u64 N = 1ull << n;
    double tot = 0.0, p1[12];
#pragma unroll
    for (int q = 0; q < 12; ++q) p1[q] = 0.0;
    for (u64 i = threadIdx.x; i < N; i += kBlock) {
        const double p = norm2d<R>(psi[i]);
        tot += p;
#pragma unroll
        for (int q = 0; q < 12; ++q)
            if ((i >> q) & 1) p1[q] += p;
    }
    const double t = block_sum(tot, sh);
    if (threadIdx.x == 0) partial[0] = t;
#pragma unroll
    for (int q = 0; q < 12; ++q) {
        if (q < n) {
            const double v = block_sum(p1[q], sh);
            if (threadIdx.x == 0) partial[1 + q] = v;
        }
    }
}

// Stage 2: sum partials[G][n+1] in a fixed order and map to the requested output.
__global__ __launch_bounds__(kBlock) void k_marginals_final(const double *__restrict__ partial, int G, int n, int mode, int q,
                                                            double *__restrict__ out) {
    __shared__ double sh[kBlock / 64];
    __shared__ double tot_sh;
    const int nv = n + 1;
    for (int v = 0; v < nv; ++v) {
        if (mode == kMargProbOne && v != 0 && v != 1 + q) continue;
        if (mode == kMargNorm && v != 0) break;
        double a = 0.0;
        for (int b = threadIdx.x; b < G; b += kBlock) a += partial[(u64)b * nv + v];
        const double sum = block_sum(a, sh);
        if (threadIdx.x == 0) {
            if (v == 0) {
                tot_sh = sum;
                if (mode == kMargNorm) out[0] = sum;
            } else if (mode == kMargZAll) {
                out[v - 1] = tot_sh - 2.0 * sum;
            } else if (mode == kMargProbOne) {
                out[0] = sum;
            }
        }
        __syncthreads();
    }
}

int launch_marginals(qs_state *s, int mode, int q, double *out_dev) {
    const int n = s->n;
    double *partial = s->scratch;
    int G = 1;
    if (n < 12) {
        if (s->dtype == QS_C128)
            hipLaunchKernelGGL(k_marginals_small<double>, dim3(1), dim3(kBlock), 0, s->stream, (const cx<double> *)s->buf, n, partial);
        else
            hipLaunchKernelGGL(k_marginals_small<float>, dim3(1), dim3(kBlock), 0, s->stream, (const cx<float> *)s->buf, n, partial);
    } else {
        const int c = n - 11 > 12 ? n - 11 : 12;  // at most 2048 blocks, 2^c amplitudes each
        G = 1 << (n - c);
        if (s->dtype == QS_C128)
            hipLaunchKernelGGL(k_marginals<double>, dim3(G), dim3(kBlock), 0, s->stream, (const cx<double> *)s->buf, n, c, partial);
        else
            hipLaunchKernelGGL(k_marginals<float>, dim3(G), dim3(kBlock), 0, s->stream, (const cx<float> *)s->buf, n, c, partial);
    }
    QS_LAUNCH_CHECK("marginals");
    hipLaunchKernelGGL(k_marginals_final, dim3(1), dim3(kBlock), 0, s->stream, partial, G, n, mode, q, out_dev);
    QS_LAUNCH_CHECK("marginals_final");
    return QS_OK;
}

// ------------------------------------------------------------------ generic M-output reductions over items
// Block b owns items [b*per, (b+1)*per) of `count`; the functor adds an
// item's contribution into acc[M].

template <int M, typename F>
__global__ __launch_bounds__(kBlock) void k_reduce(u64 count, u64 per, F f, double *__restrict__ partial) {
    __shared__ double sh[kBlock / 64];
    double acc[M];
#pragma unroll
    for (int m = 0; m < M; ++m) acc[m] = 0.0;
    const u64 lo = (u64)blockIdx.x * per;
    const u64 hi = lo + per < count ? lo + per : count;
    for (u64 i = lo + threadIdx.x; i < hi; i += kBlock) f(i, acc);
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const double v = block_sum(acc[m], sh);
        if (threadIdx.x == 0) partial[(u64)blockIdx.x * M + m] = v;
    }
}

template <int M> __global__ __launch_bounds__(kBlock) void k_reduce_final(const double *__restrict__ partial, int G, double *__restrict__ out) {
    __shared__ double sh[kBlock / 64];
    for (int m = 0; m < M; ++m) {
        double a = 0.0;
        for (int b = threadIdx.x; b < G; b += kBlock) a += partial[(u64)b * M + m];
        const double sum = block_sum(a, sh);
        if (threadIdx.x == 0) out[m] = sum;
    }
}

template <int M, typename F> static int run_reduce(qs_state *s, u64 count, F f, double *out_dev, const char *what) {
    u64 G = (count + kBlock * 64 - 1) / (kBlock * 64);  // >= 64 items per thread
    if (G > 2048) G = 2048;
    if (G < 1) G = 1;
    const u64 per = (count + G - 1) / G;
    hipLaunchKernelGGL((k_reduce<M, F>), dim3((unsigned)G), dim3(kBlock), 0, s->stream, count, per, f, s->scratch);
    QS_LAUNCH_CHECK(what);
    hipLaunchKernelGGL(k_reduce_final<M>, dim3(1), dim3(kBlock), 0, s->stream, s->scratch, (int)G, out_dev);
    QS_LAUNCH_CHECK(what);
    return QS_OK;
}

template <typename R> struct CutTerm {
    const cx<R> *psi;
    Graph g;
    __device__ void operator()(u64 i, double *acc) const { acc[0] += (double)cut_count(i, g) * norm2d<R>(psi[i]); }
};
template <typename R> struct CutTermW {
    const cx<R> *psi;
    Graph g;
    Weights w;
    __device__ void operator()(u64 i, double *acc) const { acc[0] += cut_weighted(i, g, w.w) * norm2d<R>(psi[i]); }
};
template <typename R> struct DiagTerm {
    const cx<R> *psi;
    const double *d;
    __device__ void operator()(u64 i, double *acc) const { acc[0] += d[i] * norm2d<R>(psi[i]); }
};

// <C> over chunks of 2^c amplitudes per block, cut values from cut_split
// (a table read and a few adds per amplitude instead of |E| bit tests).
template <typename R, bool W>
__global__ __launch_bounds__(kBlock) void k_cut_expect(const cx<R> *__restrict__ psi, int c, Graph g, Weights w, double *__restrict__ partial) {
    __shared__ double tab[1 << kCutLoopBits];
    __shared__ double red[kBlock / 64];
    const u64 base = (u64)blockIdx.x << c;
    const u32 t = threadIdx.x;
    double ct, coef[kCutLoopBits];
    cut_split<double, W>(g, w.w, t, base, c, ct, coef, tab, kBlock);
    __syncthreads();
    double acc = 0.0;
    // Four loop steps per iteration (c >= 12: at least 16 steps), loads first,
    // so each thread keeps four reads in flight.
    for (u32 j = 0; j < (1u << (c - 8)); j += 4) {
        cx<R> a[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) a[u] = psi[base + ((u64)(j + u) << 8) + t];
#pragma unroll
        for (int u = 0; u < 4; ++u) acc += cut_at<double>(ct, coef, tab, j + u) * norm2d<R>(a[u]);
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, 64);
    if ((t & 63) == 0) red[t >> 6] = acc;
    __syncthreads();
    if (t == 0) partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

int launch_expect_cut(qs_state *s, const Graph &g, const Weights *w, double *out_dev) {
    const u64 N = 1ull << s->n;
    if (s->n >= 8 + 4) {
        // chunk 2^c: at most 2^kCutLoopBits loop steps and at most 2048 blocks
        int c = s->n - 11 > 12 ? s->n - 11 : 12;
        if (c > 8 + kCutLoopBits) c = 8 + kCutLoopBits;
        const u64 G = N >> c;
        const Weights none{};
        if (G <= 2048 * 64) {
            const bool wt = w != nullptr;
            if (s->dtype == QS_C128) {
                if (wt)
                    hipLaunchKernelGGL((k_cut_expect<double, true>), dim3((unsigned)G), dim3(kBlock), 0, s->stream, (const cx<double> *)s->buf, c, g, *w,
                                       s->scratch);
                else
                    hipLaunchKernelGGL((k_cut_expect<double, false>), dim3((unsigned)G), dim3(kBlock), 0, s->stream, (const cx<double> *)s->buf, c, g,
                                       none, s->scratch);
            } else {
                if (wt)
                    hipLaunchKernelGGL((k_cut_expect<float, true>), dim3((unsigned)G), dim3(kBlock), 0, s->stream, (const cx<float> *)s->buf, c, g, *w,
                                       s->scratch);
                else
                    hipLaunchKernelGGL((k_cut_expect<float, false>), dim3((unsigned)G), dim3(kBlock), 0, s->stream, (const cx<float> *)s->buf, c, g,
                                       none, s->scratch);
            }
            QS_LAUNCH_CHECK("expect_cut");
            hipLaunchKernelGGL(k_reduce_final<1>, dim3(1), dim3(kBlock), 0, s->stream, s->scratch, (int)G, out_dev);
            QS_LAUNCH_CHECK("expect_cut");
            return QS_OK;
        }
    }
    if (s->dtype == QS_C128) {
        if (w) return run_reduce<1>(s, N, CutTermW<double>{(const cx<double> *)s->buf, g, *w}, out_dev, "expect_cut");
        return run_reduce<1>(s, N, CutTerm<double>{(const cx<double> *)s->buf, g}, out_dev, "expect_cut");
    }
    if (w) return run_reduce<1>(s, N, CutTermW<float>{(const cx<float> *)s->buf, g, *w}, out_dev, "expect_cut");
    return run_reduce<1>(s, N, CutTerm<float>{(const cx<float> *)s->buf, g}, out_dev, "expect_cut");
}

int launch_expect_diag(qs_state *s, const double *d_dev, double *out_dev) {
    const u64 N = 1ull << s->n;
    if (s->dtype == QS_C128) return run_reduce<1>(s, N, DiagTerm<double>{(const cx<double> *)s->buf, d_dev}, out_dev, "expect_diag");
    return run_reduce<1>(s, N, DiagTerm<float>{(const cx<float> *)s->buf, d_dev}, out_dev, "expect_diag");
}

// <psi|P|psi> = i^{ny} sum_i (-1)^{popc(i & z)} conj(a_{i^x}) a_i, ny = popc(x & z).
// With x != 0 the items are the pairs (i, i^x) with the top bit h of x clear,
// each contributing both of its terms; with x == 0 every amplitude is an item.
template <typename R> struct PauliTerm {
    const cx<R> *psi;
    u64 x, z;
    int h;
    __device__ void operator()(u64 k, double *acc) const {
        if (x == 0) {
            const double p = norm2d<R>(psi[k]);
            acc[0] += (__popcll(k & z) & 1) ? -p : p;
            return;
        }
        const u64 i = insert0(k, h), j = i ^ x;
        const cx<R> a = psi[i], b = psi[j];
        // conj(b) a (-1)^{popc(i&z)} + conj(a) b (-1)^{popc(j&z)}
        const double sa = (__popcll(i & z) & 1) ? -1.0 : 1.0, sb = (__popcll(j & z) & 1) ? -1.0 : 1.0;
        const double re = (double)b.x * a.x + (double)b.y * a.y, im = (double)b.x * a.y - (double)b.y * a.x;
        acc[0] += sa * re + sb * re;
        acc[1] += sa * im - sb * im;
    }
};

__global__ void k_pauli_phase(double *out, int ny) {
    // multiply (re, im) by i^{ny}
    double re = out[0], im = out[1];
    for (int k = 0; k < (ny & 3); ++k) {
        const double t = re;
        re = -im;
        im = t;
    }
    out[0] = re;
    out[1] = im;
}

int launch_expect_pauli(qs_state *s, u64 xmask, u64 zmask, double *out_dev) {
    const int n = s->n;
    const int h = xmask ? 63 - __builtin_clzll(xmask) : 0;
    const u64 count = xmask ? (1ull << (n - 1)) : (1ull << n);
    int rc;
    if (s->dtype == QS_C128)
        rc = run_reduce<2>(s, count, PauliTerm<double>{(const cx<double> *)s->buf, xmask, zmask, h}, out_dev, "expect_pauli");
    else
        rc = run_reduce<2>(s, count, PauliTerm<float>{(const cx<float> *)s->buf, xmask, zmask, h}, out_dev, "expect_pauli");
    if (rc != QS_OK) return rc;
    const int ny = __builtin_popcountll(xmask & zmask);
    if (ny & 3) {
        hipLaunchKernelGGL(k_pauli_phase, dim3(1), dim3(1), 0, s->stream, out_dev, ny);
        QS_LAUNCH_CHECK("pauli_phase");
    } else if (xmask == 0) {
        hipLaunchKernelGGL(k_pauli_phase, dim3(1), dim3(1), 0, s->stream, out_dev, 0);  // zero the unused imaginary slot
    }
    return QS_OK;
}

template <typename R> struct InnerTerm {
    const cx<R> *a, *b;
    __device__ void operator()(u64 i, double *acc) const {
        const cx<R> x = a[i], y = b[i];
        acc[0] += (double)x.x * y.x + (double)x.y * y.y;
        acc[1] += (double)x.x * y.y - (double)x.y * y.x;
    }
};

int launch_inner(qs_state *a, qs_state *b, double *out_dev) {
    const u64 N = 1ull << a->n;
    if (a->dtype == QS_C128) return run_reduce<2>(a, N, InnerTerm<double>{(const cx<double> *)a->buf, (const cx<double> *)b->buf}, out_dev, "inner");
    return run_reduce<2>(a, N, InnerTerm<float>{(const cx<float> *)a->buf, (const cx<float> *)b->buf}, out_dev, "inner");
}

// ------------------------------------------------------------------ sampling
// CDF in two levels: chunk sums of |a|^2 (2^cs amplitudes per chunk) and their
// inclusive prefix; a shot binary-searches the chunk prefix, then one
// wavefront scans its chunk 64 amplitudes at a time.

template <typename R>
__global__ __launch_bounds__(kBlock) void k_chunk_sums(const cx<R> *__restrict__ psi, int cs, double *__restrict__ csum) {
    __shared__ double sh[kBlock / 64];
    const u64 lo = (u64)blockIdx.x << cs, hi = lo + (1ull << cs);
    double a = 0.0;
    for (u64 i = lo + threadIdx.x; i < hi; i += kBlock) a += norm2d<R>(psi[i]);
    const double t = block_sum(a, sh);
    if (threadIdx.x == 0) csum[blockIdx.x] = t;
}

// One block: inclusive prefix of csum[G] into cdf[G] (thread-contiguous
// segments, then a sequential scan of the 256 segment totals), plus the last
// chunk with nonzero mass into *last.
__global__ __launch_bounds__(kBlock) void k_chunk_scan(const double *__restrict__ csum, int G, double *__restrict__ cdf, double *__restrict__ last) {
    __shared__ double seg[kBlock];
    __shared__ int lastnz[kBlock];
    const int per = (G + kBlock - 1) / kBlock;
    const int lo = threadIdx.x * per, hi = lo + per < G ? lo + per : G;
    double a = 0.0;
    int ln = -1;
    for (int b = lo; b < hi; ++b) {
        a += csum[b];
        if (csum[b] > 0.0) ln = b;
    }
    seg[threadIdx.x] = a;
    lastnz[threadIdx.x] = ln;
    __syncthreads();
    if (threadIdx.x == 0) {
        double run = 0.0;
        int l = -1;
        for (int t = 0; t < kBlock; ++t) {
            const double v = seg[t];
            seg[t] = run;
            run += v;
            if (lastnz[t] >= 0) l = lastnz[t];
        }
        last[0] = (double)(l < 0 ? 0 : l);
    }
    __syncthreads();
    double run = seg[threadIdx.x];
    for (int b = lo; b < hi; ++b) {
        run += csum[b];
        cdf[b] = run;
    }
}

template <typename R>
__device__ u64 last_nonzero_in_chunk(const cx<R> *psi, u64 lo, u64 len, int lane) {
    for (u64 r = len; r > 0;) {
        const u64 take = r >= 64 ? 64 : r;
        r -= take;
        const u64 i = lo + r + lane;
        const bool nz = (u64)lane < take && norm2d<R>(psi[i]) > 0.0;
        const u64 m = __ballot(nz);
        if (m) return lo + r + (63 - __clzll(m));
    }
    return lo;
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_sample(const cx<R> *__restrict__ psi, int n, int cs, int G, const double *__restrict__ cdf,
                                                    const double *__restrict__ last, int64_t shots, u32 k0, u32 k1, u64 *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int64_t s = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    if (s >= shots) return;
    const Philox4 x = philox4x32_10((u32)s, (u32)((u64)s >> 32), kTagSample, 0u, k0, k1);
    const double u = u53(x.v[0], x.v[1]);
    const u64 len = 1ull << cs;
    u64 result;
    if (!(u < cdf[G - 1])) {
        const u64 b = (u64)last[0];
        result = last_nonzero_in_chunk<R>(psi, b << cs, len, lane);
    } else {
        int lo = 0, hi = G - 1;  // first b with cdf[b] > u
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (cdf[mid] > u) hi = mid; else lo = mid + 1;
        }
        const u64 base = (u64)lo << cs;
        double run = lo > 0 ? cdf[lo - 1] : 0.0;
        result = ~0ull;
        for (u64 r = 0; r < len; r += 64) {
            const u64 i = base + r + lane;
            double v = (r + lane < len) ? norm2d<R>(psi[i]) : 0.0;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const double t = __shfl_up(v, d, 64);
                if (lane >= d) v += t;
            }
            const u64 m = __ballot(run + v > u);
            if (m) {
                result = base + r + (__ffsll((long long)m) - 1);
                break;
            }
            run += __shfl(v, 63, 64);
        }
        if (result == ~0ull) result = last_nonzero_in_chunk<R>(psi, base, len, lane);
    }
    if (lane == 0) out[s] = result;
}

int sample_chunk_bits(int n) { return n <= 12 ? n : (n - 18 > 12 ? n - 18 : 12); }

int launch_sample_buf(int n, int dtype, const void *buf, double *scratch, hipStream_t st, int64_t shots, u64 seed, u64 *out_dev) {
    const int cs = sample_chunk_bits(n);
    const int G = 1 << (n - cs);
    double *csum = scratch, *cdf = scratch + G, *last = scratch + 2 * (size_t)G;
    if (dtype == QS_C128)
        hipLaunchKernelGGL(k_chunk_sums<double>, dim3(G), dim3(kBlock), 0, st, (const cx<double> *)buf, cs, csum);
    else
        hipLaunchKernelGGL(k_chunk_sums<float>, dim3(G), dim3(kBlock), 0, st, (const cx<float> *)buf, cs, csum);
    QS_LAUNCH_CHECK("sample_chunks");
    hipLaunchKernelGGL(k_chunk_scan, dim3(1), dim3(kBlock), 0, st, csum, G, cdf, last);
    QS_LAUNCH_CHECK("sample_scan");
    if (shots <= 0) return QS_OK;
    const u64 blocks = ((u64)shots + 3) / 4;  // one wavefront per shot; shots <= 2^32 checked by the caller
    const u32 k0 = (u32)seed, k1 = (u32)(seed >> 32);
    if (dtype == QS_C128)
        hipLaunchKernelGGL(k_sample<double>, dim3((unsigned)blocks), dim3(kBlock), 0, st, (const cx<double> *)buf, n, cs, G, cdf, last,
                           shots, k0, k1, out_dev);
    else
        hipLaunchKernelGGL(k_sample<float>, dim3((unsigned)blocks), dim3(kBlock), 0, st, (const cx<float> *)buf, n, cs, G, cdf, last,
                           shots, k0, k1, out_dev);
    QS_LAUNCH_CHECK("sample");
    return QS_OK;
}

int launch_sample(qs_state *s, int64_t shots, u64 seed, u64 *out_dev) {
    return launch_sample_buf(s->n, s->dtype, s->buf, s->scratch, s->stream, shots, seed, out_dev);
}

}  // namespace qs
