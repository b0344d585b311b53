// Internal header of the HIP library: amplitude types, small device helpers,
// error plumbing shared by the translation units of libqsim_hip.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <string>

#include "../../include/qsim.h"

namespace qs {

using u64 = uint64_t;
using u32 = uint32_t;

// ------------------------------------------------------------------ errors
void set_error(const std::string &msg);
int fail(int code, const std::string &msg);
int hip_fail(hipError_t e, const char *where);

#define QS_HIP(call)                                          \
    do {                                                      \
        hipError_t _e = (call);                               \
        if (_e != hipSuccess) return ::qs::hip_fail(_e, #call); \
    } while (0)

#define QS_LAUNCH_CHECK(where)                                   \
    do {                                                         \
        hipError_t _e = hipGetLastError();                       \
        if (_e != hipSuccess) return ::qs::hip_fail(_e, where);  \
    } while (0)

// ------------------------------------------------------------------ amplitude types
// Amplitudes are clang ext-vector pairs (x = re, y = im): 16-byte aligned for
// c128 so one global_load_dwordx4 moves one amplitude.
typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));
template <typename R> struct Vec2;
template <> struct Vec2<double> { using T = d2v; };
template <> struct Vec2<float> { using T = f2v; };
template <typename R> using cx = typename Vec2<R>::T;

// 2x2 matrix, row-major, interleaved (re, im); row = output.
template <typename R> struct Mat2 {
    R m[8];
};

template <typename R> __host__ Mat2<R> to_mat(const double *u) {
    Mat2<R> o;
    for (int k = 0; k < 8; ++k) o.m[k] = (R)u[k];
    return o;
}

template <typename R> __device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b) {
    cx<R> r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}

// (u_r0 * a + u_r1 * b) for row r of a Mat2.
template <typename R> __device__ __forceinline__ cx<R> row_apply(const R *m, cx<R> a, cx<R> b) {
    cx<R> r;
    r.x = m[0] * a.x - m[1] * a.y + m[2] * b.x - m[3] * b.y;
    r.y = m[0] * a.y + m[1] * a.x + m[2] * b.y + m[3] * b.x;
    return r;
}

template <typename R> __device__ __forceinline__ void apply2(const Mat2<R> &u, cx<R> &a, cx<R> &b) {
    const cx<R> na = row_apply<R>(u.m, a, b);
    const cx<R> nb = row_apply<R>(u.m + 4, a, b);
    a = na;
    b = nb;
}

template <typename R> __device__ __forceinline__ double norm2d(cx<R> a) {
    return (double)a.x * (double)a.x + (double)a.y * (double)a.y;
}

// Insert a zero bit at position b of k.
__device__ __forceinline__ u64 insert0(u64 k, int b) {
    const u64 lo = k & ((1ull << b) - 1);
    return ((k >> b) << (b + 1)) | lo;
}

// ------------------------------------------------------------------ Philox4x32-10
// Salmon, Moraes, Dror, Shaw (SC'11): ten rounds of the 4x32 Philox bijection;
// multipliers 0xD2511F53 / 0xCD9E8D57, key schedule bumped by the Weyl
// constants 0x9E3779B9 / 0xBB67AE85 between rounds.
struct Philox4 {
    u32 v[4];
};

__device__ __forceinline__ Philox4 philox4x32_10(u32 c0, u32 c1, u32 c2, u32 c3, u32 k0, u32 k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const u32 lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        const u32 lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        const u32 n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return Philox4{{c0, c1, c2, c3}};
}

// Counter-word-2 stream tags (one per use of a seed).
constexpr u32 kTagInitRandom = 1, kTagSample = 2, kTagTraj = 3;

// 53-bit uniform in [0,1) from (lo, hi) words.
__device__ __forceinline__ double u53(u32 lo, u32 hi) {
    const u64 v = ((u64)hi << 32) | lo;
    return (double)(v >> 11) * (1.0 / 9007199254740992.0);
}

// ------------------------------------------------------------------ Max-Cut graph (kernel argument)
constexpr int kMaxEdges = 256;
// Edge e joins qubits uv[e] & 0xff and uv[e] >> 8.  Packed into dwords so a
// kernel reads an edge with one scalar load (there is no scalar byte load).
struct Graph {
    int ne;
    int weighted;
    uint32_t uv[kMaxEdges];
};
struct Weights {
    double w[kMaxEdges];
};
__host__ __device__ inline uint32_t pack_edge(int a, int b) { return (uint32_t)a | ((uint32_t)b << 8); }

// C(k) for unit weights: number of edges cut by bipartition k.
__device__ __forceinline__ int cut_count(u64 k, const Graph &g) {
    int c = 0;
    for (int e = 0; e < g.ne; ++e) {
        const uint32_t x = g.uv[e];
        c += (int)(((k >> (x & 0xffu)) ^ (k >> (x >> 8))) & 1u);
    }
    return c;
}

__device__ __forceinline__ double cut_weighted(u64 k, const Graph &g, const double *w) {
    double c = 0.0;
    for (int e = 0; e < g.ne; ++e) {
        const uint32_t x = g.uv[e];
        if (((k >> (x & 0xffu)) ^ (k >> (x >> 8))) & 1u) c += w[e];
    }
    return c;
}

// Cut values of a chunk of 2^c amplitudes i = base + j 2^8 + t (thread t < 256,
// loop index j < 2^(c - 8) <= 2^kCutLoopBits), for kernels that sweep a chunk
// per block.  An edge's cut bit depends on its endpoints' regions: thread bits
// [0, 8), loop bits [8, c), chunk bits [c, n).  Everything without a loop bit
// goes into the per-thread constant ct; loop-loop and loop-chunk edges into
// the per-block table tab[j] (shared memory, filled by all threads; the caller
// synchronises before reading it); a loop-thread edge (u loop, v thread) adds
// b_v + bit_u(j) (1 - 2 b_v), i.e. a per-thread coefficient of loop bit u.
// Then C(i) = ct + tab[j] + sum over set bits x of j of coef[x].
constexpr int kCutLoopBits = 11;

template <typename CT, bool W>
__device__ __forceinline__ void cut_split(const Graph &g, const double *w, u32 t, u64 base, int c, CT &ct, CT (&coef)[kCutLoopBits], CT *tab,
                                          int nthreads) {
    ct = (CT)0;
#pragma unroll
    for (int x = 0; x < kCutLoopBits; ++x) coef[x] = (CT)0;
    for (int e = 0; e < g.ne; ++e) {
        const uint32_t uv = g.uv[e];
        int a = (int)(uv & 0xffu), b = (int)(uv >> 8);
        const CT we = W ? (CT)w[e] : (CT)1;
        if (a >= 8 && a < c && !(b >= 8 && b < c)) {  // the loop endpoint (if exactly one) is b
            const int tmp = a;
            a = b;
            b = tmp;
        }
        const bool la = a >= 8 && a < c, lb = b >= 8 && b < c;
        if (la || (lb && a >= c)) continue;  // loop-loop, loop-chunk: in the table
        if (lb) {                              // a is a thread bit
            const int tb = (int)((t >> a) & 1u);
            ct += tb ? we : (CT)0;
#pragma unroll
            for (int x = 0; x < kCutLoopBits; ++x)
                if (x == b - 8) coef[x] += tb ? -we : we;
            continue;
        }
        const u64 ia = a < 8 ? (u64)t : base, ib = b < 8 ? (u64)t : base;
        if (((ia >> a) ^ (ib >> b)) & 1u) ct += we;
    }
    for (u32 j = t; j < (1u << (c - 8)); j += nthreads) {
        const u64 idx = base | ((u64)j << 8);
        CT v = (CT)0;
        for (int e = 0; e < g.ne; ++e) {
            const uint32_t uv = g.uv[e];
            const int a = (int)(uv & 0xffu), b = (int)(uv >> 8);
            if (a < 8 || b < 8 || !((a < c) || (b < c))) continue;  // needs a loop endpoint and no thread endpoint
            if (((idx >> a) ^ (idx >> b)) & 1u) v += W ? (CT)w[e] : (CT)1;
        }
        tab[j] = v;
    }
}

template <typename CT> __device__ __forceinline__ CT cut_at(CT ct, const CT (&coef)[kCutLoopBits], const CT *tab, u32 j) {
    CT v = ct + tab[j];
#pragma unroll
    for (int x = 0; x < kCutLoopBits; ++x)
        if ((j >> x) & 1u) v += coef[x];
    return v;
}

// ------------------------------------------------------------------ launch geometry
constexpr int kBlock = 256;

inline unsigned grid_for(u64 work, u64 per_block) {
    u64 g = (work + per_block - 1) / per_block;
    return (unsigned)(g ? g : 1);
}

// A HIP grid holds fewer than 2^32 work-items.  Kernels with one work unit per
// thread take a workgroup offset `blk0` and are launched in pieces of at most
// 2^23 workgroups (2^31 work-items at 256 threads); f(blocks, blk0) issues one
// piece.  Registers up to 2^31 units are a single piece.
constexpr u64 kPieceBlocks = 1ull << 23;

template <typename F> inline void for_pieces(u64 nblocks, F f) {
    if (nblocks == 0) nblocks = 1;
    for (u64 b0 = 0; b0 < nblocks; b0 += kPieceBlocks) f((unsigned)(nblocks - b0 < kPieceBlocks ? nblocks - b0 : kPieceBlocks), b0);
}

}  // namespace qs

// ------------------------------------------------------------------ handle
struct qs_state {
    int n;
    int dtype;
    void *buf;
    size_t bytes;
    hipStream_t stream;
    int device;
    double *scratch;        // device: partial sums (kScratchDoubles)
    size_t scratch_doubles;
    void *plan_cache;       // host-side cache of uploaded block plans
};

namespace qs {
constexpr size_t kScratchDoubles = (size_t)1 << 20;  // 8 MiB of partials per handle
inline size_t amp_bytes(int dtype) { return dtype == QS_C128 ? 16 : 8; }
}  // namespace qs
