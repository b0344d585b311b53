// QAOA Max-Cut: fused forward passes and the adjoint (reverse) sweep, batched
// over circuits.
//
// Circuit: |psi> = prod_l exp(-i beta_l B) exp(-i gamma_l C) H^n |0>, with
// B = sum_j X_j (so exp(-i beta B) = prod_j RX_j(2 beta)) and C the cut
// counter; E = <psi|C|psi>.
//
// Pass structure.  The qubits are split into groups: G_0 = the TB lowest
// qubits, then groups of at most TB - r higher qubits (their tiles also hold
// qubits 0..r-1 so every row is a 2^r-amplitude contiguous run).  Layer l is
// P passes, pass (l, g) applying RX(2 beta_l) to the qubits of G_g.  The
// diagonal cost layers ride along: exp(-i gamma_1 C) is applied at the start
// of the very first pass (on the uniform state generated in registers), and
// exp(-i gamma_{l+1} C) at the end of pass (l, P-1).  The last pass also
// accumulates E.
//
// Adjoint.  The forward writes every pass's output as a checkpoint.  The
// backward walks the passes in reverse with lambda (lambda = C psi at the
// end).  A phase at the end of a pass gives 2 Im<lambda|C|psi> there and is
// then undone on both vectors element-wise; then the pass's RX gates are
// undone one qubit at a time on both vectors, each preceded by its inner
// product 2 Im<lambda|X_j|psi> (both vectors at the same point; the RX gates
// of one mixer commute with every X_j).  The first pass's phase sits at its
// start, so its inner product uses psi regenerated on the fly
// (exp(-i gamma_1 C(k)) 2^{-n/2}).  Inner products are per-block FP64
// partial sums, reduced in a fixed order.
//
// Register tiles (n >= 10).  A tile of 2^TB amplitudes is held by 2^TT
// threads, 2^(TB-TT) amplitudes per thread, in one of two layouts:
//   L0: tile index m = t | j << TT;
//   L1: m = lane | (j mod 2^W) << 6 | wave << TT | (j >> W) << (TT + W),
// with t = wave * 64 + lane, W = TT - 6 wave bits.  Gates on register-index
// bits act inside a thread, gates on lane bits exchange with the partner lane
// (wavefront shuffle), and one LDS transpose between L0 and L1 reaches the
// remaining (wave) bits.  So a pass touches LDS once per vector, instead of
// once per gate.  Small registers (n < 10) use the LDS kernels.
//
// Cut values.  C(k) is never evaluated edge by edge per amplitude: each edge
// is classified once per pass and layout by where its endpoints sit
// (thread-index bit, register-index bit, or a qubit fixed per tile), and a
// thread folds the edges into a constant plus one coefficient per register
// bit.
//
// Batching.  blockIdx.x = circuit * G + tile; circuit c owns the workspace
// region ws + c * circ_bytes.
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "launch.h"
#include "qaoa.h"
#include "vec.h"

#define QS_API extern "C" __attribute__((visibility("default")))

namespace qs {

constexpr int kLdsThreads = 256;  // LDS kernels: m = tid + 256 j

// Cut value of the thread's 2^JB amplitudes for edge list `list`.  CT = int
// (unit weights) or double.
template <typename CT, int JB>
__device__ __forceinline__ void cut_values(const QPass &P, int list, const QWeights &W, bool weighted, u64 base, int tid, CT (&C)[1 << JB]) {
    constexpr int R = 1 << JB;
    CT cb = 0;
    CT coef[JB > 0 ? JB : 1] = {};
    int k = 0;
    const QEdge *E = P.e[list];
    const int32_t *cnt = P.cnt[list];
    auto wt = [&](const QEdge &e) -> CT { return weighted ? (CT)W.w[e.wi] : (CT)1; };
#pragma unroll 4
    for (int i = 0; i < cnt[EC_TT]; ++i, ++k) {
        const QEdge e = E[k];
        cb += (((tid >> e.a) ^ (tid >> e.b)) & 1) ? wt(e) : (CT)0;
    }
#pragma unroll 4
    for (int i = 0; i < cnt[EC_TR]; ++i, ++k) {
        const QEdge e = E[k];
        cb += (((tid >> e.a) & 1) != (int)((base >> e.b) & 1)) ? wt(e) : (CT)0;
    }
#pragma unroll 4
    for (int i = 0; i < cnt[EC_TJ]; ++i, ++k) {
        const QEdge e = E[k];
        const int ta = (tid >> e.a) & 1;
        const CT w = wt(e);
        cb += ta ? w : (CT)0;
#pragma unroll
        for (int x = 0; x < JB; ++x)
            if (x == e.b) coef[x] += ta ? -w : w;
    }
    const int kjj = k;
    k += cnt[EC_JJ];
#pragma unroll 4
    for (int i = 0; i < cnt[EC_JR]; ++i, ++k) {
        const QEdge e = E[k];
        const int br = (int)((base >> e.b) & 1);
        const CT w = wt(e);
        cb += br ? w : (CT)0;
#pragma unroll
        for (int x = 0; x < JB; ++x)
            if (x == e.a) coef[x] += br ? -w : w;
    }
#pragma unroll 4
    for (int i = 0; i < cnt[EC_RR]; ++i, ++k) {
        const QEdge e = E[k];
        cb += (((base >> e.a) ^ (base >> e.b)) & 1) ? wt(e) : (CT)0;
    }
#pragma unroll
    for (int j = 0; j < R; ++j) {
        CT c = cb;
#pragma unroll
        for (int x = 0; x < JB; ++x)
            if ((j >> x) & 1) c += coef[x];
        C[j] = c;
    }
#pragma unroll 4
    for (int i = 0; i < cnt[EC_JJ]; ++i) {
        const QEdge e = E[kjj + i];
        const CT w = wt(e);
#pragma unroll
        for (int j = 0; j < R; ++j)
            if (((j >> e.a) ^ (j >> e.b)) & 1) C[j] += w;
    }
}

// Entry i of a byte array of the pass descriptor, read through its aligned
// 32-bit word: gfx950 has no scalar byte load, so a byte read from a
// descriptor in global memory (pooled launches) would be a vector load per
// entry; the word is a scalar load.
__device__ __forceinline__ int pbyte(const uint8_t *arr, int i) {
    return (int)((reinterpret_cast<const uint32_t *>(arr)[i >> 2] >> (8 * (i & 3))) & 255u);
}

// Bit deposits through the pass's qubit maps, over the arrays' full static
// length: each entry is read at a fixed kernel-argument offset (hoisted scalar
// loads) instead of one dependent memory access per bit.
__device__ __forceinline__ u64 qtile_base(const QPass &P, u64 tile) {
    u64 base = 0;
#pragma unroll
    for (int b = 0; b < 40; ++b)
        if (b < P.nrest) base |= ((tile >> b) & 1ull) << pbyte(P.rest, b);
    return base;
}

__device__ __forceinline__ u64 qtile_off(const QPass &P, u64 m) {
    u64 off = 0;
#pragma unroll
    for (int b = 0; b < 16; ++b)
        if (b < P.tb) off |= ((m >> b) & 1ull) << pbyte(P.T, b);
    return off;
}

// exp(-i g c) for unit weights from an LDS table; per-amplitude sincos otherwise.
template <typename CT> struct Phase;
template <> struct Phase<int> {
    __device__ static d2v get(const d2v *tab, double, int c) { return tab[c]; }
};
template <> struct Phase<double> {
    __device__ static d2v get(const d2v *, double g, double c) {
        double s, co;
        sincos(g * c, &s, &co);
        d2v r;
        r.x = co;
        r.y = -s;
        return r;
    }
};

__device__ __forceinline__ d2v cmul2(d2v a, d2v b) {
    d2v r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}

__device__ __forceinline__ void fill_table(d2v *tab, int ne_total, double g) {
    for (int c = threadIdx.x; c <= ne_total; c += blockDim.x) {
        double s, co;
        sincos(g * (double)c, &s, &co);
        d2v v;
        v.x = co;
        v.y = -s;
        tab[c] = v;
    }
}

// RX(theta), (c, s) = (cos theta/2, sin theta/2): (a, v) -> (c a - i s v, -i s a + c v).
__device__ __forceinline__ void rx_pair(d2v &a, d2v &v, double c, double s) {
    d2v na, nb;
    na.x = c * a.x + s * v.y;
    na.y = c * a.y - s * v.x;
    nb.x = s * a.y + c * v.x;
    nb.y = c * v.y - s * a.x;
    a = na;
    v = nb;
}

// One lane's half of RX on a lane bit: own -> c own - i s partner.
__device__ __forceinline__ d2v rx_half(d2v a, d2v v, double c, double s) {
    d2v r;
    r.x = c * a.x + s * v.y;
    r.y = c * a.y - s * v.x;
    return r;
}

__device__ __forceinline__ double im_conj_mul(d2v l, d2v p) { return l.x * p.y - l.y * p.x; }  // Im(conj(l) p)

__device__ __forceinline__ d2v shfl_xor2(d2v v, int m) {
    d2v r;
    r.x = __shfl_xor(v.x, m, 64);
    r.y = __shfl_xor(v.y, m, 64);
    return r;
}

// The value of lane ^ 2^lb.  Bits 0 and 1 use a DPP quad permute (one VALU
// move per dword); the other bits use ds_bpermute.  A DPP / permlane form of
// bits 2..5 costs two VALU operations per dword, which run at the FP64 issue
// rate here and were measured slower than the LDS-unit permutes, whereas the
// single quad permute takes load off the LDS issue queue that the backward
// passes wait on.
template <int CTRL> __device__ __forceinline__ uint32_t dpp32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}
template <int CTRL> __device__ __forceinline__ d2v dpp2(d2v v) {
    const uint64_t a = (uint64_t)__double_as_longlong(v.x), b = (uint64_t)__double_as_longlong(v.y);
    d2v r;
    r.x = __longlong_as_double((long long)((uint64_t)dpp32<CTRL>((uint32_t)a) | ((uint64_t)dpp32<CTRL>((uint32_t)(a >> 32)) << 32)));
    r.y = __longlong_as_double((long long)((uint64_t)dpp32<CTRL>((uint32_t)b) | ((uint64_t)dpp32<CTRL>((uint32_t)(b >> 32)) << 32)));
    return r;
}
// Partner value for lane bit lb (run-time; one uniform branch per value,
// so only the partner is live across it).
__device__ __forceinline__ d2v lane_partner(d2v v, int lb) {
    if (lb == 0) return dpp2<0xB1>(v);  // quad_perm [1,0,3,2]
    if (lb == 1) return dpp2<0x4E>(v);  // quad_perm [2,3,0,1]
    return shfl_xor2(v, 1 << lb);
}

__device__ __forceinline__ double qblock_sum(double v, double *sh) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    const int nw = blockDim.x >> 6;
    for (int k = 0; k < nw; ++k) t += sh[k];
    return t;
}

// Four block sums at once (same order per value as qblock_sum, two barriers
// instead of eight); sh holds 4 x 16 doubles.
__device__ __forceinline__ void qblock_sum4(double (&v)[4], double *sh) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1)
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] += __shfl_xor(v[i], d, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int i = 0; i < 4; ++i) sh[i * 16 + (threadIdx.x >> 6)] = v[i];
    __syncthreads();
    const int nw = blockDim.x >> 6;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        double t = 0.0;
        for (int k = 0; k < nw; ++k) t += sh[i * 16 + k];
        v[i] = t;
    }
}

// Per-circuit pointers of a batched launch.
struct QCirc {
    const QPass *P;
    u64 cid, tile;
    char *region;
    const double *theta;
};

template <bool POOLED>
__device__ __forceinline__ QCirc qcirc(const QPass &Parg, const QGeom &geo, const QBatch &B) {
    QCirc q;
    const u64 c = blockIdx.x >> geo.glog;
    q.tile = blockIdx.x & ((1ull << geo.glog) - 1);
    if constexpr (POOLED) {
        q.P = B.passes + ((B.c0 + c) / B.sets) * B.np + B.k;
        q.cid = (u64)B.circ_map[B.c0 + c];
    } else {
        q.P = &Parg;
        q.cid = c;
    }
    q.region = B.ws + c * B.circ_bytes;
    q.theta = B.theta + q.cid * 2 * geo.p;
    return q;
}

// ================================================================== LDS kernels (n < 10)

__device__ __forceinline__ void lds_rx(d2v *sh, int TS, int b, double c, double s) {
    for (int k = threadIdx.x; k < TS / 2; k += kLdsThreads) {
        const int m0 = (int)insert0((u64)k, b), m1 = m0 | (1 << b);
        d2v a = sh[m0], v = sh[m1];
        rx_pair(a, v, c, s);
        sh[m0] = a;
        sh[m1] = v;
    }
}

// Tiles of up to 2^10 amplitudes, 256 threads, m = tid + 256 j (edge list 0).
template <typename CT, bool POOLED>
__global__ __launch_bounds__(kLdsThreads) void k_qaoa_fwd_lds(QPass Parg, QWeights W, QGeom geo, QBatch B) {
    constexpr int JB = 2, R = 4;
    __shared__ d2v sh[1 << 10];
    __shared__ d2v tab_a[kQMaxEdges + 1], tab_b[kQMaxEdges + 1];
    __shared__ double red[16];
    const QCirc q = qcirc<POOLED>(Parg, geo, B);
    const QPass &P = *q.P;
    const d2v *in = B.in_off >= 0 ? (const d2v *)(q.region + B.in_off) : nullptr;
    d2v *out = B.out_off >= 0 ? (d2v *)(q.region + B.out_off) : nullptr;
    const int TS = 1 << P.tb, tid = threadIdx.x, l = P.layer, p = geo.p;
    const u64 base = qtile_base(P, q.tile);
    const bool first = P.flags & QF_FIRST, pend = P.flags & QF_PHASE_END, last = P.flags & QF_LAST;
    const double g_a = q.theta[l], g_b = pend ? q.theta[l + 1] : 0.0;
    if (!geo.weighted) {
        if (first) fill_table(tab_a, geo.num_edges, g_a);
        if (pend) fill_table(tab_b, geo.num_edges, g_b);
    }
    CT C[R];
    cut_values<CT, JB>(P, 0, W, geo.weighted, base, tid, C);
    __syncthreads();
    const double amp0 = 1.0 / sqrt((double)(1ull << geo.n));
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int m = tid + kLdsThreads * j;
        if (m < TS) {
            d2v v;
            if (first) {
                const d2v f = Phase<CT>::get(tab_a, g_a, C[j]);
                v.x = amp0 * f.x;
                v.y = amp0 * f.y;
            } else {
                v = in[base | qtile_off(P, (u64)m)];
            }
            sh[m] = v;
        }
    }
    __syncthreads();
    double sb, cb;
    sincos(q.theta[p + l], &sb, &cb);
    for (int b = 0; b < P.tb; ++b) {
        if (!((P.rx_mask >> b) & 1)) continue;
        lds_rx(sh, TS, b, cb, sb);
        __syncthreads();
    }
    double e_acc = 0.0;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int m = tid + kLdsThreads * j;
        if (m < TS) {
            d2v v = sh[m];
            if (pend) v = cmul2(v, Phase<CT>::get(tab_b, g_b, C[j]));
            if (last) e_acc += (double)C[j] * (v.x * v.x + v.y * v.y);
            if (out) out[base | qtile_off(P, (u64)m)] = v;
        }
    }
    if (last) {
        const double t = qblock_sum(e_acc, red);
        if (tid == 0) ((double *)(q.region + B.epart_off))[q.tile] = t;
    }
}

template <typename CT, bool POOLED>
__global__ __launch_bounds__(kLdsThreads) void k_qaoa_bwd_lds(QPass Parg, QWeights W, QGeom geo, QBatch B) {
    constexpr int JB = 2, R = 4;
    __shared__ d2v shl[1 << 10], shp[1 << 10];
    __shared__ d2v tab_a[kQMaxEdges + 1], tab_b[kQMaxEdges + 1];
    __shared__ double red[16];
    const QCirc q = qcirc<POOLED>(Parg, geo, B);
    const QPass &P = *q.P;
    const d2v *ckpt = (const d2v *)(q.region + B.in_off);
    d2v *lam = (d2v *)(q.region + B.lam_off);
    double *partial = (double *)(q.region + B.part_off);
    const int TS = 1 << P.tb, tid = threadIdx.x, l = P.layer, p = geo.p;
    const u64 base = qtile_base(P, q.tile);
    const bool first = P.flags & QF_FIRST, pend = P.flags & QF_PHASE_END, last = P.flags & QF_LAST;
    const double g_a = q.theta[l], g_b = pend ? q.theta[l + 1] : 0.0;
    if (!geo.weighted) {
        if (first) fill_table(tab_a, geo.num_edges, g_a);
        if (pend) fill_table(tab_b, geo.num_edges, -g_b);
    }
    CT C[R];
    cut_values<CT, JB>(P, 0, W, geo.weighted, base, tid, C);
    __syncthreads();
    double ipc = 0.0, ipb = 0.0, ipc1 = 0.0;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int m = tid + kLdsThreads * j;
        if (m < TS) {
            const u64 idx = base | qtile_off(P, (u64)m);
            d2v ps = ckpt[idx], lm;
            if (last) {
                lm.x = (double)C[j] * ps.x;
                lm.y = (double)C[j] * ps.y;
            } else {
                lm = lam[idx];
            }
            if (pend) {
                ipc += (double)C[j] * im_conj_mul(lm, ps);
                const d2v f = Phase<CT>::get(tab_b, -g_b, C[j]);
                lm = cmul2(lm, f);
                ps = cmul2(ps, f);
            }
            shl[m] = lm;
            shp[m] = ps;
        }
    }
    __syncthreads();
    double sb, cb;
    sincos(q.theta[p + l], &sb, &cb);
    for (int b = 0; b < P.tb; ++b) {
        if (!((P.rx_mask >> b) & 1)) continue;
        for (int k = tid; k < TS / 2; k += kLdsThreads) {
            const int m0 = (int)insert0((u64)k, b), m1 = m0 | (1 << b);
            d2v l0 = shl[m0], l1 = shl[m1], p0 = shp[m0], p1 = shp[m1];
            ipb += im_conj_mul(l0, p1) + im_conj_mul(l1, p0);
            rx_pair(l0, l1, cb, -sb);
            rx_pair(p0, p1, cb, -sb);
            shl[m0] = l0;
            shl[m1] = l1;
            shp[m0] = p0;
            shp[m1] = p1;
        }
        __syncthreads();
    }
    const double amp0 = 1.0 / sqrt((double)(1ull << geo.n));
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int m = tid + kLdsThreads * j;
        if (m < TS) {
            const d2v lm = shl[m];
            if (first) {
                const d2v f = Phase<CT>::get(tab_a, g_a, C[j]);
                ipc1 += (double)C[j] * amp0 * (lm.x * f.y - lm.y * f.x);
            } else {
                lam[base | qtile_off(P, (u64)m)] = lm;
            }
        }
    }
    const double tc = qblock_sum(ipc, red);
    const double tbx = qblock_sum(ipb, red);
    const double tc1 = qblock_sum(ipc1, red);
    if (tid == 0) {
        double *o = partial + ((u64)P.pidx * geo.G + q.tile) * kQSlots;
        o[0] = tc;
        o[1] = tbx;
        o[2] = tc1;
        o[3] = 0.0;
    }
}

// ================================================================== register-tiled kernels (n >= 10)

// Thread maps of a (TB, TT) tile.  Thread t = lane bits 0..5 and wave bits
// 6..TT-1; each thread holds registers j = 0..R-1 (JB bits).  Three layouts:
//   L0  thread bit b -> tile bit b, register bit x -> tile bit TT + x
//       (a wavefront's loads and stores cover 1 KiB contiguous);
//   L1  the wave bits trade places with register bits 0..W-1;
//   L2  lane bits LS..5 trade places with register bits 0..S-1 (S = min(3, JB)).
// RX on a tile bit is a register-pair update in a layout that holds the bit
// in a register, or an update across lanes (wavefront exchanges).  The
// forward kernel walks all three layouts: when a pass uses L2, only lane bits
// below LS need exchanges, as an LDS transpose of the register array costs
// less than exchanging every register for three lane bits.  The backward
// kernel, which carries two vectors, uses L0 and L1 only: there the third
// layout's extra transposes and the psi updates it needs before them cost
// more (measured) than the exchanges they save.
template <int TB, int TT> struct RT {
    static constexpr int NT = 1 << TT, W = TT - 6, JB = TB - TT, R = 1 << JB, TS = 1 << TB;
    static constexpr int S = JB < 3 ? JB : 3, LS = 6 - S;
    static_assert(JB >= W, "the second layout needs a register bit per wave bit");
    // The layout is a uniform run-time value; the maps below select between
    // the three forms without branching, so one copy of the code (and one
    // set of registers) serves every layout.
    // tile index of (thread t, register j) in layout L: tpart(L, t) | jpart(L, j)
    __device__ static int tpart(int L, int t) {
        constexpr int lmask = ((1 << S) - 1) << LS;
        const int t1 = (t & 63) | ((t >> 6) << TT);
        const int t2 = (t & ~lmask) | (((t >> LS) & ((1 << S) - 1)) << TT);
        return L == 0 ? t : L == 1 ? t1 : t2;
    }
    __device__ static int jpart(int L, int j) {
        const int j1 = ((j & ((1 << W) - 1)) << 6) | ((j >> W) << (TT + W));
        const int j2 = ((j & ((1 << S) - 1)) << LS) | ((j >> S) << (TT + S));
        return L == 0 ? j << TT : L == 1 ? j1 : j2;
    }
    // tile bit of register bit x / of thread bit b in layout L
    __host__ __device__ static constexpr int reg_bit(int L, int x) {
        return L == 0 ? TT + x : L == 1 ? (x < W ? 6 + x : TT + x) : (x < S ? LS + x : TT + x);
    }
    __host__ __device__ static constexpr int thr_bit(int L, int b) {
        return L == 0 ? b : L == 1 ? (b < 6 ? b : TT + (b - 6)) : (b >= LS && b < 6 ? TT + (b - LS) : b);
    }
    // tile bits layout L holds in registers
    __host__ __device__ static constexpr u32 regs(int L) {
        u32 r = 0;
        for (int x = 0; x < JB; ++x) r |= 1u << reg_bit(L, x);
        return r;
    }
};

// Global offsets (relative to the tile base) of the thread's amplitudes in layout L.
template <int TB, int TT>
__device__ __forceinline__ void rt_offsets(const QPass &P, int t, int L, u64 (&off)[1 << (TB - TT)]) {
    using G = RT<TB, TT>;
    // Branch-free in t, so the map entries are uniform scalar loads.
    u64 ot = 0;
#pragma unroll
    for (int b = 0; b < TT; ++b) ot |= (u64)((t >> b) & 1) << pbyte(P.T, G::thr_bit(L, b));
#pragma unroll
    for (int j = 0; j < G::R; ++j) {
        u64 o = ot;
#pragma unroll
        for (int x = 0; x < G::JB; ++x)
            if ((j >> x) & 1) o |= 1ull << pbyte(P.T, G::reg_bit(L, x));
        off[j] = o;
    }
}

// LDS transpose of one register array from layout `from` to layout `to`
// (ends with a barrier).
template <int TB, int TT>
__device__ __forceinline__ void rt_xpose(d2v (&a)[1 << (TB - TT)], d2v *sh, int from, int to) {
    using G = RT<TB, TT>;
    const int t = threadIdx.x, tf = G::tpart(from, t), tt = G::tpart(to, t);
#pragma unroll
    for (int j = 0; j < G::R; ++j) sh[tf | G::jpart(from, j)] = a[j];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < G::R; ++j) a[j] = sh[tt | G::jpart(to, j)];
    __syncthreads();
}

// RX(2 beta), (cb, sb) = (cos beta, sin beta), on the register bits of layout
// L whose tile bits are in `todo` (a uniform skip for the others: a walk
// revisits bits that an earlier layout has done).
template <int TB, int TT>
__device__ __forceinline__ void rt_rx_regs(d2v (&a)[1 << (TB - TT)], u32 todo, double cb, double sb, int L) {
    using G = RT<TB, TT>;
#pragma unroll
    for (int x = 0; x < G::JB; ++x) {
        if (!((todo >> G::reg_bit(L, x)) & 1)) continue;
#pragma unroll
        for (int j = 0; j < G::R; ++j)
            if (!((j >> x) & 1)) rx_pair(a[j], a[j | (1 << x)], cb, sb);
    }
}

// Lane bits (a mask below 64; every layout keeps lane bits 0..LS-1 on tile
// bits 0..LS-1, and L0 / L1 keep all six) through wavefront exchanges, one
// bit at a time.
template <int R>
__device__ __forceinline__ void rt_rx_lanes(d2v (&a)[R], u32 lanes, double cb, double sb) {
#pragma unroll 1
    for (u32 m = lanes; m; m &= m - 1) {
        const int lb = __builtin_ctz(m);
#pragma unroll
        for (int j = 0; j < R; ++j) a[j] = rx_half(a[j], lane_partner(a[j], lb), cb, sb);
    }
}

// Next layout of a mixer walk: one that holds some of the remaining bits in
// registers, L0 last (stores from L0 cover 1 KiB per wavefront).
template <int TB, int TT>
__device__ __forceinline__ int rt_next(u32 todo, int cur) {
    using G = RT<TB, TT>;
    if (cur != 2 && (todo & G::regs(2))) return 2;
    if (cur != 1 && (todo & G::regs(1))) return 1;
    return 0;
}

template <int TB, int TT>
__device__ __forceinline__ u32 rt_regs(int L) {
    using G = RT<TB, TT>;
    return L == 0 ? G::regs(0) : L == 1 ? G::regs(1) : G::regs(2);
}

// One mixer: RX(cb, sb) on every tile bit of `todo`, starting in layout
// `cur`: the exchange lane bits `xl`, the current layout's register bits,
// then the layouts that hold the remaining bits (every tile bit is a lane
// bit below LS, in `xl`, or a register bit of some layout, so at most three
// layouts are visited).  Returns the final layout.
template <int TB, int TT>
__device__ __forceinline__ int rt_mixer(d2v (&a)[1 << (TB - TT)], d2v *sh, u32 todo, u32 xl, double cb, double sb, int cur) {
    rt_rx_lanes(a, todo & xl, cb, sb);
    todo &= ~xl;
#pragma unroll 1
    for (int step = 0; step < 3; ++step) {
        const u32 here = todo & rt_regs<TB, TT>(cur);
        rt_rx_regs<TB, TT>(a, here, cb, sb, cur);
        todo &= ~here;
        if (!todo) break;
        const int next = rt_next<TB, TT>(todo, cur);
        rt_xpose<TB, TT>(a, sh, cur, next);
        cur = next;
    }
    return cur;
}

// Lane bits a pass updates through exchanges: all six, or those below LS
// when the pass uses the third layout.
template <int TB, int TT>
__device__ __forceinline__ u32 rt_exchange_lanes(const QPass &P) {
    return P.use_l2 ? (1u << RT<TB, TT>::LS) - 1u : 63u;
}

// TABS: the pass applies a cost phase from a table (unit weights: the first
// pass, a pass ending in a phase, a merged pass).  Passes without one leave
// the tables out, which lowers the block's LDS and lets more blocks share a CU.
template <typename CT, int TB, int TT, bool POOLED, bool MERGE, bool TABS>
__global__ __launch_bounds__(1 << TT) void k_qaoa_fwd_rt(QPass Parg, QWeights W, QGeom geo, QBatch B) {
    using G = RT<TB, TT>;
    constexpr int R = G::R, JB = G::JB;
    __shared__ d2v sh[G::TS];
    __shared__ d2v tab_a[TABS ? kQMaxEdges + 1 : 1], tab_b[TABS ? kQMaxEdges + 1 : 1];
    __shared__ double red[16];
    const QCirc q = qcirc<POOLED>(Parg, geo, B);
    const QPass &P = *q.P;
    const d2v *in = B.in_off >= 0 ? (const d2v *)(q.region + B.in_off) : nullptr;
    d2v *out = B.out_off >= 0 ? (d2v *)(q.region + B.out_off) : nullptr;
    const int t = threadIdx.x, l = P.layer, p = geo.p;
    const u64 base = qtile_base(P, q.tile);
    // Merged passes are never first or last and carry no end phase.
    constexpr bool merge = MERGE;
    const bool first = !MERGE && (P.flags & QF_FIRST), pend = !MERGE && (P.flags & QF_PHASE_END), last = !MERGE && (P.flags & QF_LAST);
    const double g_a = q.theta[l], g_b = pend || merge ? q.theta[l + 1] : 0.0;
    if constexpr (TABS) {
        if (!geo.weighted) {
            if (first) fill_table(tab_a, geo.num_edges, g_a);
            if (pend || merge) fill_table(tab_b, geo.num_edges, g_b);
        }
    }
    const double amp0 = 1.0 / sqrt((double)(1ull << geo.n));
    d2v a[R];
    if (!first) {
        u64 off[R];
        rt_offsets<TB, TT>(P, t, 0, off);
#pragma unroll
        for (int j = 0; j < R; ++j) a[j] = ld<true>(in + (base | off[j]));
    }
    // Cut values of the phase after the first mixer, in the layout that
    // mixer ends in (the plan's lay_mid), computed while the loads are in
    // flight.
    CT C0[R], C1[R];
    if (first) cut_values<CT, JB>(P, 0, W, geo.weighted, base, t, C0);
    if (pend || last || merge) cut_values<CT, JB>(P, P.lay_mid, W, geo.weighted, base, t, C1);
    __syncthreads();
    if (first) {
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const d2v f = Phase<CT>::get(tab_a, g_a, C0[j]);
            a[j].x = amp0 * f.x;
            a[j].y = amp0 * f.y;
        }
    }
    double sb, cb;
    sincos(q.theta[p + l], &sb, &cb);  // RX(2 beta): cos(beta), sin(beta)
    const u32 rx = P.rx_mask, xl = rt_exchange_lanes<TB, TT>(P);
    int cur = rt_mixer<TB, TT>(a, sh, rx, xl, cb, sb, 0);
    if constexpr (MERGE) {
        // exp(-i gamma_{l+1} C), then layer l+1's RX gates on the same bits,
        // starting in the layout the first set ended in.
#pragma unroll
        for (int j = 0; j < R; ++j) a[j] = cmul2(a[j], Phase<CT>::get(tab_b, g_b, C1[j]));
        double sb2, cb2;
        sincos(q.theta[p + l + 1], &sb2, &cb2);
        cur = rt_mixer<TB, TT>(a, sh, rx, xl, cb2, sb2, cur);
    }
    int ts = t;
    asm volatile("" : "+v"(ts));  // offsets formed here, not kept live through the pass
    u64 off[R];
    rt_offsets<TB, TT>(P, ts, cur, off);
    double e_acc = 0.0;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        d2v v = a[j];
        if (pend) v = cmul2(v, Phase<CT>::get(tab_b, g_b, C1[j]));
        if (last) e_acc += (double)C1[j] * (v.x * v.x + v.y * v.y);
        if (out) st<true>(out + (base | off[j]), v);
    }
    if (last) {
        const double s = qblock_sum(e_acc, red);
        if (t == 0) ((double *)(q.region + B.epart_off))[q.tile] = s;
    }
}

// ------------------------------------------------------------ backward helpers (L0 and L1)

// psi from layout FROM to layout TO through LDS, taking on the way the inner
// products of the lane bits in `lanes` with lambda (already in TO, at the same
// point): while psi sits in LDS a lane's partner value is one 16-byte read per
// register instead of four wavefront exchanges (L0 and L1 hold the lane bits
// alike, so the partner of lambda's register j is psi's TO slot of the
// partner thread).
template <int TB, int TT, int FROM, int TO>
__device__ __forceinline__ void rt_xpose_ip_lanes(d2v (&ps)[1 << (TB - TT)], const d2v (&lm)[1 << (TB - TT)], d2v *sh, u32 lanes, double &acc) {
    using G = RT<TB, TT>;
    const int t = threadIdx.x;
#pragma unroll
    for (int j = 0; j < G::R; ++j) sh[G::tpart(FROM, t) | G::jpart(FROM, j)] = ps[j];
    __syncthreads();
#pragma unroll 1
    for (u32 m = lanes; m; m &= m - 1) {
        const int tp = G::tpart(TO, t ^ (1 << __builtin_ctz(m)));
        double a = 0.0;
#pragma unroll
        for (int j = 0; j < G::R; ++j) a += im_conj_mul(lm[j], sh[tp | G::jpart(TO, j)]);
        acc += a;
    }
#pragma unroll
    for (int j = 0; j < G::R; ++j) ps[j] = sh[G::tpart(TO, t) | G::jpart(TO, j)];
    __syncthreads();
}

// Which register bits a helper covers: none, register bits 0..W-1 (the bits
// the other layout holds as wave bits), all, or register bits 0..S-1 (in the
// third layout, the upper lane bits of the first).
enum { kRegsNone = 0, kRegsLow = 1, kRegsAll = 2, kRegsLowS = 3 };

// RX(2 beta), (cb, sb) = (cos beta, sin beta), on the tile bits of `rx` that
// layout L holds in the selected register bits and, when `lanes`, on the lane
// bits.
// Register-bit gates are applied without a branch, as the identity
// (cos, sin) = (1, 0) where the bit takes no RX: a uniform branch around an
// in-place update of the register array makes the compiler copy the whole
// array, and register bits almost always take the gate.
template <int TB, int TT, int L>
__device__ __forceinline__ void rt_rx_sel(d2v (&a)[1 << (TB - TT)], u32 rx, double cb, double sb, int regs, bool lanes) {
    using G = RT<TB, TT>;
#pragma unroll
    for (int x = 0; x < G::JB; ++x) {
        if (regs == kRegsNone || (regs == kRegsLow && x >= G::W) || (regs == kRegsLowS && x >= G::S)) continue;
        const bool on = (rx >> G::reg_bit(L, x)) & 1;
        const double c = on ? cb : 1.0, s = on ? sb : 0.0;
#pragma unroll
        for (int j = 0; j < G::R; ++j)
            if (!((j >> x) & 1)) rx_pair(a[j], a[j | (1 << x)], c, s);
    }
    if (lanes) {
        // The lane bits that take RX form a top range [lo, 5] (a pass's tile
        // holds its new qubits on the highest positions); a run-time loop over
        // that range does no shuffles for the others, and identity
        // coefficients keep any other mask correct.
        const u32 lm = rx & 63u;
        const int lo = lm ? __builtin_ctz(lm) : 6;
#pragma unroll 1
        for (int lb = lo; lb < 6; ++lb) {
            const bool on = (lm >> lb) & 1;
            const double c = on ? cb : 1.0, s = on ? sb : 0.0;
#pragma unroll
            for (int j = 0; j < G::R; ++j) a[j] = rx_half(a[j], lane_partner(a[j], lb), c, s);
        }
    }
}

// The same over every register bit of the layout the registers are in
// (`in_l1` chosen at run time), so one copy of the code serves both layouts.
template <int TB, int TT>
__device__ __forceinline__ void rt_rx_cur(d2v (&a)[1 << (TB - TT)], u32 rx, double cb, double sb, bool in_l1, bool lanes) {
    using G = RT<TB, TT>;
#pragma unroll
    for (int x = 0; x < G::JB; ++x) {
        const int tbit = in_l1 ? G::reg_bit(1, x) : G::reg_bit(0, x);
        const bool on = (rx >> tbit) & 1;
        const double c = on ? cb : 1.0, s = on ? sb : 0.0;
#pragma unroll
        for (int j = 0; j < G::R; ++j)
            if (!((j >> x) & 1)) rx_pair(a[j], a[j | (1 << x)], c, s);
    }
    if (lanes) rt_rx_sel<TB, TT, 0>(a, rx, cb, sb, kRegsNone, true);
}

// Inner products 2 Im<lam|X_j|psi> (without the factor 2) summed over the
// tile bits j of `rx` that layout L reaches, with the same selection as rt_rx_sel.
// A lane pair contributes both of its terms, one in each lane.
template <int TB, int TT, int L>
__device__ __forceinline__ void rt_ip_sel(const d2v (&lm)[1 << (TB - TT)], const d2v (&ps)[1 << (TB - TT)], u32 rx, int regs, bool lanes, double &acc) {
    using G = RT<TB, TT>;
#pragma unroll
    for (int x = 0; x < G::JB; ++x) {
        if (regs == kRegsNone || (regs == kRegsLow && x >= G::W) || (regs == kRegsLowS && x >= G::S)) continue;
        if ((rx >> G::reg_bit(L, x)) & 1) {
#pragma unroll
            for (int j = 0; j < G::R; ++j) {
                if ((j >> x) & 1) continue;
                const int k = j | (1 << x);
                acc += im_conj_mul(lm[j], ps[k]) + im_conj_mul(lm[k], ps[j]);
            }
        }
    }
    if (lanes) {
        const u32 lmask = rx & 63u;
        const int lo = lmask ? __builtin_ctz(lmask) : 6;
#pragma unroll 1
        for (int lb = lo; lb < 6; ++lb) {
            double t = 0.0;
#pragma unroll
            for (int j = 0; j < G::R; ++j) t += im_conj_mul(lm[j], lane_partner(ps[j], lb));
            if ((lmask >> lb) & 1) acc += t;
        }
    }
}

// The same for the inner products.
template <int TB, int TT>
__device__ __forceinline__ void rt_ip_cur(const d2v (&lm)[1 << (TB - TT)], const d2v (&ps)[1 << (TB - TT)], u32 rx, bool in_l1, bool lanes,
                                          double &acc) {
    using G = RT<TB, TT>;
#pragma unroll
    for (int x = 0; x < G::JB; ++x) {
        const int tbit = in_l1 ? G::reg_bit(1, x) : G::reg_bit(0, x);
        if (!((rx >> tbit) & 1)) continue;
#pragma unroll
        for (int j = 0; j < G::R; ++j) {
            if ((j >> x) & 1) continue;
            const int k = j | (1 << x);
            acc += im_conj_mul(lm[j], ps[k]) + im_conj_mul(lm[k], ps[j]);
        }
    }
    if (lanes) rt_ip_sel<TB, TT, 0>(lm, ps, rx, kRegsNone, true, acc);
}

// Inner products and RX(2 beta) on both vectors, bit by bit: for each bit
// the inner product is taken with lambda and psi at the same point, then the
// bit's gate is applied to both (bits of one mixer commute, so every inner
// product is the one at the mixer's end).  A lane bit exchanges each vector
// once and uses the partner values for the inner product and both updates.
template <int TB, int TT, int L>
__device__ __forceinline__ void rt_ip_rx2_sel(d2v (&lm)[1 << (TB - TT)], d2v (&ps)[1 << (TB - TT)], u32 rx, double cb, double sb, int regs, bool lanes,
                                          double &acc) {
    using G = RT<TB, TT>;
#pragma unroll
    for (int x = 0; x < G::JB; ++x) {
        if (regs == kRegsNone || (regs == kRegsLow && x >= G::W) || (regs == kRegsLowS && x >= G::S)) continue;
        const bool on = (rx >> G::reg_bit(L, x)) & 1;
        if (on) {
#pragma unroll
            for (int j = 0; j < G::R; ++j) {
                if ((j >> x) & 1) continue;
                const int k = j | (1 << x);
                acc += im_conj_mul(lm[j], ps[k]) + im_conj_mul(lm[k], ps[j]);
            }
        }
        const double c = on ? cb : 1.0, s = on ? sb : 0.0;
#pragma unroll
        for (int j = 0; j < G::R; ++j)
            if (!((j >> x) & 1)) {
                rx_pair(lm[j], lm[j | (1 << x)], c, s);
                rx_pair(ps[j], ps[j | (1 << x)], c, s);
            }
    }
    if (lanes) {
        const u32 lmask = rx & 63u;
        const int lo = lmask ? __builtin_ctz(lmask) : 6;
#pragma unroll 1
        for (int lb = lo; lb < 6; ++lb) {
            const bool on = (lmask >> lb) & 1;
            const double c = on ? cb : 1.0, s = on ? sb : 0.0;
            double t = 0.0;
#pragma unroll
            for (int j = 0; j < G::R; ++j) {
                const d2v pp = lane_partner(ps[j], lb), pl = lane_partner(lm[j], lb);
                t += im_conj_mul(lm[j], pp);
                lm[j] = rx_half(lm[j], pl, c, s);
                ps[j] = rx_half(ps[j], pp, c, s);
            }
            if (on) acc += t;
        }
    }
}

// WALK, for passes whose RX bits include upper lane bits (LS..5): lambda ends
// the pass in L2, where those bits are register bits, instead of exchanging
// them across the wavefront (one transpose of lambda in place of an exchange
// per upper lane bit; it is stored from L2).  Merged passes take it when
// every RX lane bit is an upper one and some RX bit is an L0 wave bit; they
// then also undo layer l+1's mixer on both vectors through L0, L2 and L1, two
// transposes per vector in place of an exchange of both per upper lane bit.
template <typename CT, int TB, int TT, bool POOLED, bool MERGE, bool TABS, bool WALK = false>
__global__ __launch_bounds__(1 << TT) void k_qaoa_bwd_rt(QPass Parg, QWeights W, QGeom geo, QBatch B) {
    using G = RT<TB, TT>;
    constexpr int R = G::R, JB = G::JB;
    __shared__ d2v sh[G::TS];
    __shared__ d2v tab_a[TABS ? kQMaxEdges + 1 : 1], tab_b[TABS ? kQMaxEdges + 1 : 1];
    __shared__ double red[64];  // qblock_sum4: 4 values x up to 16 waves
    const QCirc q = qcirc<POOLED>(Parg, geo, B);
    const QPass &P = *q.P;
    const d2v *ckpt = (const d2v *)(q.region + B.in_off);
    d2v *lam = (d2v *)(q.region + B.lam_off);
    double *partial = (double *)(q.region + B.part_off);
    const int t = threadIdx.x, l = P.layer, p = geo.p;
    const u64 base = qtile_base(P, q.tile);
    constexpr bool merge = MERGE;
    const bool first = !MERGE && (P.flags & QF_FIRST), pend = !MERGE && (P.flags & QF_PHASE_END), last = !MERGE && (P.flags & QF_LAST);
    const bool l1 = (MERGE && WALK) || ((P.rx_mask >> 6) & ((1u << G::W) - 1)) != 0;  // some RX bit is a wave bit in L0
    const double g_a = q.theta[l], g_b = pend || merge ? q.theta[l + 1] : 0.0;
    if constexpr (TABS) {
        if (!geo.weighted) {
            if (first) fill_table(tab_a, geo.num_edges, g_a);
            if (pend || merge) fill_table(tab_b, geo.num_edges, -g_b);  // exp(+i gamma C): undo the phase
        }
    }
    // Register bits of the two layouts: A bits (tile 6..6+W-1) only in L1,
    // B bits (tile TT..TT+W-1) only in L0, the rest of the register bits and
    // the lane bits in both.  Inner products of one mixer may be taken at any
    // point inside it as long as lambda and psi are at the same point (the RX
    // gates of a mixer commute with every X_j); psi is transformed only as far
    // as later inner products need it.
    d2v lm[R], ps[R];
    double ipc = 0.0, ipb = 0.0, ipc1 = 0.0, ipb2 = 0.0;
    {
        // The checkpoint's loads first: the cut values are computed while
        // they are in flight (lambda's loads as well would hold twice the
        // registers through that computation).
        u64 off[R];
        rt_offsets<TB, TT>(P, t, 0, off);
#pragma unroll
        for (int j = 0; j < R; ++j) ps[j] = ld<true>(ckpt + (base | off[j]));
        CT Cs[R];
        if (last || pend) cut_values<CT, JB>(P, 0, W, geo.weighted, base, t, Cs);
        __syncthreads();  // phase tables
#pragma unroll
        for (int j = 0; j < R; ++j) {
            if (last) {
                lm[j].x = (double)Cs[j] * ps[j].x;
                lm[j].y = (double)Cs[j] * ps[j].y;
            } else {
                lm[j] = ld<true>(lam + (base | off[j]));
            }
            if (pend) {
                // Im(conj(lam) psi) weighted by C, then undo exp(-i gamma C) on both.
                ipc += (double)Cs[j] * im_conj_mul(lm[j], ps[j]);
                const d2v f = Phase<CT>::get(tab_b, -g_b, Cs[j]);
                lm[j] = cmul2(lm[j], f);
                ps[j] = cmul2(ps[j], f);
            }
        }
    }
    double sb, cb;
    sincos(q.theta[p + l], &sb, &cb);
    const double sn = -sb;  // RX(-2 beta)
    const u32 rx = P.rx_mask;
    int lay = 0;  // the layout the registers end in
    if constexpr (MERGE) {
        // Layer l+1's RX gates: inner products at the end point, then undone
        // on both vectors (psi is needed again below), L0 first, then L1.
        double sb2, cb2;
        sincos(q.theta[p + l + 1], &sb2, &cb2);
        const double sn2 = -sb2;
        if constexpr (WALK) {
            rt_ip_rx2_sel<TB, TT, 0>(lm, ps, rx, cb2, sn2, kRegsAll, false, ipb2);
            rt_xpose<TB, TT>(lm, sh, 0, 2);
            rt_xpose<TB, TT>(ps, sh, 0, 2);
            rt_ip_rx2_sel<TB, TT, 2>(lm, ps, rx, cb2, sn2, kRegsLowS, false, ipb2);
            rt_xpose<TB, TT>(lm, sh, 2, 1);
            rt_xpose<TB, TT>(ps, sh, 2, 1);
            rt_ip_rx2_sel<TB, TT, 1>(lm, ps, rx, cb2, sn2, kRegsLow, false, ipb2);
            lay = 1;
        } else {
            rt_ip_rx2_sel<TB, TT, 0>(lm, ps, rx, cb2, sn2, kRegsAll, true, ipb2);
            if (l1) {
                rt_xpose<TB, TT>(lm, sh, 0, 1);
                rt_xpose<TB, TT>(ps, sh, 0, 1);
                rt_ip_rx2_sel<TB, TT, 1>(lm, ps, rx, cb2, sn2, kRegsLow, false, ipb2);
                lay = 1;
            }
        }
        // The cost phase between the two mixers, in the current layout.  Its
        // inner product Im(conj(lam) C psi) is unchanged by the common unit
        // factor, so it is taken after the undo, on the new values.
        {
            CT Cm[R];
            cut_values<CT, JB>(P, l1 ? 1 : 0, W, geo.weighted, base, t, Cm);
#pragma unroll
            for (int j = 0; j < R; ++j) {
                const d2v f = Phase<CT>::get(tab_b, -g_b, Cm[j]);
                lm[j] = cmul2(lm[j], f);
                ps[j] = cmul2(ps[j], f);
                ipc += (double)Cm[j] * im_conj_mul(lm[j], ps[j]);
            }
        }
        // Layer l's RX gates, back to L0: inner products of the bits the
        // current layout reaches; with L1, the A bits undone on both, the
        // transpose and the B-bit inner products; then lambda alone undoes
        // the rest and is stored from L0.
        rt_ip_cur<TB, TT>(lm, ps, rx, l1, !l1, ipb);
        if (l1) {
            rt_rx_sel<TB, TT, 1>(lm, rx, cb, sn, kRegsLow, false);
            rt_rx_sel<TB, TT, 1>(ps, rx, cb, sn, kRegsLow, false);
            rt_xpose<TB, TT>(lm, sh, 1, 0);
            rt_xpose_ip_lanes<TB, TT, 1, 0>(ps, lm, sh, rx & 63u, ipb);
            rt_ip_sel<TB, TT, 0>(lm, ps, rx, kRegsLow, false, ipb);
        }
        if constexpr (WALK) {
            rt_rx_sel<TB, TT, 0>(lm, rx, cb, sn, kRegsAll, false);
            rt_xpose<TB, TT>(lm, sh, 0, 2);
            rt_rx_sel<TB, TT, 2>(lm, rx, cb, sn, kRegsLowS, false);
            lay = 2;
        } else {
            rt_rx_sel<TB, TT, 0>(lm, rx, cb, sn, kRegsAll, true);
            lay = 0;
        }
    } else {
        // One mixer: inner products of the L0 register bits; if some RX bit
        // needs L1, undo the B bits on both, take the lane-bit inner products
        // while psi passes through LDS, transpose, take the A-bit inner
        // products (without L1, the lane bits by exchanges); psi is then dead
        // and lambda undoes every bit not yet undone.
        rt_ip_sel<TB, TT, 0>(lm, ps, rx, kRegsAll, !l1, ipb);
        if (l1) {
            rt_rx_sel<TB, TT, 0>(lm, rx, cb, sn, kRegsLow, false);
            rt_rx_sel<TB, TT, 0>(ps, rx, cb, sn, kRegsLow, false);
            rt_xpose<TB, TT>(lm, sh, 0, 1);
            rt_xpose_ip_lanes<TB, TT, 0, 1>(ps, lm, sh, rx & 63u, ipb);
            rt_ip_sel<TB, TT, 1>(lm, ps, rx, kRegsLow, false, ipb);
            lay = 1;
        }
        if constexpr (WALK) {
            rt_rx_cur<TB, TT>(lm, rx, cb, sn, l1, false);
            rt_xpose<TB, TT>(lm, sh, lay, 2);
            rt_rx_sel<TB, TT, 2>(lm, rx, cb, sn, kRegsLowS, false);
            rt_rx_lanes(lm, rx & ((1u << G::LS) - 1u), cb, sn);
            lay = 2;
        } else {
            rt_rx_cur<TB, TT>(lm, rx, cb, sn, l1, true);
        }
    }
    const double amp0 = 1.0 / sqrt((double)(1ull << geo.n));
    if (first) {
        CT Cf[R];
        cut_values<CT, JB>(P, lay, W, geo.weighted, base, t, Cf);
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const d2v f = Phase<CT>::get(tab_a, g_a, Cf[j]);  // phi_1 = 2^{-n/2} exp(-i gamma_1 C)
            ipc1 += (double)Cf[j] * amp0 * (lm[j].x * f.y - lm[j].y * f.x);
        }
    } else {
        // Recompute the store offsets rather than keep the load addresses
        // live through the pass (an empty asm hides that t is unchanged).
        int ts = t;
        asm volatile("" : "+v"(ts));
        u64 off[R];
        rt_offsets<TB, TT>(P, ts, lay, off);
#pragma unroll
        for (int j = 0; j < R; ++j) st<true>(lam + (base | off[j]), lm[j]);
    }
    double sums[4] = {ipc, ipb, ipc1, ipb2};
    qblock_sum4(sums, red);
    if (t == 0) {
        double *o = partial + ((u64)P.pidx * geo.G + q.tile) * kQSlots;
        o[0] = sums[0];
        o[1] = sums[1];
        o[2] = sums[2];
        o[3] = sums[3];
    }
}

// ================================================================== reduction of the partials

// E and gradient of circuit blockIdx.y: one block per output, partials summed
// in a fixed order.  Output k < 2p: gradient component; k = 2p: E.  Without a
// gradient the grid has one block per circuit, which computes E.
template <bool POOLED>
__global__ __launch_bounds__(256) void k_qaoa_final(QGeom geo, QBatch B, QMap map, double *__restrict__ E_out, double *__restrict__ grad_out,
                                                     int with_grad) {
    __shared__ double red[16];
    const int p = geo.p, G = geo.G;
    const int k = with_grad ? (int)blockIdx.x : 2 * p;
    const u64 c = blockIdx.y;
    const u64 cid = POOLED ? (u64)B.circ_map[B.c0 + c] : c;
    const char *region = B.ws + c * B.circ_bytes;
    const double *partial = (const double *)(region + B.part_off);
    const double *e_partial = (const double *)(region + B.epart_off);
    double a = 0.0;
    if (k == 2 * p) {
        for (int b = threadIdx.x; b < G; b += blockDim.x) a += e_partial[b];
    } else {
        for (int i = map.start[k]; i < map.start[k + 1]; ++i) {
            const int pidx = map.item[i] >> 2, slot = map.item[i] & 3;
            double v = 0.0;
            for (int b = threadIdx.x; b < G; b += blockDim.x) v += partial[((u64)pidx * G + b) * kQSlots + slot];
            a += v;
        }
    }
    const double t = qblock_sum(a, red);
    if (threadIdx.x == 0) {
        if (k == 2 * p)
            E_out[cid] = t;
        else
            grad_out[cid * 2 * p + k] = 2.0 * t;
    }
}

// ================================================================== host planning

int qaoa_passes_per_layer(int n, QShape s) {
    const int tb = n < s.TB ? n : s.TB;
    if (n <= tb) return 1;
    const int per = tb - s.r;
    return 1 + (n - tb + per - 1) / per;
}

static int threads_bits_for(int TB) { return TB >= 12 ? 9 : 8; }

QShape qaoa_default_shape(int n) {
    static const int env_tb = [] {
        const char *e = getenv("QSIM_QAOA_TB");
        return e ? atoi(e) : 0;
    }();
    static const int env_r = [] {
        const char *e = getenv("QSIM_QAOA_R");
        return e ? atoi(e) : 0;
    }();
    if (n < 10) return QShape{n, 8, n < 3 ? n : 3};
    if (env_tb >= 10 && env_tb <= 13) {
        const int tb = env_tb < n ? env_tb : n;
        return QShape{tb, threads_bits_for(tb), env_r >= 2 && env_r <= 4 ? env_r : 3};
    }
    // Measured on MI355X (adjoint gradient, p = 8, one angle set): small
    // registers are latency-bound and favour the 16 KiB tiles (more blocks);
    // from 20 qubits on, the shape with the fewest passes per layer and the
    // most blocks at that pass count wins.  13-qubit tiles would save a pass
    // for some n, but their backward kernel exceeds the register file.
    if (n <= 16) return QShape{10, 8, 3};
    if (n <= 18) return QShape{10, 8, 2};
    if (n <= 20) return QShape{12, 9, 3};
    if (n <= 22) return QShape{12, 9, 2};
    if (n <= 26) return QShape{11, 8, 3};
    return QShape{12, 9, 3};
}

std::vector<QShape> qaoa_candidate_shapes(int n) {
    std::vector<QShape> v;
    if (n < 10) return {qaoa_default_shape(n)};
    for (QShape s : {QShape{10, 8, 3}, QShape{10, 8, 2}, QShape{11, 8, 3}, QShape{12, 9, 3}, QShape{12, 9, 2}})
        if (s.TB <= n) v.push_back(s);
    return v;
}

// Tile bit b -> (is thread bit, index) in layout L of a (TB, TT) tile (the
// thread maps of RT in the kernels).
static void layout_kind(int L, int TB, int TT, int b, bool &thread, int &idx) {
    const int W = TT - 6, S = TB - TT < 3 ? TB - TT : 3, LS = 6 - S;
    if (L == 0) {
        thread = b < TT;
        idx = thread ? b : b - TT;
        return;
    }
    if (L == 1) {
        if (b < 6) { thread = true; idx = b; }
        else if (b < 6 + W) { thread = false; idx = b - 6; }
        else if (b < TT + W) { thread = true; idx = 6 + (b - TT); }
        else { thread = false; idx = b - TT; }
        return;
    }
    if (b < LS) { thread = true; idx = b; }
    else if (b < 6) { thread = false; idx = b - LS; }
    else if (b < TT) { thread = true; idx = b; }
    else if (b < TT + S) { thread = true; idx = LS + (b - TT); }
    else { thread = false; idx = b - TT; }
}

// The layout a mixer walk of the register-tiled forward kernel ends in,
// from layout `cur` (the same register maps and choice of the next layout as
// RT, rt_next and rt_mixer on the device).
static int rt_walk_end(int TB, int TT, uint32_t todo, uint32_t xl, int cur) {
    const int W = TT - 6, JB = TB - TT, S = JB < 3 ? JB : 3, LS = 6 - S;
    auto reg_bit = [&](int L, int x) { return L == 0 ? TT + x : L == 1 ? (x < W ? 6 + x : TT + x) : (x < S ? LS + x : TT + x); };
    auto regs = [&](int L) {
        uint32_t r = 0;
        for (int x = 0; x < JB; ++x) r |= 1u << reg_bit(L, x);
        return r;
    };
    todo &= ~xl;
    for (int step = 0; step < 3; ++step) {
        todo &= ~regs(cur);
        if (!todo) break;
        cur = cur != 2 && (todo & regs(2)) ? 2 : cur != 1 && (todo & regs(1)) ? 1 : 0;
    }
    return cur;
}

int build_qplan(int n, int p, int num_edges, const int32_t *edges, const double *w, QShape shape, QPlan &plan) {
    const bool rt = n >= 10;
    if (!rt) shape = QShape{n, 8, n < 3 ? n : 3};
    const int tb = n < shape.TB ? n : shape.TB;
    if (rt) shape.TB = tb, shape.TT = threads_bits_for(tb);
    const int r = shape.r < tb ? shape.r : tb;
    std::vector<std::vector<int>> groups;
    {
        std::vector<int> g0;
        for (int q = 0; q < tb; ++q) g0.push_back(q);
        groups.push_back(g0);
        int q = tb;
        while (q < n) {
            std::vector<int> g;
            for (int k = 0; k < tb - r && q < n; ++k) g.push_back(q++);
            groups.push_back(g);
        }
    }
    const int P = (int)groups.size();
    // Pass order.  With several qubit groups the RX gates of one mixer may be
    // applied in any group order, so odd layers walk the groups in the reverse
    // of even layers and every layer starts on the group the previous layer
    // ended with; the two passes on that group can merge into one (RX of
    // layer l, the cost phase of layer l+1, RX of layer l+1): p(P-1)+1 passes
    // instead of pP.  A merged pass does twice the arithmetic on the same
    // traffic; on the first group, whose lane bits all take RX (lane-bit gates
    // need wavefront shuffles), that costs more than the saved pass at 24
    // qubits, so with three or more groups the first group sits in the middle
    // of every layer and is never a boundary.  Tuning knob QSIM_QAOA_MERGE:
    // 0 never merge, 1 merge every boundary (default), 2 skip boundaries on
    // the first group.
    static const int merge_mode = [] {
        const char *e = getenv("QSIM_QAOA_MERGE");
        return e ? atoi(e) : 1;
    }();
    std::vector<int> order;  // even layers; odd layers use the reverse
    if (P >= 3) {
        order.push_back(1);
        order.push_back(0);
        for (int g = 2; g < P; ++g) order.push_back(g);
    } else {
        for (int g = 0; g < P; ++g) order.push_back(g);
    }
    struct Step {
        int layer, g, flags;
    };
    std::vector<Step> seq;
    for (int l = 0; l < p; ++l) {
        for (int i = 0; i < P; ++i) {
            const int g = P >= 2 && (l & 1) ? order[P - 1 - i] : order[i];
            const bool boundary = l > 0 && i == 0 && P >= 2;  // same group as the previous pass
            if (boundary && (merge_mode == 1 || (merge_mode == 2 && g != 0))) {
                seq.back().flags |= QF_MERGE;
                continue;
            }
            if (l > 0 && i == 0) seq.back().flags |= QF_PHASE_END;  // the previous layer's last pass
            seq.push_back(Step{l, g, l == 0 && i == 0 ? QF_FIRST : 0});
        }
    }
    seq.back().flags |= QF_LAST;
    // Output map: gamma_1 from the first pass (slot 2); gamma_{l+1} from the
    // pass that applies that phase (slot 0); beta_l from every pass holding
    // layer l's RX gates (slot 1, or slot 3 for the second layer of a merged pass).
    {
        std::vector<std::vector<uint16_t>> comp(2 * p);
        for (int k = 0; k < (int)seq.size(); ++k) {
            const int l = seq[k].layer, f = seq[k].flags;
            if (f & QF_FIRST) comp[0].push_back((uint16_t)(k << 2 | 2));
            if (f & (QF_PHASE_END | QF_MERGE)) comp[l + 1].push_back((uint16_t)(k << 2 | 0));
            comp[p + l].push_back((uint16_t)(k << 2 | 1));
            if (f & QF_MERGE) comp[p + l + 1].push_back((uint16_t)(k << 2 | 3));
        }
        int at = 0;
        for (int c = 0; c < 2 * p; ++c) {
            plan.map.start[c] = (uint16_t)at;
            for (uint16_t x : comp[c]) {
                if (at >= kQMaxItems) return fail(QS_ERR_UNSUPPORTED, "QAOA plan exceeds the output map");
                plan.map.item[at++] = x;
            }
        }
        plan.map.start[2 * p] = (uint16_t)at;
    }
    plan.merged.clear();
    for (const Step &st : seq) plan.merged.push_back((st.flags & QF_MERGE) ? 1 : 0);
    plan.shape = shape;
    plan.rt = rt;
    plan.geo = QGeom{n, p, P, tb, 1 << (n - tb), n - tb, num_edges, w != nullptr, (int)seq.size()};
    for (int e = 0; e < num_edges; ++e) plan.W.w[e] = w ? w[e] : 1.0;
    plan.passes.clear();
    const int TT = shape.TT;
    for (int k = 0; k < (int)seq.size(); ++k) {
        {
            const int l = seq[k].layer, g = seq[k].g;
            QPass Q{};
            uint64_t T = 0;
            if (g == 0) {
                for (int q : groups[0]) T |= 1ull << q;
            } else {
                for (int q = 0; q < r; ++q) T |= 1ull << q;
                for (int q : groups[g]) T |= 1ull << q;
                for (int q = 0; q < n && __builtin_popcountll(T) < tb; ++q) T |= 1ull << q;
            }
            int pos[64];
            Q.tb = 0;
            Q.nrest = 0;
            for (int q = 0; q < n; ++q) {
                if ((T >> q) & 1) {
                    pos[q] = Q.tb;
                    Q.T[Q.tb++] = (uint8_t)q;
                } else {
                    pos[q] = -1;
                    Q.rest[Q.nrest++] = (uint8_t)q;
                }
            }
            Q.rx_mask = 0;
            for (int q : groups[g]) Q.rx_mask |= 1u << pos[q];
            {
                // Upper lane bits taking RX: through the third layout unless
                // QSIM_QAOA_L2=0 (then by wavefront exchanges).
                static const bool l2_on = [] {
                    const char *e = getenv("QSIM_QAOA_L2");
                    return !e || atoi(e) != 0;
                }();
                const int S = tb - TT < 3 ? tb - TT : 3;
                Q.use_l2 = rt && l2_on && S > 0 && ((Q.rx_mask >> (6 - S)) & ((1u << S) - 1)) != 0;
                const uint32_t xl = Q.use_l2 ? (1u << (6 - S)) - 1u : 63u;
                Q.lay_mid = rt ? rt_walk_end(tb, TT, Q.rx_mask, xl, 0) : 0;
            }
            Q.layer = l;
            Q.pidx = k;
            Q.flags = seq[k].flags;
            for (int L = 0; L < (rt ? 3 : 1); ++L) {
                std::vector<QEdge> cls[EC_N];
                for (int e = 0; e < num_edges; ++e) {
                    int u = edges[2 * e], v = edges[2 * e + 1];
                    // kind: 0 = thread bit, 1 = register bit, 2 = fixed per tile
                    int ku = 2, kv = 2, iu = u, iv = v;
                    bool th;
                    if (pos[u] >= 0) { layout_kind(L, tb, TT, pos[u], th, iu); ku = th ? 0 : 1; }
                    if (pos[v] >= 0) { layout_kind(L, tb, TT, pos[v], th, iv); kv = th ? 0 : 1; }
                    if (ku > kv) {
                        std::swap(ku, kv);
                        std::swap(iu, iv);
                    }
                    QEdge x{};
                    x.wi = (uint8_t)e;
                    x.a = (uint8_t)iu;
                    x.b = (uint8_t)iv;
                    const int c = ku == 0 ? (kv == 0 ? EC_TT : kv == 2 ? EC_TR : EC_TJ) : ku == 1 ? (kv == 1 ? EC_JJ : EC_JR) : EC_RR;
                    cls[c].push_back(x);
                }
                int k = 0;
                for (int c = 0; c < EC_N; ++c) {
                    Q.cnt[L][c] = (int32_t)cls[c].size();
                    for (auto &x : cls[c]) Q.e[L][k++] = x;
                }
            }
            plan.passes.push_back(Q);
        }
    }
    return QS_OK;
}

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

QLayout qaoa_layout(const QGeom &g, int with_grad) {
    QLayout L{};
    const size_t sb = ((size_t)1 << g.n) * 16;
    const size_t np = (size_t)g.np;
    size_t off = 0;
    if (with_grad) {
        L.ckpt = off;
        off += np * sb;
        L.lam = off;
        off += sb;
        L.part = off;
        off = align256(off + np * (size_t)g.G * kQSlots * sizeof(double));
    } else {
        L.ckpt = off;  // the in-place state
        off += sb;
        L.lam = L.part = -1;
    }
    L.epart = off;
    off = align256(off + (size_t)g.G * sizeof(double));
    L.bytes = off;
    return L;
}

// Kernel pair for one (weights, shape) choice.
template <typename CT, int TB, int TT, bool POOLED> struct RtKernels {
    static constexpr int threads = 1 << TT;
    static void fwd(dim3 grid, hipStream_t st, const QPass &P, const QWeights &W, const QGeom &g, const QBatch &B, bool merged, bool tabs) {
        if (merged)
            hipLaunchKernelGGL((k_qaoa_fwd_rt<CT, TB, TT, POOLED, true, true>), grid, dim3(threads), 0, st, P, W, g, B);
        else if (tabs)
            hipLaunchKernelGGL((k_qaoa_fwd_rt<CT, TB, TT, POOLED, false, true>), grid, dim3(threads), 0, st, P, W, g, B);
        else
            hipLaunchKernelGGL((k_qaoa_fwd_rt<CT, TB, TT, POOLED, false, false>), grid, dim3(threads), 0, st, P, W, g, B);
    }
    static void bwd(dim3 grid, hipStream_t st, const QPass &P, const QWeights &W, const QGeom &g, const QBatch &B, bool merged, bool tabs,
                    bool walk) {
        if (merged && walk)
            hipLaunchKernelGGL((k_qaoa_bwd_rt<CT, TB, TT, POOLED, true, true, true>), grid, dim3(threads), 0, st, P, W, g, B);
        else if (merged)
            hipLaunchKernelGGL((k_qaoa_bwd_rt<CT, TB, TT, POOLED, true, true>), grid, dim3(threads), 0, st, P, W, g, B);
        else if (tabs && walk)
            hipLaunchKernelGGL((k_qaoa_bwd_rt<CT, TB, TT, POOLED, false, true, true>), grid, dim3(threads), 0, st, P, W, g, B);
        else if (tabs)
            hipLaunchKernelGGL((k_qaoa_bwd_rt<CT, TB, TT, POOLED, false, true>), grid, dim3(threads), 0, st, P, W, g, B);
        else if (walk)
            hipLaunchKernelGGL((k_qaoa_bwd_rt<CT, TB, TT, POOLED, false, false, true>), grid, dim3(threads), 0, st, P, W, g, B);
        else
            hipLaunchKernelGGL((k_qaoa_bwd_rt<CT, TB, TT, POOLED, false, false>), grid, dim3(threads), 0, st, P, W, g, B);
    }
};
// LDS kernels serve n < 10: one qubit group, so no merged passes.
template <typename CT, bool POOLED> struct LdsKernels {
    static void fwd(dim3 grid, hipStream_t st, const QPass &P, const QWeights &W, const QGeom &g, const QBatch &B, bool, bool) {
        hipLaunchKernelGGL((k_qaoa_fwd_lds<CT, POOLED>), grid, dim3(kLdsThreads), 0, st, P, W, g, B);
    }
    static void bwd(dim3 grid, hipStream_t st, const QPass &P, const QWeights &W, const QGeom &g, const QBatch &B, bool, bool, bool) {
        hipLaunchKernelGGL((k_qaoa_bwd_lds<CT, POOLED>), grid, dim3(kLdsThreads), 0, st, P, W, g, B);
    }
};

// Forward (+ backward + final) launches for nb circuits.  Single-graph mode
// takes the pass descriptors by value from `passes`; pooled mode reads them
// from B.passes on the device.
template <typename K, bool POOLED>
static void launch_seq(const QPlan &plan, const QPass *passes, const QWeights &W, QBatch B, int nb, double *E_out, double *grad_out,
                       hipStream_t st) {
    const QGeom &g = plan.geo;
    const QLayout L = qaoa_layout(g, grad_out != nullptr);
    const size_t sb = ((size_t)1 << g.n) * 16;
    const int np = g.np;
    const dim3 grid((unsigned)((u64)nb << g.glog));
    B.lam_off = L.lam;
    B.part_off = L.part;
    B.epart_off = L.epart;
    static const QPass dummy{};
    auto pass = [&](int k) -> const QPass & { return POOLED ? dummy : passes[k]; };
    auto merged = [&](int k) { return plan.merged[k] != 0; };
    // Phase tables: unit weights only, and only where a pass applies a phase
    // (every graph of a pooled class shares the prototype's pass flags).
    auto tabs = [&](int k) {
        if (g.weighted) return false;
        if ((size_t)k >= plan.passes.size()) return true;
        return merged(k) || (plan.passes[k].flags & (QF_FIRST | QF_PHASE_END)) != 0;
    };
    // Backward passes ending in the third layout (the kernel's WALK): some RX
    // bit is an upper lane bit; for merged passes also every RX lane bit is
    // one, and some RX bit is an L0 wave bit.
    auto walk = [&](int k) {
        if (!plan.rt || (size_t)k >= plan.passes.size()) return false;
        const QPass &Q = plan.passes[k];
        const int TT = plan.shape.TT, JB = g.tb - TT, S = JB < 3 ? JB : 3, W = TT - 6;
        const u32 lanes = Q.rx_mask & 63u, upper = ((1u << S) - 1u) << (6 - S);
        if (S < 1 || !(lanes & upper)) return false;
        if (!merged(k)) return true;
        return (lanes & ~upper) == 0 && ((Q.rx_mask >> 6) & ((1u << W) - 1u)) != 0;
    };
    if (grad_out) {
        for (int k = 0; k < np; ++k) {
            B.k = k;
            B.in_off = k == 0 ? -1 : (long long)(L.ckpt + (size_t)(k - 1) * sb);
            B.out_off = (long long)(L.ckpt + (size_t)k * sb);
            K::fwd(grid, st, pass(k), W, g, B, merged(k), tabs(k));
        }
        for (int k = np - 1; k >= 0; --k) {
            B.k = k;
            B.in_off = (long long)(L.ckpt + (size_t)k * sb);
            K::bwd(grid, st, pass(k), W, g, B, merged(k), tabs(k), walk(k));
        }
        hipLaunchKernelGGL(k_qaoa_final<POOLED>, dim3(2 * g.p + 1, nb), dim3(256), 0, st, g, B, plan.map, E_out, grad_out, 1);
    } else {
        for (int k = 0; k < np; ++k) {
            B.k = k;
            B.in_off = k == 0 ? -1 : (long long)L.ckpt;
            B.out_off = k == np - 1 ? -1 : (long long)L.ckpt;
            K::fwd(grid, st, pass(k), W, g, B, merged(k), tabs(k));
        }
        hipLaunchKernelGGL(k_qaoa_final<POOLED>, dim3(1, nb), dim3(256), 0, st, g, B, plan.map, E_out, (double *)nullptr, 0);
    }
}

template <typename CT, bool POOLED>
static void launch_ct(const QPlan &plan, const QPass *passes, const QWeights &W, const QBatch &B, int nb, double *E_out, double *grad_out, hipStream_t st) {
    if (!plan.rt) return launch_seq<LdsKernels<CT, POOLED>, POOLED>(plan, passes, W, B, nb, E_out, grad_out, st);
    switch (plan.shape.TB) {
    case 10: return launch_seq<RtKernels<CT, 10, 8, POOLED>, POOLED>(plan, passes, W, B, nb, E_out, grad_out, st);
    case 11: return launch_seq<RtKernels<CT, 11, 8, POOLED>, POOLED>(plan, passes, W, B, nb, E_out, grad_out, st);
    case 12: return launch_seq<RtKernels<CT, 12, 9, POOLED>, POOLED>(plan, passes, W, B, nb, E_out, grad_out, st);
    default: return launch_seq<RtKernels<CT, 13, 9, POOLED>, POOLED>(plan, passes, W, B, nb, E_out, grad_out, st);
    }
}

int launch_qaoa_batch(const QPlan &plan, const double *theta, int nb, double *E_out, double *grad_out, char *ws, size_t circ_bytes, hipStream_t st) {
    QBatch B{};
    B.ws = ws;
    B.circ_bytes = circ_bytes;
    B.theta = theta;
    if (plan.geo.weighted)
        launch_ct<double, false>(plan, plan.passes.data(), plan.W, B, nb, E_out, grad_out, st);
    else
        launch_ct<int, false>(plan, plan.passes.data(), plan.W, B, nb, E_out, grad_out, st);
    QS_LAUNCH_CHECK("qaoa");
    return QS_OK;
}

int launch_qaoa_pooled(const QPlan &proto, const QBatch &B, int nb, double *E_out, double *grad_out, hipStream_t st) {
    static const QWeights unit = [] {
        QWeights w;
        for (int e = 0; e < kQMaxEdges; ++e) w.w[e] = 1.0;
        return w;
    }();
    launch_ct<int, true>(proto, nullptr, unit, B, nb, E_out, grad_out, st);
    QS_LAUNCH_CHECK("qaoa_pool");
    return QS_OK;
}

int check_edges(int n, int ne, const int32_t *edges) {
    if (!edges || ne < 1 || ne > kQMaxEdges) return fail(QS_ERR_ARG, "QAOA needs 1..128 edges");
    for (int e = 0; e < ne; ++e) {
        const int a = edges[2 * e], b = edges[2 * e + 1];
        if (a < 0 || b < 0 || a >= n || b >= n || a == b) return fail(QS_ERR_ARG, "QAOA edge out of range or self-loop");
    }
    return QS_OK;
}

// Plans of recent problems, keyed by the descriptor's contents (n, p, edges,
// weights): a variational loop calls qs_qaoa_run with one graph many times,
// and a plan takes longer to build on the host than a small circuit takes on
// the device.  At most kQPlanCache entries; beyond, the least recently used
// one is dropped (callers still holding it keep their shared copy).
constexpr size_t kQPlanCache = 16;
struct QPlanEntry {
    std::shared_ptr<const QPlan> plan;
    uint64_t last_use = 0;
};

static int cached_qplan(const qs_qaoa_desc *d, std::shared_ptr<const QPlan> &out) {
    static std::mutex mu;
    static std::unordered_map<std::string, QPlanEntry> cache;
    static uint64_t clock = 0;
    std::string key;
    auto add = [&](const void *p, size_t n) { key.append((const char *)p, n); };
    add(&d->n, sizeof d->n);
    add(&d->p, sizeof d->p);
    add(&d->num_edges, sizeof d->num_edges);
    add(d->edges, sizeof(int32_t) * 2 * (size_t)d->num_edges);
    const char weighted = d->w != nullptr;
    add(&weighted, 1);
    if (d->w) add(d->w, sizeof(double) * (size_t)d->num_edges);
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(key);
    if (it == cache.end()) {
        auto plan = std::make_shared<QPlan>();
        if (int rc = build_qplan(d->n, d->p, d->num_edges, d->edges, d->w, qaoa_default_shape(d->n), *plan)) return rc;
        if (cache.size() >= kQPlanCache) {
            auto lru = cache.begin();
            for (auto j = cache.begin(); j != cache.end(); ++j)
                if (j->second.last_use < lru->second.last_use) lru = j;
            cache.erase(lru);
        }
        it = cache.emplace(std::move(key), QPlanEntry{std::move(plan), 0}).first;
    }
    it->second.last_use = ++clock;
    out = it->second.plan;
    return QS_OK;
}

static int check_desc(const qs_qaoa_desc *d) {
    if (!d) return fail(QS_ERR_ARG, "null QAOA descriptor");
    if (d->n < 2 || d->n > QS_MAX_QUBITS_C128) return fail(QS_ERR_ARG, "QAOA n must be in [2, 34]");
    if (d->p < 1 || d->p > 64) return fail(QS_ERR_ARG, "QAOA p must be in [1, 64]");
    return check_edges(d->n, d->num_edges, d->edges);
}

}  // namespace qs

using namespace qs;

QS_API int qs_qaoa_workspace_bytes(const qs_qaoa_desc *d, int with_grad, size_t *bytes) {
    try {
        if (int rc = check_desc(d)) return rc;
        if (!bytes) return fail(QS_ERR_ARG, "null output");
        std::shared_ptr<const QPlan> plan;
        if (int rc = cached_qplan(d, plan)) return rc;
        *bytes = qaoa_layout(plan->geo, with_grad).bytes;
        return QS_OK;
    } catch (...) {
        return fail(QS_ERR_UNSUPPORTED, "unexpected internal error");
    }
}

QS_API int qs_qaoa_run(const qs_qaoa_desc *d, const double *angles_dev, int B, double *E_dev, double *grad_dev, void *ws, size_t ws_bytes,
                       void *stream) {
    try {
        if (int rc = check_desc(d)) return rc;
        if (!angles_dev || !E_dev || !ws || B < 0) return fail(QS_ERR_ARG, "null angles, energies or workspace");
        std::shared_ptr<const QPlan> plan;
        if (int rc = cached_qplan(d, plan)) return rc;
        const size_t circ = qaoa_layout(plan->geo, grad_dev != nullptr).bytes;
        if (ws_bytes < circ) return fail(QS_ERR_SIZE, "QAOA workspace too small");
        // As many angle sets per launch as the workspace holds.
        const u64 fit = ws_bytes / circ;
        const int per = (int)(fit < (u64)B ? fit : (u64)B);
        hipStream_t st = (hipStream_t)stream;
        for (int b0 = 0; b0 < B; b0 += per) {
            const int nb = B - b0 < per ? B - b0 : per;
            const int rc = launch_qaoa_batch(*plan, angles_dev + (size_t)b0 * 2 * d->p, nb, E_dev + b0,
                                             grad_dev ? grad_dev + (size_t)b0 * 2 * d->p : nullptr, (char *)ws, circ, st);
            if (rc) return rc;
        }
        return QS_OK;
    } catch (...) {
        return fail(QS_ERR_UNSUPPORTED, "unexpected internal error");
    }
}
