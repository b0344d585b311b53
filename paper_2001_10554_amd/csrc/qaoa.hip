// QAOA Max-Cut: fused forward passes and the adjoint (reverse) sweep, batched
// over circuits that share one graph.
//
// Circuit: |psi> = prod_l exp(-i beta_l B) exp(-i gamma_l C) H^n |0>, with
// B = sum_j X_j (so exp(-i beta B) = prod_j RX_j(2 beta)) and C the cut
// counter; E = <psi|C|psi>.
//
// Pass structure.  The qubits are split into groups: G_0 = the TB lowest
// qubits, then groups of at most TB - 3 higher qubits (their tiles also hold
// qubits 0..2 so every row is a 128-byte line).  Layer l is P passes, pass
// (l, g) applying RX(2 beta_l) to the qubits of G_g inside an LDS tile.  The
// diagonal cost layers ride along: exp(-i gamma_1 C) is applied at the start
// of the very first pass (on the uniform state generated in registers), and
// exp(-i gamma_{l+1} C) at the end of pass (l, P-1).  The last pass also
// accumulates E.
//
// Adjoint.  The forward writes every pass's output as a checkpoint.  The
// backward walks the passes in reverse with lambda (lambda = C psi at the
// end): because all RX of one mixer commute with each X_j, the derivative
// inner products 2 Im<lambda|X_j|psi> of a pass's qubits can all be taken at
// the pass's end point, where lambda and the checkpoint coincide; a phase at
// the end of the pass gives 2 Im<lambda|C|psi> there and is then undone on
// both vectors element-wise; finally RX(-2 beta) is applied to lambda only.
// psi is therefore never transformed through LDS.  The first pass's phase sits
// at its start, so its inner product uses psi regenerated on the fly
// (exp(-i gamma_1 C(k)) 2^{-n/2}).  Inner products are per-block FP64 partial
// sums, reduced in a fixed order.
//
// Cut values.  C(k) is never evaluated edge by edge per amplitude: for the
// thread map m = tid + 256 j each edge is classified once per pass by where
// its endpoints sit (thread-index bit, register-index bit, or a bit fixed per
// tile), and a thread folds the edges into a constant plus one coefficient per
// register bit.
//
// Batching.  blockIdx.x = circuit * G + tile; circuit c owns the workspace
// region ws + c * circ_bytes and the angle vector theta + c * 2p.
#include <cmath>
#include <vector>

#include "launch.h"
#include "qaoa.h"
#include "vec.h"

#define QS_API extern "C" __attribute__((visibility("default")))

namespace qs {

// Cut value of the thread's R amplitudes m = tid + 256 j.  CT = int (unit
// weights) or double.  JB = register-index bits of the tile size.
template <typename CT, int JB>
__device__ __forceinline__ void cut_values(const QPass &P, const QWeights &W, bool weighted, u64 base, int tid, CT (&C)[1 << JB]) {
    constexpr int R = 1 << JB;
    CT cb = 0;
    CT coef[JB > 0 ? JB : 1] = {};
    int k = 0;
    auto wt = [&](const QEdge &e) -> CT { return weighted ? (CT)W.w[e.wi] : (CT)1; };
    for (int i = 0; i < P.cnt[EC_TT]; ++i, ++k) {
        const QEdge e = P.e[k];
        cb += (((tid >> e.a) ^ (tid >> e.b)) & 1) ? wt(e) : (CT)0;
    }
    for (int i = 0; i < P.cnt[EC_TR]; ++i, ++k) {
        const QEdge e = P.e[k];
        cb += (((tid >> e.a) & 1) != (int)((base >> e.b) & 1)) ? wt(e) : (CT)0;
    }
    for (int i = 0; i < P.cnt[EC_TJ]; ++i, ++k) {
        const QEdge e = P.e[k];
        const int ta = (tid >> e.a) & 1;
        const CT w = wt(e);
        cb += ta ? w : (CT)0;
#pragma unroll
        for (int x = 0; x < JB; ++x)
            if (x == e.b) coef[x] += ta ? -w : w;
    }
    const int kjj = k;
    k += P.cnt[EC_JJ];
    for (int i = 0; i < P.cnt[EC_JR]; ++i, ++k) {
        const QEdge e = P.e[k];
        const int br = (int)((base >> e.b) & 1);
        const CT w = wt(e);
        cb += br ? w : (CT)0;
#pragma unroll
        for (int x = 0; x < JB; ++x)
            if (x == e.a) coef[x] += br ? -w : w;
    }
    for (int i = 0; i < P.cnt[EC_RR]; ++i, ++k) {
        const QEdge e = P.e[k];
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
    for (int i = 0; i < P.cnt[EC_JJ]; ++i) {
        const QEdge e = P.e[kjj + i];
        const CT w = wt(e);
#pragma unroll
        for (int j = 0; j < R; ++j)
            if (((j >> e.a) ^ (j >> e.b)) & 1) C[j] += w;
    }
}

__device__ __forceinline__ u64 qtile_base(const QPass &P, u64 tile) {
    u64 base = 0;
    for (int b = 0; b < P.nrest; ++b) base |= ((tile >> b) & 1ull) << P.rest[b];
    return base;
}

__device__ __forceinline__ u64 qtile_off(const QPass &P, u64 m) {
    u64 off = 0;
    for (int b = 0; b < P.tb; ++b) off |= ((m >> b) & 1ull) << P.T[b];
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
    for (int c = threadIdx.x; c <= ne_total; c += kQThreads) {
        double s, co;
        sincos(g * (double)c, &s, &co);
        d2v v;
        v.x = co;
        v.y = -s;
        tab[c] = v;
    }
}

// RX(theta) with (c, s) = (cos theta/2, sin theta/2) on LDS pairs of tile bit b.
__device__ __forceinline__ void lds_rx(d2v *sh, int TS, int b, double c, double s) {
    for (int k = threadIdx.x; k < TS / 2; k += kQThreads) {
        const int m0 = (int)insert0((u64)k, b), m1 = m0 | (1 << b);
        const d2v a = sh[m0], v = sh[m1];
        d2v na, nb;
        na.x = c * a.x + s * v.y;
        na.y = c * a.y - s * v.x;
        nb.x = s * a.y + c * v.x;
        nb.y = c * v.y - s * a.x;
        sh[m0] = na;
        sh[m1] = nb;
    }
}

__device__ __forceinline__ double qblock_sum(double v, double *sh) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    for (int k = 0; k < kQThreads / 64; ++k) t += sh[k];
    return t;
}

// Forward pass.  in_off < 0 only for the first pass (uniform state generated
// on the fly); out_off < 0 skips the store (E-only last pass).
template <typename CT, int TB, bool POOLED>
__global__ __launch_bounds__(kQThreads) void k_qaoa_fwd(QPass Parg, QWeights W, QGeom geo, QBatch B) {
    constexpr int JB = TB - 8, R = 1 << JB;
    __shared__ d2v sh[1 << TB];
    __shared__ d2v tab_a[kQMaxEdges + 1], tab_b[kQMaxEdges + 1];
    __shared__ double red[kQThreads / 64];
    const u64 c = blockIdx.x >> geo.glog, tile = blockIdx.x & ((1ull << geo.glog) - 1);
    const QPass *Pp;
    u64 cid;
    if constexpr (POOLED) {
        Pp = B.passes + ((B.c0 + c) / B.sets) * B.np + B.k;
        cid = (u64)B.circ_map[B.c0 + c];
    } else {
        Pp = &Parg;
        cid = c;
    }
    const QPass &P = *Pp;
    char *region = B.ws + c * B.circ_bytes;
    const d2v *in = B.in_off >= 0 ? (const d2v *)(region + B.in_off) : nullptr;
    d2v *out = B.out_off >= 0 ? (d2v *)(region + B.out_off) : nullptr;
    const double *theta = B.theta + cid * 2 * geo.p;
    const int TS = 1 << P.tb;
    const int tid = threadIdx.x;
    const int l = P.layer, p = geo.p;
    const u64 base = qtile_base(P, tile);
    const bool first = P.flags & QF_FIRST, pend = P.flags & QF_PHASE_END, last = P.flags & QF_LAST;
    const double g_a = theta[l], g_b = pend ? theta[l + 1] : 0.0;
    if (!geo.weighted) {
        if (first) fill_table(tab_a, geo.num_edges, g_a);
        if (pend) fill_table(tab_b, geo.num_edges, g_b);
    }
    CT C[R];
    cut_values<CT, JB>(P, W, geo.weighted, base, tid, C);
    __syncthreads();

    const double amp0 = 1.0 / sqrt((double)(1ull << geo.n));
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int m = tid + kQThreads * j;
        if (m < TS) {
            d2v v;
            if (first) {
                const d2v f = Phase<CT>::get(tab_a, g_a, C[j]);
                v.x = amp0 * f.x;
                v.y = amp0 * f.y;
            } else {
                v = ld<true>(in + (base | qtile_off(P, (u64)m)));
            }
            sh[m] = v;
        }
    }
    __syncthreads();
    double sb, cb;
    sincos(theta[p + l], &sb, &cb);  // RX(2 beta): cos(beta), sin(beta)
    for (int b = 0; b < P.tb; ++b) {
        if (!((P.rx_mask >> b) & 1)) continue;
        lds_rx(sh, TS, b, cb, sb);
        __syncthreads();
    }
    double e_acc = 0.0;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int m = tid + kQThreads * j;
        if (m < TS) {
            d2v v = sh[m];
            if (pend) v = cmul2(v, Phase<CT>::get(tab_b, g_b, C[j]));
            if (last) e_acc += (double)C[j] * (v.x * v.x + v.y * v.y);
            if (out) st<true>(out + (base | qtile_off(P, (u64)m)), v);
        }
    }
    if (last) {
        const double t = qblock_sum(e_acc, red);
        if (tid == 0) ((double *)(region + B.epart_off))[tile] = t;
    }
}

// Backward pass: see the file comment.  partial[pidx][tile][3] = (Im<lam|C|psi>
// at the end phase, sum_j Im<lam|X_j|psi>, Im<lam|C|phi_1> at the first pass's
// start phase).  The checkpoint is read from in_off, lambda lives at lam_off.
template <typename CT, int TB, bool POOLED>
__global__ __launch_bounds__(kQThreads) void k_qaoa_bwd(QPass Parg, QWeights W, QGeom geo, QBatch B) {
    constexpr int JB = TB - 8, R = 1 << JB;
    __shared__ d2v shl[1 << TB], shp[1 << TB];
    __shared__ d2v tab_a[kQMaxEdges + 1], tab_b[kQMaxEdges + 1];
    __shared__ double red[kQThreads / 64];
    const u64 c = blockIdx.x >> geo.glog, tile = blockIdx.x & ((1ull << geo.glog) - 1);
    const QPass *Pp;
    u64 cid;
    if constexpr (POOLED) {
        Pp = B.passes + ((B.c0 + c) / B.sets) * B.np + B.k;
        cid = (u64)B.circ_map[B.c0 + c];
    } else {
        Pp = &Parg;
        cid = c;
    }
    const QPass &P = *Pp;
    char *region = B.ws + c * B.circ_bytes;
    const d2v *ckpt = (const d2v *)(region + B.in_off);
    d2v *lam = (d2v *)(region + B.lam_off);
    double *partial = (double *)(region + B.part_off);
    const double *theta = B.theta + cid * 2 * geo.p;
    const int TS = 1 << P.tb;
    const int tid = threadIdx.x;
    const int l = P.layer, p = geo.p;
    const u64 base = qtile_base(P, tile);
    const bool first = P.flags & QF_FIRST, pend = P.flags & QF_PHASE_END, last = P.flags & QF_LAST;
    const double g_a = theta[l], g_b = pend ? theta[l + 1] : 0.0;
    if (!geo.weighted) {
        if (first) fill_table(tab_a, geo.num_edges, g_a);
        if (pend) fill_table(tab_b, geo.num_edges, -g_b);  // exp(+i gamma C): undo the phase
    }
    CT C[R];
    cut_values<CT, JB>(P, W, geo.weighted, base, tid, C);
    __syncthreads();

    double ipc = 0.0, ipb = 0.0, ipc1 = 0.0;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int m = tid + kQThreads * j;
        if (m < TS) {
            const u64 idx = base | qtile_off(P, (u64)m);
            d2v ps = ld<true>(ckpt + idx);
            d2v lm;
            if (last) {
                lm.x = (double)C[j] * ps.x;
                lm.y = (double)C[j] * ps.y;
            } else {
                lm = ld<true>(lam + idx);
            }
            if (pend) {
                // Im(conj(lam) psi) weighted by C, then undo exp(-i gamma C) on both.
                ipc += (double)C[j] * (lm.x * ps.y - lm.y * ps.x);
                const d2v f = Phase<CT>::get(tab_b, -g_b, C[j]);
                lm = cmul2(lm, f);
                ps = cmul2(ps, f);
            }
            shl[m] = lm;
            shp[m] = ps;
        }
    }
    __syncthreads();
    for (int b = 0; b < P.tb; ++b) {
        if (!((P.rx_mask >> b) & 1)) continue;
        for (int k = tid; k < TS / 2; k += kQThreads) {
            const int m0 = (int)insert0((u64)k, b), m1 = m0 | (1 << b);
            const d2v l0 = shl[m0], l1 = shl[m1], p0 = shp[m0], p1 = shp[m1];
            ipb += (l0.x * p1.y - l0.y * p1.x) + (l1.x * p0.y - l1.y * p0.x);
        }
    }
    __syncthreads();  // all inner products read lambda before RX(-2 beta) rewrites it
    double sb, cb;
    sincos(theta[p + l], &sb, &cb);
    for (int b = 0; b < P.tb; ++b) {
        if (!((P.rx_mask >> b) & 1)) continue;
        lds_rx(shl, TS, b, cb, -sb);  // RX(-2 beta)
        __syncthreads();
    }
    const double amp0 = 1.0 / sqrt((double)(1ull << geo.n));
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int m = tid + kQThreads * j;
        if (m < TS) {
            const d2v lm = shl[m];
            if (first) {
                const d2v f = Phase<CT>::get(tab_a, g_a, C[j]);  // phi_1 = 2^{-n/2} exp(-i gamma_1 C)
                ipc1 += (double)C[j] * amp0 * (lm.x * f.y - lm.y * f.x);
            } else {
                st<true>(lam + (base | qtile_off(P, (u64)m)), lm);
            }
        }
    }
    const double tc = qblock_sum(ipc, red);
    const double tbx = qblock_sum(ipb, red);
    const double tc1 = qblock_sum(ipc1, red);
    if (tid == 0) {
        double *o = partial + ((u64)P.pidx * geo.G + tile) * 3;
        o[0] = tc;
        o[1] = tbx;
        o[2] = tc1;
    }
}

// E and gradient of circuit blockIdx.y: one block per output, partials summed
// in a fixed order.  Output k < 2p: gradient component; k = 2p: E.  Without a
// gradient the grid has one block per circuit, which computes E.
template <bool POOLED>
__global__ __launch_bounds__(kQThreads) void k_qaoa_final(QGeom geo, QBatch B, double *__restrict__ E_out, double *__restrict__ grad_out, int with_grad) {
    __shared__ double red[kQThreads / 64];
    const int p = geo.p, P = geo.P, G = geo.G;
    const int k = with_grad ? (int)blockIdx.x : 2 * p;
    const u64 c = blockIdx.y;
    const u64 cid = POOLED ? (u64)B.circ_map[B.c0 + c] : c;
    const char *region = B.ws + c * B.circ_bytes;
    const double *partial = (const double *)(region + B.part_off);
    const double *e_partial = (const double *)(region + B.epart_off);
    double a = 0.0;
    if (k == 2 * p) {
        for (int b = threadIdx.x; b < G; b += kQThreads) a += e_partial[b];
    } else if (k < p) {
        // gamma_{k+1}: phase at the start of pass 0 (k = 0, slot 2) or the end of pass (k-1, P-1) (slot 0).
        const int pidx = k == 0 ? 0 : (k - 1) * P + (P - 1);
        const int slot = k == 0 ? 2 : 0;
        for (int b = threadIdx.x; b < G; b += kQThreads) a += partial[((u64)pidx * G + b) * 3 + slot];
    } else {
        const int l = k - p;
        for (int g = 0; g < P; ++g) {
            const int pidx = l * P + g;
            for (int b = threadIdx.x; b < G; b += kQThreads) a += partial[((u64)pidx * G + b) * 3 + 1];
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

// ------------------------------------------------------------------ host planning

int build_qplan(int n, int p, int num_edges, const int32_t *edges, const double *w, int TB, QPlan &plan) {
    const int tb = n < TB ? n : TB;
    const int r = tb < 3 ? tb : 3;
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
    plan.TB = TB;
    plan.geo = QGeom{n, p, P, tb, 1 << (n - tb), n - tb, num_edges, w != nullptr};
    for (int e = 0; e < num_edges; ++e) plan.W.w[e] = w ? w[e] : 1.0;
    plan.passes.clear();
    for (int l = 0; l < p; ++l) {
        for (int g = 0; g < P; ++g) {
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
            Q.layer = l;
            Q.pidx = l * P + g;
            Q.flags = 0;
            if (l == 0 && g == 0) Q.flags |= QF_FIRST;
            if (g == P - 1 && l < p - 1) Q.flags |= QF_PHASE_END;
            if (g == P - 1 && l == p - 1) Q.flags |= QF_LAST;
            // Classify edges for the thread map m = tid + 256 j: tile bits 0..7
            // are thread-index bits, higher tile bits register-index bits.
            std::vector<QEdge> cls[EC_N];
            for (int e = 0; e < num_edges; ++e) {
                int u = edges[2 * e], v = edges[2 * e + 1];
                int pu = pos[u], pv = pos[v];
                auto kind = [](int ps) { return ps < 0 ? 2 : (ps < 8 ? 0 : 1); };  // 0 = t, 1 = j, 2 = r
                int ku = kind(pu), kv = kind(pv);
                if (ku > kv) {
                    std::swap(u, v);
                    std::swap(pu, pv);
                    std::swap(ku, kv);
                }
                QEdge x{};
                x.wi = (uint8_t)e;
                if (ku == 0 && kv == 0) { x.a = pu; x.b = pv; cls[EC_TT].push_back(x); }
                else if (ku == 0 && kv == 2) { x.a = pu; x.b = v; cls[EC_TR].push_back(x); }
                else if (ku == 0 && kv == 1) { x.a = pu; x.b = pv - 8; cls[EC_TJ].push_back(x); }
                else if (ku == 1 && kv == 1) { x.a = pu - 8; x.b = pv - 8; cls[EC_JJ].push_back(x); }
                else if (ku == 1 && kv == 2) { x.a = pu - 8; x.b = v; cls[EC_JR].push_back(x); }
                else { x.a = u; x.b = v; cls[EC_RR].push_back(x); }
            }
            int k = 0;
            for (int c = 0; c < EC_N; ++c) {
                Q.cnt[c] = (uint16_t)cls[c].size();
                for (auto &x : cls[c]) Q.e[k++] = x;
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
    const size_t np = (size_t)g.p * g.P;
    size_t off = 0;
    if (with_grad) {
        L.ckpt = off;
        off += np * sb;
        L.lam = off;
        off += sb;
        L.part = off;
        off = align256(off + np * (size_t)g.G * 3 * sizeof(double));
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

// Forward (+ backward + final) launches for nb circuits.  Single-graph mode
// takes the pass descriptors by value from `passes`; pooled mode reads them
// from B.passes on the device.
template <typename CT, int TB, bool POOLED>
static void launch_batch_t(const QGeom &g, const QPass *passes, const QWeights &W, QBatch B, int nb, double *E_out, double *grad_out,
                           hipStream_t st) {
    const QLayout L = qaoa_layout(g, grad_out != nullptr);
    const size_t sb = ((size_t)1 << g.n) * 16;
    const int np = g.p * g.P;
    const dim3 grid((unsigned)((u64)nb << g.glog)), block(kQThreads);
    B.lam_off = L.lam;
    B.part_off = L.part;
    B.epart_off = L.epart;
    const QPass dummy{};
    auto pass = [&](int k) -> const QPass & { return POOLED ? dummy : passes[k]; };
    if (grad_out) {
        for (int k = 0; k < np; ++k) {
            B.k = k;
            B.in_off = k == 0 ? -1 : (long long)(L.ckpt + (size_t)(k - 1) * sb);
            B.out_off = (long long)(L.ckpt + (size_t)k * sb);
            hipLaunchKernelGGL((k_qaoa_fwd<CT, TB, POOLED>), grid, block, 0, st, pass(k), W, g, B);
        }
        for (int k = np - 1; k >= 0; --k) {
            B.k = k;
            B.in_off = (long long)(L.ckpt + (size_t)k * sb);
            hipLaunchKernelGGL((k_qaoa_bwd<CT, TB, POOLED>), grid, block, 0, st, pass(k), W, g, B);
        }
        hipLaunchKernelGGL(k_qaoa_final<POOLED>, dim3(2 * g.p + 1, nb), block, 0, st, g, B, E_out, grad_out, 1);
    } else {
        for (int k = 0; k < np; ++k) {
            B.k = k;
            B.in_off = k == 0 ? -1 : (long long)L.ckpt;
            B.out_off = k == np - 1 ? -1 : (long long)L.ckpt;
            hipLaunchKernelGGL((k_qaoa_fwd<CT, TB, POOLED>), grid, block, 0, st, pass(k), W, g, B);
        }
        hipLaunchKernelGGL(k_qaoa_final<POOLED>, dim3(1, nb), block, 0, st, g, B, E_out, (double *)nullptr, 0);
    }
}

template <bool POOLED>
static int launch_any(int TB, const QGeom &g, const QPass *passes, const QWeights &W, const QBatch &B, int nb, double *E_out, double *grad_out,
                      hipStream_t st) {
    const bool w = g.weighted;
    switch (TB) {
    case 10: w ? launch_batch_t<double, 10, POOLED>(g, passes, W, B, nb, E_out, grad_out, st)
               : launch_batch_t<int, 10, POOLED>(g, passes, W, B, nb, E_out, grad_out, st); break;
    case 12: w ? launch_batch_t<double, 12, POOLED>(g, passes, W, B, nb, E_out, grad_out, st)
               : launch_batch_t<int, 12, POOLED>(g, passes, W, B, nb, E_out, grad_out, st); break;
    default: w ? launch_batch_t<double, 11, POOLED>(g, passes, W, B, nb, E_out, grad_out, st)
               : launch_batch_t<int, 11, POOLED>(g, passes, W, B, nb, E_out, grad_out, st); break;
    }
    QS_LAUNCH_CHECK("qaoa");
    return QS_OK;
}

int launch_qaoa_batch(const QPlan &plan, const double *theta, int nb, double *E_out, double *grad_out, char *ws, size_t circ_bytes, hipStream_t st) {
    QBatch B{};
    B.ws = ws;
    B.circ_bytes = circ_bytes;
    B.theta = theta;
    return launch_any<false>(plan.TB, plan.geo, plan.passes.data(), plan.W, B, nb, E_out, grad_out, st);
}

int launch_qaoa_pooled(int TB, const QGeom &geo, const QBatch &B, int nb, double *E_out, double *grad_out, hipStream_t st) {
    static const QWeights unit = [] {
        QWeights w;
        for (int e = 0; e < kQMaxEdges; ++e) w.w[e] = 1.0;
        return w;
    }();
    return launch_any<true>(TB, geo, nullptr, unit, B, nb, E_out, grad_out, st);
}

static int check_desc(const qs_qaoa_desc *d) {
    if (!d) return fail(QS_ERR_ARG, "null QAOA descriptor");
    if (d->n < 2 || d->n > QS_MAX_QUBITS_C128) return fail(QS_ERR_ARG, "QAOA n must be in [2, 34]");
    if (d->p < 1 || d->p > 64) return fail(QS_ERR_ARG, "QAOA p must be in [1, 64]");
    return check_edges(d->n, d->num_edges, d->edges);
}

int check_edges(int n, int ne, const int32_t *edges) {
    if (!edges || ne < 1 || ne > kQMaxEdges) return fail(QS_ERR_ARG, "QAOA needs 1..128 edges");
    for (int e = 0; e < ne; ++e) {
        const int a = edges[2 * e], b = edges[2 * e + 1];
        if (a < 0 || b < 0 || a >= n || b >= n || a == b) return fail(QS_ERR_ARG, "QAOA edge out of range or self-loop");
    }
    return QS_OK;
}

// Tile bits for a single QAOA instance: QSIM_QAOA_TB overrides the default.
int qaoa_default_tb(int n) {
    static int env = [] {
        const char *e = getenv("QSIM_QAOA_TB");
        return e ? atoi(e) : 0;
    }();
    if (env == 10 || env == 11 || env == 12) return env;
    (void)n;
    return 11;
}

}  // namespace qs

using namespace qs;

QS_API int qs_qaoa_workspace_bytes(const qs_qaoa_desc *d, int with_grad, size_t *bytes) {
    try {
        if (int rc = check_desc(d)) return rc;
        if (!bytes) return fail(QS_ERR_ARG, "null output");
        QPlan plan;
        build_qplan(d->n, d->p, d->num_edges, d->edges, d->w, qaoa_default_tb(d->n), plan);
        *bytes = qaoa_layout(plan.geo, with_grad).bytes;
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
        QPlan plan;
        build_qplan(d->n, d->p, d->num_edges, d->edges, d->w, qaoa_default_tb(d->n), plan);
        const size_t circ = qaoa_layout(plan.geo, grad_dev != nullptr).bytes;
        if (ws_bytes < circ) return fail(QS_ERR_SIZE, "QAOA workspace too small");
        // As many angle sets per launch as the workspace holds.
        const u64 fit = ws_bytes / circ;
        const int per = (int)(fit < (u64)B ? fit : (u64)B);
        hipStream_t st = (hipStream_t)stream;
        for (int b0 = 0; b0 < B; b0 += per) {
            const int nb = B - b0 < per ? B - b0 : per;
            const int rc = launch_qaoa_batch(plan, angles_dev + (size_t)b0 * 2 * d->p, nb, E_dev + b0,
                                             grad_dev ? grad_dev + (size_t)b0 * 2 * d->p : nullptr, (char *)ws, circ, st);
            if (rc) return rc;
        }
        return QS_OK;
    } catch (...) {
        return fail(QS_ERR_UNSUPPORTED, "unexpected internal error");
    }
}
