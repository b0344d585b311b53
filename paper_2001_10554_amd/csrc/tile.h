// Tile-pass plans shared by the fused-block and trajectory kernels.
#pragma once

#include <vector>

#include "common.h"

namespace qs {

// A gate of a pass, with its qubits also given as tile-bit positions.
struct DGate {
    int32_t kind;
    int8_t p0, p1;  // tile-bit positions of q0 / q1, -1 when outside the tile
    int8_t q0, q1;
    int32_t pad;
    double u[8];
};

// One pass: the tile qubit set and the slice of the gate list it applies.
struct DPass {
    int tb;
    int nrest;
    uint8_t T[16];     // tile bit -> qubit (ascending)
    uint8_t rest[40];  // remaining bits -> qubit (ascending)
    int gate_begin, gate_count;
};

inline int tile_bits_max(int dtype) { return dtype == QS_C128 ? 12 : 13; }

// Greedy split of a gate list into passes: a pass takes the longest prefix of
// the remaining gates whose targets (1Q target, C1Q target, both SWAP qubits)
// fit in a tile of tile_bits_max(dtype) qubits that also holds the lowest
// qubits; diagonal gates and controls outside the tile ride along.
void make_plan(int n, int dtype, const qs_gate *g, int count, std::vector<DPass> &passes, std::vector<DGate> &dg);

template <typename R> __device__ __forceinline__ Mat2<R> load_mat(const double *u) {
    Mat2<R> m;
#pragma unroll
    for (int k = 0; k < 8; ++k) m.m[k] = (R)u[k];
    return m;
}

__device__ __forceinline__ u64 pass_base(const DPass &P, u64 tile) {
    u64 base = 0;
    for (int b = 0; b < P.nrest; ++b) base |= ((tile >> b) & 1ull) << P.rest[b];
    return base;
}

__device__ __forceinline__ u64 pass_off(const DPass &P, u64 m) {
    u64 off = 0;
    for (int b = 0; b < P.tb; ++b) off |= ((m >> b) & 1ull) << P.T[b];
    return off;
}

// Apply one gate to an LDS tile of TS = 2^tb amplitudes whose fixed (non-tile)
// bits are `base`.  cval: the control value a C1Q gate fires on (1 normally).
// u: the 2x2 matrix (1Q / C1Q) or the 4 diagonal entries (DIAG2), as doubles.
// Ends with a barrier.
template <typename R, int NT>
__device__ __forceinline__ void lds_apply_gate(cx<R> *sh, u64 TS, u64 base, int kind, int p0, int p1, int q0, int q1, int cval,
                                               const double *u) {
    if (kind == QS_G_1Q || (kind == QS_G_C1Q && p0 < 0)) {
        const int p = kind == QS_G_1Q ? p0 : p1;
        const bool on = kind == QS_G_1Q || (int)((base >> q0) & 1ull) == cval;
        if (on) {
            const Mat2<R> m = load_mat<R>(u);
            for (u64 k = threadIdx.x; k < TS / 2; k += NT) {
                const u64 m0 = insert0(k, p), m1 = m0 | (1ull << p);
                cx<R> a = sh[m0], b = sh[m1];
                apply2<R>(m, a, b);
                sh[m0] = a;
                sh[m1] = b;
            }
        }
    } else if (kind == QS_G_C1Q) {
        const Mat2<R> m = load_mat<R>(u);
        const int lo = p0 < p1 ? p0 : p1, hi = p0 < p1 ? p1 : p0;
        const u64 cbit = cval ? (1ull << p0) : 0ull;
        for (u64 k = threadIdx.x; k < TS / 4; k += NT) {
            const u64 m0 = insert0(insert0(k, lo), hi) | cbit, m1 = m0 | (1ull << p1);
            cx<R> a = sh[m0], b = sh[m1];
            apply2<R>(m, a, b);
            sh[m0] = a;
            sh[m1] = b;
        }
    } else if (kind == QS_G_DIAG2) {
        for (u64 mm = threadIdx.x; mm < TS; mm += NT) {
            const int b0 = p0 >= 0 ? (int)((mm >> p0) & 1) : (int)((base >> q0) & 1);
            const int b1 = p1 >= 0 ? (int)((mm >> p1) & 1) : (int)((base >> q1) & 1);
            const int e = 2 * b1 + b0;
            cx<R> f;
            f.x = (R)u[2 * e];
            f.y = (R)u[2 * e + 1];
            sh[mm] = cmul<R>(sh[mm], f);
        }
    } else if (kind == QS_G_SWAP) {
        const int lo = p0 < p1 ? p0 : p1, hi = p0 < p1 ? p1 : p0;
        for (u64 k = threadIdx.x; k < TS / 4; k += NT) {
            const u64 b = insert0(insert0(k, lo), hi);
            const u64 i = b | (1ull << p0), j = b | (1ull << p1);
            const cx<R> x = sh[i], y = sh[j];
            sh[i] = y;
            sh[j] = x;
        }
    }
    __syncthreads();
}

}  // namespace qs
