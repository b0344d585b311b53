// Tile-pass plans shared by the fused-block and trajectory kernels.
#pragma once

#include <string>
#include <vector>

#include "common.h"

namespace qs {

// Threads of an LDS-pass workgroup: one 8-amplitude register group each for a
// 12-bit c128 tile (two for a 13-bit c64 tile), and 8 waves per workgroup so
// that LDS and barrier latency is hidden within the CU.
constexpr int kTileThreads = 512;

// A gate of a pass, with its qubits also given as tile-bit positions.
//
// Sweeps: the gates of a pass are further cut into runs whose non-diagonal
// targets (1Q / noise target, C1Q target, both SWAP qubits) lie in at most
// three tile bits, the sweep's group bits g[0] < g[1] < g[2].  A sweep is
// applied to groups of 8 amplitudes that differ only in those bits, held in
// registers: one LDS read, one LDS write and one barrier per sweep instead of
// per gate.  Diagonal gates and the controls of C1Q gates may sit on any bit.
struct DGate {
    int32_t kind;
    int8_t p0, p1;  // tile-bit positions of q0 / q1, -1 when outside the tile
    int8_t q0, q1;
    int8_t s0, s1;  // group slot (0..2) of p0 / p1 in the gate's sweep, -1 if not a group bit
    int8_t g[3];    // first gate of a sweep: the group bits (ascending); unused otherwise
    int8_t pad0;    // trajectory plans: 1 = also applies the next gate (a noise gate on its qubit), 2 = that noise gate
    int16_t run;    // first gate of a sweep: gates in the sweep; 0 for the others
    int16_t nidx;   // noise gates: index among the list's noise gates
    int32_t gidx;   // index of the gate in the caller's list (passes may reorder commuting gates)
    double u[8];
};

// One pass: the tile qubit set and its slice [gate_begin, gate_begin +
// gate_count) of the plan's gates (execution order).
struct DPass {
    int tb;
    int nrest;
    uint8_t T[16];     // tile bit -> qubit (ascending)
    uint8_t rest[40];  // remaining bits -> qubit (ascending)
    int gate_begin, gate_count;
    u64 hi[16];        // state offset of tile index k * kTileThreads (its bits are tile bits >= 9)
};

inline int tile_bits_max(int dtype) { return dtype == QS_C128 ? 12 : 13; }

// Run-time compiled passes of a block plan (jit_block.hip).
struct JitFns {
    hipModule_t mod = nullptr;         // loaded on the plan's device; unloaded with the plan
    std::vector<hipFunction_t> fn;     // kernel of pass p: (C *psi, const R *vals, unsigned ntiles)
    std::vector<unsigned> max_blocks;  // per pass: resident workgroups on the device (persistent grid size)
    std::vector<unsigned> threads;     // per pass: workgroup size
};
// Tile sizes of compiled fused-block passes (make_plan's tile_bits and
// low_bits).  complex64: the interpreter's 13-bit tile.  complex128: 12-bit
// tiles (64 KiB of LDS, two 512-thread workgroups per CU, rows of 8 contiguous
// amplitudes) for passes over the lowest 12 qubits, 13-bit tiles (128 KiB,
// one 1024-thread workgroup per CU, rows of 16) for the others, from
// kJitMixedMinQubits qubits on.  Passes over high qubits gain from the longer
// rows, a pass over the low qubits (one contiguous 64 KiB stretch per tile)
// from the second workgroup.  Measured on the sweep (one-qubit gate on every
// qubit, CNOT chain) against 12-bit tiles throughout: 20 and 21 qubits 13 %
// and 7 % slower (too few 13-bit tiles to fill 256 CUs), 22-24 qubits 0-4 %
// faster, 26 1.5 % slower, 28 / 30 / 32 qubits 5.5 / 10 / 6 % faster.
// QSIM_JIT_TB=12 or 13 forces one size.
constexpr int kJitMixedMinQubits = 22;
void jit_tile_shape(int n, int dtype, int &tile_bits, int &low_bits);
int jit_threads(int dtype, int tile_bits);  // workgroup size of a compiled pass
// Source of the plan's pass kernels; "" when a pass's tile is not a size the
// generator supports (complex128: 12 or 13 bits, complex64: 13).
std::string jit_block_source(const std::vector<DPass> &passes, const std::vector<DGate> &dg, int dtype);
// Kernels of a plan: compiled once per source (host cache), loaded into a
// module of the caller's current device that the plan owns.  threads: the
// workgroup size of each pass (empty: kTileThreads for all).
int jit_block_functions(const std::string &src, int npass, int device, JitFns &out, const char *prefix = "qs_pass",
                        const std::vector<unsigned> &threads = {});
// Source of a trajectory plan's pass kernels (qs_tpass0, ...): per-trajectory
// gate values and control values from tables; "" when a pass's tile is not
// 12 bits.
std::string jit_traj_source(const std::vector<DPass> &passes, const std::vector<DGate> &dg, int dtype);
// The exact-value class of a gate that the generated code specialises on (a
// matrix equal to I or X, a diagonal matrix, diagonal entries equal to +-1).
int gate_value_class(int kind, const double *u);



// Greedy split of a gate list into passes.  A pass scans the remaining gates
// in list order and takes each one whose targets (1Q / noise target, C1Q
// target, both SWAP qubits) fit in a tile of tile_bits qubits (at most
// tile_bits_max(dtype)) that also holds the lowest qubits, provided it
// commutes with every gate it would overtake: those left for later passes.
// Gates on disjoint qubits commute, and so do two diagonal gates.  (Under a
// Pauli frame a diagonal gate stays diagonal, so trajectories may reorder the
// same way, each gate keeping the frame of its list position.)  This split is
// used when it has fewer passes than the plain one (each pass the longest
// fitting prefix of the list).  Diagonal gates and controls outside the tile
// ride along.  Each pass of at least 3 tile bits is then cut into sweeps (see
// DGate).
//
// cap > 0: passes that start among the first cap_region gates of the list
// hold at most cap gates (trajectories: shorter early passes let more noisy
// trajectories start late from the noiseless run's state).
//
// low_bits > 0 (below tile_bits): mixed tile sizes.  A pass first tries a tile
// of low_bits bits; if all of its targets then lie among the lowest low_bits
// qubits (one contiguous stretch of the state per tile) it keeps that tile,
// otherwise it is planned again with tile_bits.  DPass::tb gives each pass's size.
void make_plan(int n, int dtype, int tile_bits, const qs_gate *g, int count, std::vector<DPass> &passes, std::vector<DGate> &dg,
               int cap = 0, int cap_region = 0, int low_bits = 0);
// Passes of the plan qs_apply_block builds for this list (the compiled
// passes' tile sizes unless the interpreter is selected).
int block_pass_count(int n, int dtype, const qs_gate *g, int count);

// LDS tiles are stored swizzled: amplitude m of a tile sits at slot swz(m),
// the low 3 bits (the 16-byte slot within a 128-byte row) XORed with bits
// 3..5.  Any 8 consecutive lanes then touch 8 distinct slots of a row, also
// when each lane walks 8 consecutive amplitudes (a sweep over the lowest tile
// bits), which would otherwise put every lane of a b128 access on the same
// banks.  A bijection on [0, 2^tb) for every tb.
__device__ __forceinline__ u32 swz(u64 m) { return (u32)m ^ ((u32)(m >> 3) & 7u); }

template <typename R> __device__ __forceinline__ Mat2<R> load_mat(const double *u) {
    Mat2<R> m;
#pragma unroll
    for (int k = 0; k < 8; ++k) m.m[k] = (R)u[k];
    return m;
}

// Bit deposits through the pass's qubit maps.  The loops run over the
// arrays' full static length so that every entry is read at a fixed offset of
// the kernel argument (a hoisted scalar load, not a dependent memory access
// per bit).
__device__ __forceinline__ u64 pass_base(const DPass &P, u64 tile) {
    u64 base = 0;
#pragma unroll
    for (int b = 0; b < 40; ++b)
        if (b < P.nrest) base |= ((tile >> b) & 1ull) << P.rest[b];
    return base;
}

__device__ __forceinline__ u64 pass_off(const DPass &P, u64 m) {
    u64 off = 0;
#pragma unroll
    for (int b = 0; b < 16; ++b)
        if (b < P.tb) off |= ((m >> b) & 1ull) << P.T[b];
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
                cx<R> a = sh[swz(m0)], b = sh[swz(m1)];
                apply2<R>(m, a, b);
                sh[swz(m0)] = a;
                sh[swz(m1)] = b;
            }
        }
    } else if (kind == QS_G_C1Q) {
        const Mat2<R> m = load_mat<R>(u);
        const int lo = p0 < p1 ? p0 : p1, hi = p0 < p1 ? p1 : p0;
        const u64 cbit = cval ? (1ull << p0) : 0ull;
        for (u64 k = threadIdx.x; k < TS / 4; k += NT) {
            const u64 m0 = insert0(insert0(k, lo), hi) | cbit, m1 = m0 | (1ull << p1);
            cx<R> a = sh[swz(m0)], b = sh[swz(m1)];
            apply2<R>(m, a, b);
            sh[swz(m0)] = a;
            sh[swz(m1)] = b;
        }
    } else if (kind == QS_G_DIAG2) {
        cx<R> d[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            d[e].x = (R)u[2 * e];
            d[e].y = (R)u[2 * e + 1];
        }
        for (u64 mm = threadIdx.x; mm < TS; mm += NT) {
            const int b0 = p0 >= 0 ? (int)((mm >> p0) & 1) : (int)((base >> q0) & 1);
            const int b1 = p1 >= 0 ? (int)((mm >> p1) & 1) : (int)((base >> q1) & 1);
            const int e = 2 * b1 + b0;
            const cx<R> f = e == 0 ? d[0] : e == 1 ? d[1] : e == 2 ? d[2] : d[3];
            sh[swz(mm)] = cmul<R>(sh[swz(mm)], f);
        }
    } else if (kind == QS_G_SWAP) {
        const int lo = p0 < p1 ? p0 : p1, hi = p0 < p1 ? p1 : p0;
        for (u64 k = threadIdx.x; k < TS / 4; k += NT) {
            const u64 b = insert0(insert0(k, lo), hi);
            const u64 i = b | (1ull << p0), j = b | (1ull << p1);
            const cx<R> x = sh[swz(i)], y = sh[swz(j)];
            sh[swz(i)] = y;
            sh[swz(j)] = x;
        }
    }
    __syncthreads();
}

// Tile load / store: each thread issues all of its global accesses before it
// touches LDS (PER = 2^TBMAX / NT amplitudes per thread at most).  With
// `fill`, the tile is not read but set to the basis state |basis>.
template <typename R, int NT, int PER, bool NTEMP>
__device__ __forceinline__ void tile_load(cx<R> *sh, const cx<R> *psi, const DPass &P, u64 base, bool fill, u64 basis) {
    static_assert(NT == kTileThreads, "hi[] is laid out for kTileThreads");
    // m = thread + k NT: the deposit splits into a per-thread part and the
    // precomputed part hi[k] of the higher tile bits (disjoint bits).
    const u64 ot = base | pass_off(P, threadIdx.x);
    if (P.tb == 31 - __builtin_clz(PER * NT)) {  // a full tile: every slot is in range
        cx<R> v[PER];
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const u64 idx = ot | P.hi[k];
            if (fill) {
                v[k].x = idx == basis ? (R)1 : (R)0;
                v[k].y = (R)0;
            } else {
                v[k] = NTEMP ? __builtin_nontemporal_load(psi + idx) : psi[idx];
            }
        }
#pragma unroll
        for (int k = 0; k < PER; ++k) sh[swz(threadIdx.x + (u32)k * NT)] = v[k];
    } else {
        for (u32 m = threadIdx.x; m < (1u << P.tb); m += NT) {
            const u64 idx = base | pass_off(P, m);
            cx<R> v;
            if (fill) {
                v.x = idx == basis ? (R)1 : (R)0;
                v.y = (R)0;
            } else {
                v = psi[idx];
            }
            sh[swz(m)] = v;
        }
    }
}

template <typename R, int NT, int PER, bool NTEMP>
__device__ __forceinline__ void tile_store(const cx<R> *sh, cx<R> *psi, const DPass &P, u64 base) {
    if (P.tb == 31 - __builtin_clz(PER * NT)) {
        const u64 ot = base | pass_off(P, threadIdx.x);
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const cx<R> v = sh[swz(threadIdx.x + (u32)k * NT)];
            if (NTEMP)
                __builtin_nontemporal_store(v, psi + (ot | P.hi[k]));
            else
                psi[ot | P.hi[k]] = v;
        }
    } else {
        for (u32 m = threadIdx.x; m < (1u << P.tb); m += NT) psi[base | pass_off(P, m)] = sh[swz(m)];
    }
}

// ------------------------------------------------------------------ sweeps in registers

// Tile index of amplitude j (0..7) of a group whose slot bits are clear in m0.
__device__ __forceinline__ u32 grp_off(int j, int g0, int g1, int g2) {
    return ((u32)(j & 1) << g0) | ((u32)((j >> 1) & 1) << g1) | ((u32)((j >> 2) & 1) << g2);
}

template <typename R, int S> __device__ __forceinline__ void regs_2x2(cx<R> *v, const Mat2<R> &m) {
#pragma unroll
    for (int j = 0; j < 8; ++j)
        if (!((j >> S) & 1)) apply2<R>(m, v[j], v[j | (1 << S)]);
}

// Controlled: the pair (j, j | 1 << S) changes iff the control bit of its
// tile index equals cval (both members share the control bit).
template <typename R, int S>
__device__ __forceinline__ void regs_c2x2(cx<R> *v, const Mat2<R> &m, u32 m0, int g0, int g1, int g2, int pc, int cval) {
#pragma unroll
    for (int j = 0; j < 8; ++j)
        if (!((j >> S) & 1))
            if ((int)(((m0 | grp_off(j, g0, g1, g2)) >> pc) & 1u) == cval) apply2<R>(m, v[j], v[j | (1 << S)]);
}

template <typename R> __device__ __forceinline__ void swap2(cx<R> &a, cx<R> &b) {
    const cx<R> t = a;
    a = b;
    b = t;
}

// The 2x2 matrix (1Q, C1Q) or the 4 diagonal entries (DIAG2) of a gate.
template <typename R> struct GateVals {
    Mat2<R> m;
    cx<R> d[4];
};

template <typename R> __device__ __forceinline__ GateVals<R> gate_vals(int kind, const double *u) {
    GateVals<R> gv;
#pragma unroll
    for (int k = 0; k < 8; ++k) gv.m.m[k] = (R)u[k];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        gv.d[e].x = (R)u[2 * e];
        gv.d[e].y = (R)u[2 * e + 1];
    }
    return gv;
}

// One gate of a sweep on one group.  base: the pass's fixed bits (for qubits
// outside the tile).
// dv: the gate's four diagonal entries in LDS (DIAG2), read with a per-lane
// index.
template <typename R>
__device__ __forceinline__ void regs_apply_gate(cx<R> *v, u32 m0, int g0, int g1, int g2, u64 base, int kind, int p0, int p1, int q0,
                                                int q1, int s0, int s1, int cval, const GateVals<R> &gv, const cx<R> *dv) {
    const Mat2<R> &m = gv.m;
    if (kind == QS_G_1Q || (kind == QS_G_C1Q && p0 < 0)) {
        if (kind == QS_G_C1Q && (int)((base >> q0) & 1ull) != cval) return;
        const int S = kind == QS_G_1Q ? s0 : s1;
        if (S == 0) regs_2x2<R, 0>(v, m);
        else if (S == 1) regs_2x2<R, 1>(v, m);
        else regs_2x2<R, 2>(v, m);
    } else if (kind == QS_G_C1Q) {
        if (s1 == 0) regs_c2x2<R, 0>(v, m, m0, g0, g1, g2, p0, cval);
        else if (s1 == 1) regs_c2x2<R, 1>(v, m, m0, g0, g1, g2, p0, cval);
        else regs_c2x2<R, 2>(v, m, m0, g0, g1, g2, p0, cval);
    } else if (kind == QS_G_DIAG2) {
        // Entry d[2 b1 + b0] comes from LDS with a per-lane index instead of a
        // select over the four entries.  A qubit outside the tile contributes
        // the pass's fixed bit, parked on bit 31 / 30 of the index (tile
        // indices stay below 2^13).
        const int P0 = p0 < 0 ? 31 : p0, P1 = p1 < 0 ? 30 : p1;
        const u32 X = (p0 < 0 ? (u32)((base >> q0) & 1ull) << 31 : 0u) | (p1 < 0 ? (u32)((base >> q1) & 1ull) << 30 : 0u);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const u32 idx = m0 | grp_off(j, g0, g1, g2) | X;
            const u32 e = ((idx >> P0) & 1u) | (((idx >> P1) & 1u) << 1);
            v[j] = cmul<R>(v[j], dv[e]);
        }
    } else if (kind == QS_G_SWAP) {
        const int a = s0 < s1 ? s0 : s1, b = s0 < s1 ? s1 : s0;
        if (a == 0 && b == 1) { swap2<R>(v[1], v[2]); swap2<R>(v[5], v[6]); }
        else if (a == 0) { swap2<R>(v[1], v[4]); swap2<R>(v[3], v[6]); }
        else { swap2<R>(v[2], v[4]); swap2<R>(v[3], v[5]); }
    }
}

// A gate staged in LDS, ready to apply: kind 0 = skip; val = the 2x2 matrix
// (1Q, C1Q) or the 4 diagonal entries (DIAG2), interleaved (re, im).
// The header is one 16-byte word and the values whole 16-byte vectors, so a
// gate is read with a few wide LDS reads rather than one read per field:
//   h.x = kind | p0 << 8 | p1 << 16 | q0 << 24,  h.y = q1 | s0 << 8 | s1 << 16 | cval << 24,
//   h.z = g0 | g1 << 8 | g2 << 16,               h.w = run   (fields as signed bytes).
template <typename R> struct alignas(16) SGate {
    uint4 h;
    R val[8];
};

__device__ __forceinline__ int sbyte(uint32_t w, int k) { return (int)(int8_t)(uint8_t)(w >> (8 * k)); }

// A staged header is the same in every lane (all lanes read one LDS address);
// moving it to scalar registers lets the compiler branch on the gate kind and
// bit positions with scalar branches instead of per-lane masks and selects.
__device__ __forceinline__ uint4 uniform_header(uint4 h) {
    h.x = __builtin_amdgcn_readfirstlane(h.x);
    h.y = __builtin_amdgcn_readfirstlane(h.y);
    h.z = __builtin_amdgcn_readfirstlane(h.z);
    h.w = __builtin_amdgcn_readfirstlane(h.w);
    return h;
}

// Gates are staged in LDS this many at a time (and sweeps hold at most this
// many gates), so their parameters are fetched by all threads at once rather
// than one dependent global load per gate.
constexpr int kStage = 64;

// Sweeps of one pass on the LDS tile `sh` (2^tb amplitudes, fixed bits
// `base`), block size NT, at most GMAX groups of 8 per thread.
// prep(gidx, gate, vals, cval, kind) fills a gate's values (gidx: its list
// index) and may skip it
// (return false) or change its kind / control value.
template <typename R, int NT, int GMAX, typename Prep>
__device__ __forceinline__ void run_sweeps(cx<R> *sh, SGate<R> *sg, int tb, u64 base, const DGate *__restrict__ gates, int begin, int count,
                                           Prep prep) {
    const u32 groups = 1u << (tb - 3);
    int cb = 0, ce = 0;
    auto stage = [&](int at) {
        const int cnt = count - at < kStage ? count - at : kStage;
        __syncthreads();  // every thread is done with the previous chunk
        if ((int)threadIdx.x < cnt) {
            const DGate &x = gates[begin + at + threadIdx.x];
            GateVals<R> gv;
            int cval = 1, kind = x.kind;
            if (!prep(x.gidx, x, gv, cval, kind)) kind = 0;
            SGate<R> o;
            auto byte = [](int v) { return (uint32_t)(uint8_t)(int8_t)v; };
            o.h.x = byte(kind) | byte(x.p0) << 8 | byte(x.p1) << 16 | byte(x.q0) << 24;
            o.h.y = byte(x.q1) | byte(x.s0) << 8 | byte(x.s1) << 16 | byte(cval) << 24;
            o.h.z = byte(x.g[0]) | byte(x.g[1]) << 8 | byte(x.g[2]) << 16;
            o.h.w = (uint32_t)x.run;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const cx<R> d = gv.d[e];
                o.val[2 * e] = kind == QS_G_DIAG2 ? d.x : gv.m.m[2 * e];
                o.val[2 * e + 1] = kind == QS_G_DIAG2 ? d.y : gv.m.m[2 * e + 1];
            }
            sg[threadIdx.x] = o;
        }
        cb = at;
        ce = at + cnt;
        __syncthreads();
    };
    int gi = 0;
    while (gi < count) {
        if (gi >= ce) stage(gi);
        if (gi + (int)__builtin_amdgcn_readfirstlane(sg[gi - cb].h.w) > ce) stage(gi);
        const uint4 hh = uniform_header(sg[gi - cb].h);
        const int run = (int)hh.w, g0 = sbyte(hh.z, 0), g1 = sbyte(hh.z, 1), g2 = sbyte(hh.z, 2);
        cx<R> v[GMAX][8];
        u32 m0[GMAX];
#pragma unroll
        for (int k = 0; k < GMAX; ++k) {
            const u32 grp = threadIdx.x + (u32)k * NT;
            m0[k] = (u32)insert0(insert0(insert0(grp, g0), g1), g2);
            if (grp < groups) {
#pragma unroll
                for (int j = 0; j < 8; ++j) v[k][j] = sh[swz(m0[k] | grp_off(j, g0, g1, g2))];
            }
        }
        for (int r = 0; r < run; ++r) {
            const SGate<R> &x = sg[gi - cb + r];
            const uint4 h = uniform_header(x.h);
            cx<R> val[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) val[e] = reinterpret_cast<const cx<R> *>(x.val)[e];
            const int kind = sbyte(h.x, 0);  // 0 (a skipped gate) matches no branch below
            GateVals<R> gv;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                gv.m.m[2 * e] = val[e].x;
                gv.m.m[2 * e + 1] = val[e].y;
                gv.d[e] = val[e];
            }
#pragma unroll
            for (int k = 0; k < GMAX; ++k)
                if (threadIdx.x + (u32)k * NT < groups)
                    regs_apply_gate<R>(v[k], m0[k], g0, g1, g2, base, kind, sbyte(h.x, 1), sbyte(h.x, 2), sbyte(h.x, 3), sbyte(h.y, 0),
                                       sbyte(h.y, 1), sbyte(h.y, 2), sbyte(h.y, 3), gv, reinterpret_cast<const cx<R> *>(x.val));
        }
#pragma unroll
        for (int k = 0; k < GMAX; ++k) {
            if (threadIdx.x + (u32)k * NT < groups) {
#pragma unroll
                for (int j = 0; j < 8; ++j) sh[swz(m0[k] | grp_off(j, g0, g1, g2))] = v[k][j];
            }
        }
        __syncthreads();
        gi += run;
    }
}

}  // namespace qs
