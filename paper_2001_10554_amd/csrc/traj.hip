// Noise trajectories: stochastic Pauli insertion (depolarizing channel)
// averaged over an ensemble of pure-state runs.
//
// Pauli frames.  An inserted Pauli is not applied to the amplitudes.  Each
// trajectory keeps a frame F = X^a Z^b (n-bit masks a, b; global phases are
// irrelevant to every read-out) with psi_true = F psi_stored.  A gate G then
// acts on the stored state as F^dagger G F:
//   1Q U on q:        U' = P^dagger U P with P = X^{a_q} Z^{b_q};
//   C1Q (c, t, U):    control value 1 xor a_c, target matrix conjugated as above;
//   DIAG2 (q0, q1):   entries permuted by the X part on q0 / q1;
//   SWAP (x, y):      applied as is, and the frame's bits x and y are exchanged.
// An insertion of X, Y or Z on q flips a_q, a_q and b_q, or b_q.  So every
// trajectory runs the same fused pass schedule as the noiseless circuit and an
// insertion costs no extra pass.  Read-outs undo the frame:
//   <Z_q> = (-1)^{a_q} <Z_q>_stored, <X_q> = (-1)^{b_q} <X_q>_stored,
//   p(k) = |psi_stored(k xor a)|^2,
//   <ideal|psi> = sum_j conj(ideal(j xor a)) (-1)^{popc(b & j)} psi_stored(j).
//
// Draws.  Draw `slot` of trajectory t is Philox4x32-10(key = seed, counter =
// (t, slot, 3, 0)); after each gate one draw per touched qubit (q0, then q1);
// insert iff x0 < floor(p 2^32); Pauli = 1 + floor(3 x1 / 2^32).  The frames
// kernel replays these integer decisions once per trajectory and stores the
// frame seen by every gate, so the decisions are bit-exact by construction.
#include <algorithm>
#include <cmath>
#include <cstddef>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "launch.h"
#include "tile.h"
#include "vec.h"

#define QS_API extern "C" __attribute__((visibility("default")))

namespace qs {

constexpr int kTrajMaxQubits = 20;
constexpr int kTrajMaxGates = 4096;

struct TGate {  // gate list on the device (kind, q0, q1, u)
    int32_t kind, q0, q1, pad;
    double u[8];
};
static_assert(sizeof(TGate) == sizeof(qs_gate), "TGate mirrors qs_gate");
static_assert(kTrajMaxGates % 8 == 0, "the frames kernel reads gate records in groups of eight");
static_assert(2 * kTrajMaxGates <= 0xffff, "draw slots and execution positions share a 32-bit field");

// SWAP gates at the end of the list only relabel qubits, so they are not
// simulated: the read-outs see them instead.  With S their product, the true
// state is S psi', psi' the simulated one: bit p of a true index is bit src[p]
// of the simulated index, and the final frame F is carried back as
// S^dagger F S (X_p -> X_src[p]).  active = 0: no trailing SWAPs.
struct QPerm {
    uint8_t src[kTrajMaxQubits];
    int active;
};
// Simulated index -> true index.
__device__ __forceinline__ u64 perm_index(const QPerm &P, int n, u64 k) {
    u64 r = 0;
    for (int p = 0; p < n; ++p) r |= ((k >> P.src[p]) & 1ull) << p;
    return r;
}
// A frame mask in true qubit labels -> simulated labels.
__device__ __forceinline__ u32 perm_mask(const QPerm &P, int n, u32 m) {
    u32 r = 0;
    for (int p = 0; p < n; ++p) r |= ((m >> p) & 1u) << P.src[p];
    return r;
}

// frames[t * count + g] = (a | b << 32) before gate g; final[t] after all gates;
// counts[t] = number of insertions.  first[t] = the earliest execution
// position (index into the plan's gate order) of a gate that sees a
// non-identity frame (count if none): the trajectory equals the noiseless run
// before that position.  nins_ws[t] > 0 marks a trajectory simulated on its own:
// one with a gate after its first insertion (insertions after the last gate
// only change the frame the read-outs undo), or every noisy trajectory with
// force_all (noise gates make each trajectory's state differ even without
// insertions; first[t] = 0 then).
//
// One wavefront per trajectory (t = n_traj is the extra noiseless one): its
// lanes make the draws of all gates at once and keep one decision byte per
// gate in LDS (bits 0-1: the Pauli drawn for q0, 2-3: for q1, 0 = none;
// gates[g].pad holds the gate's first slot in its low 16 bits and its
// execution position in the high 16); lane 0 then replays the gates in
// order, eight records at a time, which fixes the frames, the insertion log
// and the first affected gate.
constexpr int kFrameWaves = 4;
__global__ __launch_bounds__(64 * kFrameWaves) void k_traj_frames(const TGate *__restrict__ gates, int count, int n_traj, u32 thr, u32 k0,
                                                                   u32 k1, uint64_t *__restrict__ frames, uint64_t *__restrict__ final_frame,
                                                                   int32_t *__restrict__ nins_ws, int32_t *__restrict__ first,
                                                                   int32_t *__restrict__ counts, uint32_t *__restrict__ log, int log_cap,
                                                                   int force_all, QPerm perm, int n) {
    __shared__ uint32_t hdr[kTrajMaxGates];  // kind | q0 << 8 | q1 << 16
    __shared__ uint16_t epos[kTrajMaxGates];
    __shared__ uint8_t dec[kFrameWaves][kTrajMaxGates];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int t = blockIdx.x * kFrameWaves + w;
    const bool ideal = t == n_traj;
    for (int g = threadIdx.x; g < count; g += blockDim.x) {
        hdr[g] = ((u32)gates[g].kind & 0xffu) | ((u32)gates[g].q0 & 0xffu) << 8 | ((u32)gates[g].q1 & 0xffu) << 16;
        epos[g] = (uint16_t)((u32)gates[g].pad >> 16);
    }
    if (t <= n_traj)
        for (int g = lane; g < count; g += 64) {
            const int kind = gates[g].kind;
            const int nt = kind == QS_G_NOISE ? 0 : kind == QS_G_1Q ? 1 : 2;
            const u32 s0 = (u32)gates[g].pad & 0xffffu;
            u32 d = 0;
            for (int k = 0; k < nt && !ideal; ++k) {
                const Philox4 r = philox4x32_10((u32)t, s0 + (u32)k, kTagTraj, 0u, k0, k1);
                if (r.v[0] < thr) d |= (1u + (u32)(((u64)r.v[1] * 3u) >> 32)) << (2 * k);
            }
            dec[w][g] = (uint8_t)d;
        }
    __syncthreads();
    if (t > n_traj || lane != 0) return;
    const uint8_t *D = dec[w];
    uint64_t *fr = frames + (u64)t * count;
    u32 a = 0, b = 0;
    int nins = 0, e1 = count;
    constexpr int kU = 8;  // kTrajMaxGates is a multiple: the records read past count stay inside the arrays
    for (int g0 = 0; g0 < count; g0 += kU) {
        u32 H[kU], Dg[kU], Ep[kU];
#pragma unroll
        for (int j = 0; j < kU; ++j) {
            H[j] = hdr[g0 + j];
            Dg[j] = D[g0 + j];
            Ep[j] = epos[g0 + j];
        }
#pragma unroll
        for (int j = 0; j < kU; ++j) {
            const int g = g0 + j;
            if (g >= count) break;
            fr[g] = (u64)a | ((u64)b << 32);
            if ((a | b) && (int)Ep[j] < e1) e1 = (int)Ep[j];
            const u32 q0 = (H[j] >> 8) & 0xffu, q1 = H[j] >> 16;
            const u32 x = 1u << q0, y = 1u << (q1 & 31u);
            if ((H[j] & 0xffu) == (u32)QS_G_SWAP) {
                if (((a & x) != 0) != ((a & y) != 0)) a ^= x | y;
                if (((b & x) != 0) != ((b & y) != 0)) b ^= x | y;
            }
            const u32 d0 = Dg[j] & 3u, d1 = Dg[j] >> 2;
            a ^= (d0 == 1u || d0 == 2u ? x : 0u) ^ (d1 == 1u || d1 == 2u ? y : 0u);
            b ^= (d0 == 2u || d0 == 3u ? x : 0u) ^ (d1 == 2u || d1 == 3u ? y : 0u);
            if (Dg[j]) {  // rare: log in slot order
                const u32 s0 = (u32)gates[g].pad & 0xffffu;
                if (d0) {
                    if (log && nins < log_cap) log[(u64)t * log_cap + nins] = (s0 << 2) | d0;
                    ++nins;
                }
                if (d1) {
                    if (log && nins < log_cap) log[(u64)t * log_cap + nins] = ((s0 + 1u) << 2) | d1;
                    ++nins;
                }
            }
        }
    }
    if (perm.active) {
        a = perm_mask(perm, n, a);
        b = perm_mask(perm, n, b);
    }
    final_frame[t] = (u64)a | ((u64)b << 32);
    const bool own = force_all ? !ideal : e1 < count;
    nins_ws[t] = own ? nins + 1 : 0;
    first[t] = force_all ? 0 : e1;
    if (counts && !ideal) counts[t] = nins;
}

// A trajectory without insertions has exactly the noiseless state: only the
// noisy trajectories and the noiseless run itself (t = n_traj) are simulated,
// the others read the noiseless run's state and read-outs.
__device__ __forceinline__ bool traj_simulated(const int32_t *nins, u64 t, int n_traj) { return t == (u64)n_traj || nins[t] > 0; }
__device__ __forceinline__ u64 traj_rep(const int32_t *nins, u64 t, int n_traj) { return nins[t] > 0 ? t : (u64)n_traj; }

// u <- w u (2x2 complex, row-major interleaved).
__device__ __forceinline__ void mat2_mul(const double *w, double *u) {
    double r[8];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            double re = 0.0, im = 0.0;
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const double wr = w[(2 * i + k) * 2], wi = w[(2 * i + k) * 2 + 1];
                const double ur = u[(2 * k + j) * 2], ui = u[(2 * k + j) * 2 + 1];
                re += wr * ur - wi * ui;
                im += wr * ui + wi * ur;
            }
            r[(2 * i + j) * 2] = re;
            r[(2 * i + j) * 2 + 1] = im;
        }
#pragma unroll
    for (int k = 0; k < 8; ++k) u[k] = r[k];
}

// U' = P^dagger U P for P = X^xa Z^zb (row-major interleaved u[8]).
__device__ __forceinline__ void conj_pauli(double *u, int xa, int zb) {
    if (xa) {  // X U X: swap rows and columns
        double t[8];
        for (int k = 0; k < 8; ++k) t[k] = u[k];
        u[0] = t[6]; u[1] = t[7]; u[2] = t[4]; u[3] = t[5];
        u[4] = t[2]; u[5] = t[3]; u[6] = t[0]; u[7] = t[1];
    }
    if (zb) {  // Z U Z: negate the off-diagonal
        u[2] = -u[2]; u[3] = -u[3]; u[4] = -u[4]; u[5] = -u[5];
    }
}

// Noise gate of duration d for trajectory t, gate index gidx: the composed
// rotation R_Z(a_z) R_Y(a_y) R_X(a_x) with Box-Muller normals from Philox
// (key = seed, counter = (t, gidx, 7, w)), angle variances d/T1, d/T1 and
// 2d/T2 - d/T1.
constexpr u32 kTagNoise = 7;
__device__ __forceinline__ void noise_matrix(double *u, double d, double inv_T1, double inv_T2, u32 t, u32 gidx, u32 k0, u32 k1) {
    const double two_pi = 6.283185307179586476925286766559;
    const Philox4 x0 = philox4x32_10(t, gidx, kTagNoise, 0u, k0, k1);
    const Philox4 x1 = philox4x32_10(t, gidx, kTagNoise, 1u, k0, k1);
    const double r0 = sqrt(-2.0 * log(1.0 - u53(x0.v[0], x0.v[1]))), t0 = two_pi * u53(x0.v[2], x0.v[3]);
    const double r1 = sqrt(-2.0 * log(1.0 - u53(x1.v[0], x1.v[1]))), t1 = two_pi * u53(x1.v[2], x1.v[3]);
    const double vxy = d * inv_T1, vz = 2.0 * d * inv_T2 - d * inv_T1;
    const double ax = sqrt(vxy) * (r0 * cos(t0)), ay = sqrt(vxy) * (r0 * sin(t0)), az = sqrt(vz > 0.0 ? vz : 0.0) * (r1 * cos(t1));
    const double cx = cos(0.5 * ax), sx = sin(0.5 * ax), cy = cos(0.5 * ay), sy = sin(0.5 * ay), cz = cos(0.5 * az), sz = sin(0.5 * az);
    // Y X = [[cy, -sy], [sy, cy]] [[cx, -i sx], [-i sx, cx]]
    const double m00r = cy * cx, m00i = sy * sx, m01r = -sy * cx, m01i = -cy * sx;
    const double m10r = sy * cx, m10i = -cy * sx, m11r = cy * cx, m11i = -sy * sx;
    // Z (Y X): row 0 times e^{-i az/2}, row 1 times e^{+i az/2}
    u[0] = cz * m00r + sz * m00i; u[1] = cz * m00i - sz * m00r;
    u[2] = cz * m01r + sz * m01i; u[3] = cz * m01i - sz * m01r;
    u[4] = cz * m10r - sz * m10i; u[5] = cz * m10i + sz * m10r;
    u[6] = cz * m11r - sz * m11i; u[7] = cz * m11i + sz * m11r;
}

// Noise matrices of every (noisy trajectory, noise gate), computed once:
// nm[(t * nnoise + nidx) * 8].
__global__ void k_traj_noise_mats(const DGate *__restrict__ gates, int count, int n_traj, int nnoise, u32 k0, u32 k1, double inv_T1,
                                  double inv_T2, double *__restrict__ nm) {
    const u64 id = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (u64)n_traj * count) return;
    const u32 t = (u32)(id / count);
    const DGate &g = gates[id % count];
    if (g.kind != QS_G_NOISE) return;
    double u[8];
    noise_matrix(u, g.u[0], inv_T1, inv_T2, t, (u32)g.gidx, k0, k1);
    double *o = nm + ((u64)t * nnoise + g.nidx) * 8;
#pragma unroll
    for (int k = 0; k < 8; ++k) o[k] = u[k];
}

// Per (simulated trajectory, plan gate): the gate as the compiled passes apply
// it, F^dagger G F for the trajectory's frame F before the gate (the same
// values the interpreter's staging computes): tv[(t * ngates + i) * 8 + k]
// the 2x2 matrix (1Q, C1Q, noise) or the 4 diagonal entries (DIAG2), tc the
// control value a C1Q gate fires on.  Noise gates of the noiseless run are the
// identity; a one-qubit gate followed by a noise gate on its qubit takes that
// gate's matrix into its own.
template <typename R>
__global__ void k_traj_vals(const DGate *__restrict__ gates, int ngates, const uint64_t *__restrict__ frames, int count,
                            const int32_t *__restrict__ nins, int n_traj, const double *__restrict__ nm, int nnoise, R *__restrict__ tv,
                            int32_t *__restrict__ tc) {
    const u64 id = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (u64)(n_traj + 1) * ngates) return;
    const u64 t = id / ngates;
    const int i = (int)(id % ngates);
    if (!traj_simulated(nins, t, n_traj)) return;
    const bool ideal = t == (u64)n_traj;
    const DGate &g = gates[i];
    const u64 f = frames[t * count + g.gidx];
    const u32 a = (u32)f, b = (u32)(f >> 32);
    double u[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) u[k] = g.u[k];
    int cval = 1;
    if (g.kind == QS_G_NOISE) {
        if (ideal || g.pad0 == 2) {
            const double id2[8] = {1, 0, 0, 0, 0, 0, 1, 0};
#pragma unroll
            for (int k = 0; k < 8; ++k) u[k] = id2[k];
        } else {
            const double *src = nm + ((u64)t * nnoise + g.nidx) * 8;
#pragma unroll
            for (int k = 0; k < 8; ++k) u[k] = src[k];
            conj_pauli(u, (a >> g.q0) & 1, (b >> g.q0) & 1);
        }
    } else if (g.kind == QS_G_1Q) {
        conj_pauli(u, (a >> g.q0) & 1, (b >> g.q0) & 1);
        if (g.pad0 == 1 && !ideal) {
            const DGate &nx = gates[i + 1];
            const u64 f2 = frames[t * count + nx.gidx];
            const double *src = nm + ((u64)t * nnoise + nx.nidx) * 8;
            double w[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) w[k] = src[k];
            conj_pauli(w, ((u32)f2 >> g.q0) & 1, ((u32)(f2 >> 32) >> g.q0) & 1);
            mat2_mul(w, u);
        }
    } else if (g.kind == QS_G_C1Q) {
        cval = 1 ^ (int)((a >> g.q0) & 1);
        conj_pauli(u, (a >> g.q1) & 1, (b >> g.q1) & 1);
    } else if (g.kind == QS_G_DIAG2) {  // entries permuted by the frame's X part on q0 / q1
        auto sw = [&](int e0, int e1) {
            const double r = u[2 * e0], m = u[2 * e0 + 1];
            u[2 * e0] = u[2 * e1];
            u[2 * e0 + 1] = u[2 * e1 + 1];
            u[2 * e1] = r;
            u[2 * e1 + 1] = m;
        };
        if ((a >> g.q0) & 1) {
            sw(0, 1);
            sw(2, 3);
        }
        if ((a >> g.q1) & 1) {
            sw(0, 2);
            sw(1, 3);
        }
    }
    R *o = tv + id * 8;
#pragma unroll
    for (int k = 0; k < 8; ++k) o[k] = (R)u[k];
    tc[id] = cval;
}

// One pass of every simulated trajectory: block = (trajectory, tile).  Gates
// act on the stored state as F^dagger G F for the trajectory's frame F before
// the gate; sweeps of gates run in registers (see DGate).
// Noiseless run: reads ideal_in (the previous pass's output) and writes
// ideal_out (two buffers used in turn, the last pass writing its own state
// slot), so that a trajectory whose first non-identity frame falls in this
// pass can start from ideal_in while the noiseless run updates its state.
// Trajectories whose first such gate lies beyond this pass skip it (their
// state still equals the noiseless one).  first_pass: the input is |basis>.
template <typename R, int TBMAX>
__global__ __launch_bounds__(kTileThreads) void k_traj_pass(cx<R> *__restrict__ states, u64 N, int tiles_log2, DPass P, const DGate *__restrict__ gates,
                                                      const uint64_t *__restrict__ frames, int count, int first_pass, u64 basis,
                                                      const int32_t *__restrict__ nins, const int32_t *__restrict__ first, int n_traj,
                                                      const double *__restrict__ nm, int nnoise, const cx<R> *ideal_in, cx<R> *ideal_out) {
    __shared__ cx<R> sh[1 << TBMAX];
    __shared__ SGate<R> sg[kStage];
    const u64 tile = blockIdx.x & ((1ull << tiles_log2) - 1);
    const u64 t = blockIdx.x >> tiles_log2;
    if (!traj_simulated(nins, t, n_traj)) return;  // whole block: shares the noiseless state
    const bool ideal = t == (u64)n_traj;
    const int g1 = ideal ? 0 : first[t];
    if (!ideal && g1 >= P.gate_begin + P.gate_count) return;  // still the noiseless state after this pass
    const bool from_ideal = ideal || g1 >= P.gate_begin;       // first pass that differs: start from the noiseless run
    constexpr int NT = kTileThreads, PER = (1 << TBMAX) / NT;
    cx<R> *psi = ideal ? ideal_out : states + t * N;
    const cx<R> *src = from_ideal ? ideal_in : psi;
    const u64 TS = 1ull << P.tb;
    const u64 base = pass_base(P, tile);
    tile_load<R, NT, PER, true>(sh, src, P, base, from_ideal && first_pass != 0, basis);
    __syncthreads();
    auto prep = [&](int gidx, const DGate &g, GateVals<R> &gv, int &cval, int &kind) -> bool {
        const u64 f = frames[t * count + gidx];
        const u32 a = (u32)f, b = (u32)(f >> 32);
        double u[8];
        if (kind == QS_G_NOISE) {
            if (ideal || g.pad0 == 2) return false;  // the noiseless reference run / folded into the gate before
            const double *src = nm + ((u64)t * nnoise + g.nidx) * 8;
#pragma unroll
            for (int k = 0; k < 8; ++k) u[k] = src[k];
            conj_pauli(u, (a >> g.q0) & 1, (b >> g.q0) & 1);
            kind = QS_G_1Q;
        } else {
#pragma unroll
            for (int k = 0; k < 8; ++k) u[k] = g.u[k];
            if (kind == QS_G_1Q) {
                conj_pauli(u, (a >> g.q0) & 1, (b >> g.q0) & 1);
                if (g.pad0 == 1 && !ideal) {
                    // The next gate (execution order) is a noise gate on the same
                    // qubit: apply both as one matrix, each conjugated by its own frame.
                    const DGate &nx = (&g)[1];
                    const u64 f2 = frames[t * count + nx.gidx];
                    const double *src = nm + ((u64)t * nnoise + nx.nidx) * 8;
                    double w[8];
#pragma unroll
                    for (int k = 0; k < 8; ++k) w[k] = src[k];
                    conj_pauli(w, ((u32)f2 >> g.q0) & 1, ((u32)(f2 >> 32) >> g.q0) & 1);
                    mat2_mul(w, u);
                }
            } else if (kind == QS_G_C1Q) {
                cval = 1 ^ (int)((a >> g.q0) & 1);
                conj_pauli(u, (a >> g.q1) & 1, (b >> g.q1) & 1);
            }
        }
        gv = gate_vals<R>(kind, u);
        if (kind == QS_G_DIAG2) {  // entries permuted by the frame's X part on q0 / q1
            if ((a >> g.q0) & 1) {
                swap2<R>(gv.d[0], gv.d[1]);
                swap2<R>(gv.d[2], gv.d[3]);
            }
            if ((a >> g.q1) & 1) {
                swap2<R>(gv.d[0], gv.d[2]);
                swap2<R>(gv.d[1], gv.d[3]);
            }
        }
        return true;
    };
    if (P.tb >= 3) {
        run_sweeps<R, NT, ((1 << (TBMAX - 3)) + NT - 1) / NT>(sh, sg, P.tb, base, gates, P.gate_begin, P.gate_count, prep);
    } else {
        for (int gi = 0; gi < P.gate_count; ++gi) {
            const DGate &g = gates[P.gate_begin + gi];
            GateVals<R> gv;
            int cval = 1, kind = g.kind;
            if (!prep(g.gidx, g, gv, cval, kind)) continue;
            double u[8];
            if (kind == QS_G_DIAG2) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    u[2 * e] = (double)gv.d[e].x;
                    u[2 * e + 1] = (double)gv.d[e].y;
                }
            } else {
#pragma unroll
                for (int k = 0; k < 8; ++k) u[k] = (double)gv.m.m[k];
            }
            lds_apply_gate<R, NT>(sh, TS, base, kind, g.p0, g.p1, g.q0, g.q1, cval, u);
        }
    }
    tile_store<R, NT, PER, true>(sh, psi, P, base);
}

__device__ __forceinline__ double tblock_sum(double v, double *red) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    return red[0] + red[1] + red[2] + red[3];
}

// Per simulated trajectory and chunk of amplitudes: [0, n) = sum (-1)^{k_q}
// |psi_k|^2, (n, n+1) = <ideal|F psi> (re, im) and n+2 = sum_k d_k |(F psi)_k|^2
// for a diagonal observable d.  The chunk's index bits
// below log2(256) are fixed per thread, the others per loop step, so each
// <Z_q> needs one add per amplitude only for the q the loop varies.
// FID false: no fidelity asked for, so the noiseless state is not read.
template <typename R, bool FID>
__global__ __launch_bounds__(kBlock) void k_traj_zf(const cx<R> *__restrict__ states, int n, int chunk_log2, int chunks_log2,
                                                    const uint64_t *__restrict__ final_frame, const int32_t *__restrict__ nins, int n_traj,
                                                    const double *__restrict__ diag, double *__restrict__ partial, QPerm perm) {
    __shared__ double red[kBlock / 64];
    const u64 N = 1ull << n;
    const u64 c = blockIdx.x & ((1ull << chunks_log2) - 1);
    const u64 t = blockIdx.x >> chunks_log2;
    // A trajectory not simulated on its own but with a non-identity final
    // frame (all its insertions after the last simulated gate) reads the
    // noiseless state; its fidelity and diagonal observable still depend on
    // its frame, so it gets partials of its own.
    if (!traj_simulated(nins, t, n_traj) && final_frame[t] == 0) return;
    const cx<R> *psi = states + traj_rep(nins, t, n_traj) * N;
    const cx<R> *ideal = states + (u64)n_traj * N;
    const u64 f = final_frame[t];
    const u32 fa = (u32)f, fb = (u32)(f >> 32);
    double z[kTrajMaxQubits], fre = 0.0, fim = 0.0, dsum = 0.0;
#pragma unroll
    for (int q = 0; q < kTrajMaxQubits; ++q) z[q] = 0.0;
    const u64 lo = c << chunk_log2, hi = lo + (1ull << chunk_log2);
    auto step = [&](u64 i, cx<R> v, cx<R> id, double dg) {
        const double p = (double)v.x * v.x + (double)v.y * v.y;
#pragma unroll
        for (int q = 0; q < kTrajMaxQubits; ++q) z[q] += ((i >> q) & 1) ? -p : p;
        if (FID) {
            const double sgn = (__popcll(i & fb) & 1) ? -1.0 : 1.0;
            fre += sgn * ((double)id.x * v.x + (double)id.y * v.y);
            fim += sgn * ((double)id.x * v.y - (double)id.y * v.x);
        }
        dsum += p * dg;
    };
    u64 i = lo + threadIdx.x;
    for (; i + 3 * kBlock < hi; i += 4 * kBlock) {  // four steps, loads first; same summation order
        cx<R> v[4], id[4]{};
        double dg[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const u64 k = i + (u64)s * kBlock;
            v[s] = psi[k];
            if (FID) id[s] = ideal[k ^ fa];
            dg[s] = diag ? diag[perm.active ? perm_index(perm, n, k ^ fa) : k ^ fa] : 0.0;
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) step(i + (u64)s * kBlock, v[s], id[s], dg[s]);
    }
    for (; i < hi; i += kBlock) step(i, psi[i], FID ? ideal[i ^ fa] : cx<R>{}, diag ? diag[perm.active ? perm_index(perm, n, i ^ fa) : i ^ fa] : 0.0);
    const int nv = n + 3;
    double *out = partial + (u64)blockIdx.x * nv;
#pragma unroll
    for (int q = 0; q < kTrajMaxQubits; ++q) {
        const double s = tblock_sum(z[q], red);
        if (threadIdx.x == 0 && q < n) out[q] = s;
    }
    const double tre = tblock_sum(fre, red);
    const double tim = tblock_sum(fim, red);
    const double tds = tblock_sum(dsum, red);
    if (threadIdx.x == 0) {
        out[n] = tre;
        out[n + 1] = tim;
        out[n + 2] = tds;
    }
}

// <X_q>_stored partials: block (t, q, chunk) sums 2 Re(conj(psi_i) psi_{i + 2^q})
// over the chunk's pairs (i with bit q clear).
template <typename R>
__global__ __launch_bounds__(kBlock) void k_traj_x(const cx<R> *__restrict__ states, int n, int chunk_log2, int chunks_log2,
                                                   const int32_t *__restrict__ nins, int n_traj, double *__restrict__ partial) {
    __shared__ double red[kBlock / 64];
    const u64 N = 1ull << n;
    const u64 c = blockIdx.x & ((1ull << chunks_log2) - 1);
    const u64 rest = blockIdx.x >> chunks_log2;
    const int q = (int)(rest % (u64)n);
    const u64 t = rest / (u64)n;
    if (!traj_simulated(nins, t, n_traj)) return;
    const cx<R> *psi = states + t * N;
    const u64 npairs = N >> 1, per = npairs >> chunks_log2;
    double acc = 0.0;
    const u64 k1 = (c + 1) * per;
    u64 k = c * per + threadIdx.x;
    for (; k + 3 * kBlock < k1; k += 4 * kBlock) {  // four steps, loads first; same summation order
        cx<R> a[4], b[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const u64 i = insert0(k + (u64)s * kBlock, q);
            a[s] = psi[i];
            b[s] = psi[i | (1ull << q)];
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) acc += 2.0 * ((double)a[s].x * b[s].x + (double)a[s].y * b[s].y);
    }
    for (; k < k1; k += kBlock) {
        const u64 i = insert0(k, q);
        const cx<R> a = psi[i], b = psi[i | (1ull << q)];
        acc += 2.0 * ((double)a.x * b.x + (double)a.y * b.y);
    }
    const double s = tblock_sum(acc, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// One thread per (trajectory, value): sum the chunk partials of the
// trajectory's representative in order, then undo the trajectory's frame.
__global__ void k_traj_final(const double *__restrict__ pzf, const double *__restrict__ px, int n, int chunks, int n_traj,
                             const uint64_t *__restrict__ final_frame, const int32_t *__restrict__ nins, double *__restrict__ z,
                             double *__restrict__ x, double *__restrict__ fid, double *__restrict__ dval, QPerm perm) {
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    const int per = n + n + 2;  // z values, x values, fidelity, diagonal observable
    if (id >= n_traj * per) return;
    const int t = id / per, v = id % per;
    const u64 rep = traj_rep(nins, t, n_traj);
    const u64 f = final_frame[t];
    const u32 a = (u32)f, b = (u32)(f >> 32);
    const int nv = n + 3;
    const u64 zsrc = traj_simulated(nins, t, n_traj) || f != 0 ? (u64)t : rep;  // whose Z / fidelity partials (see k_traj_zf)
    if (v < n) {
        const int qs = perm.active ? perm.src[v] : v;  // the simulated qubit that ends on qubit v
        const double *p = pzf + zsrc * chunks * nv;
        double s = 0.0;
        for (int c = 0; c < chunks; ++c) s += p[(u64)c * nv + qs];
        if (z) z[(u64)t * n + v] = ((a >> qs) & 1) ? -s : s;
    } else if (v < 2 * n) {
        const int q = v - n, qs = perm.active ? perm.src[q] : q;
        const double *p = px + (rep * n + qs) * chunks;
        double s = 0.0;
        for (int c = 0; c < chunks; ++c) s += p[c];
        if (x) x[(u64)t * n + q] = ((b >> qs) & 1) ? -s : s;
    } else if (v == 2 * n) {
        const double *p = pzf + zsrc * chunks * nv;
        double re = 0.0, im = 0.0;
        for (int c = 0; c < chunks; ++c) {
            re += p[(u64)c * nv + n];
            im += p[(u64)c * nv + n + 1];
        }
        if (fid) fid[t] = re * re + im * im;
    } else {
        const double *p = pzf + zsrc * chunks * nv;
        double s = 0.0;
        for (int c = 0; c < chunks; ++c) s += p[(u64)c * nv + n + 2];
        if (dval) dval[t] = s;
    }
}

// p_mean(k) = (1/T) sum_t |psi_t(k xor a_t)|^2, trajectories summed in order
// (a noiseless trajectory reads the noiseless run's state).
// Trajectories whose probabilities are not those of the noiseless run (their
// own state, or the noiseless state under a frame with X bits): list[0..m),
// in index order; cnt[0] = m, cnt[1] = number of the others.  One block.
__global__ __launch_bounds__(1024) void k_traj_pm_list(int n_traj, const uint64_t *__restrict__ final_frame, const int32_t *__restrict__ nins,
                                                       int32_t *__restrict__ list, int32_t *__restrict__ cnt) {
    __shared__ int32_t wsum[16];
    __shared__ int32_t base;
    if (threadIdx.x == 0) base = 0;
    __syncthreads();
    for (int t0 = 0; t0 < n_traj; t0 += 1024) {
        const int t = t0 + (int)threadIdx.x;
        const int in = t < n_traj && (traj_rep(nins, (u64)t, n_traj) != (u64)n_traj || (u32)final_frame[t] != 0u) ? 1 : 0;
        // exclusive prefix sum over the block: within the wave, then over waves
        const u64 ball = __ballot(in);
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        const int before = __popcll(ball & ((1ull << lane) - 1));
        if (lane == 0) wsum[wv] = __popcll(ball);
        __syncthreads();
        int off = base;
        for (int k = 0; k < wv; ++k) off += wsum[k];
        if (in) list[off + before] = t;
        __syncthreads();
        if (threadIdx.x == 0) {
            int tot = 0;
            for (int k = 0; k < 16; ++k) tot += wsum[k];
            base += tot;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        cnt[0] = base;
        cnt[1] = n_traj - base;
    }
}

// Mean over trajectories of p_t(k) = |psi_rep(t)(k xor a_t)|^2: the
// trajectories that share the noiseless probabilities enter as one weighted
// term, the listed ones one by one (four loads in flight per thread).
template <typename R>
__global__ __launch_bounds__(kBlock) void k_traj_prob_mean(const cx<R> *__restrict__ states, u64 N, int n_traj, const uint64_t *__restrict__ final_frame,
                                                           const int32_t *__restrict__ nins, const int32_t *__restrict__ list,
                                                           const int32_t *__restrict__ cnt, double *__restrict__ out, QPerm perm, int n) {
    const u64 k = (u64)blockIdx.x * kBlock + threadIdx.x;
    if (k >= N) return;
    const int m = cnt[0];
    const cx<R> v0 = states[(u64)n_traj * N + k];
    double s = (double)cnt[1] * ((double)v0.x * v0.x + (double)v0.y * v0.y);
    int i = 0;
    for (; i + 4 <= m; i += 4) {
        cx<R> v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int t = list[i + u];
            v[u] = states[traj_rep(nins, (u64)t, n_traj) * N + (k ^ (u32)final_frame[t])];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) s += (double)v[u].x * v[u].x + (double)v[u].y * v[u].y;
    }
    for (; i < m; ++i) {
        const int t = list[i];
        const cx<R> v = states[traj_rep(nins, (u64)t, n_traj) * N + (k ^ (u32)final_frame[t])];
        s += (double)v.x * v.x + (double)v.y * v.y;
    }
    out[perm.active ? perm_index(perm, n, k) : k] = s / (double)n_traj;
}

// ------------------------------------------------------------------ host side

struct TrajLayout {
    size_t states, ideal2, frames, final_frame, nins, first, pmlist, pzf, px, gates, dgates, nm, tv, tc, total;
    int chunk_log2, chunks_log2;
    bool tables;  // room for the compiled passes' per-trajectory gate tables
};

// Per-trajectory gate tables of the compiled passes: used for registers of at
// least one full 12-qubit tile when they stay within this size.
constexpr size_t kTrajTableMax = (size_t)1 << 30;

static int count_noise(const qs_gate *gates, int count) {
    int c = 0;
    for (int k = 0; k < count; ++k) c += gates[k].kind == QS_G_NOISE;
    return c;
}

// nnoise: noise gates in the list (their matrices are stored per trajectory).
static TrajLayout traj_layout(int n, int dtype, int count, int n_traj, int nnoise) {
    TrajLayout L{};
    const u64 N = 1ull << n;
    auto align = [](size_t v) { return (v + 255) & ~(size_t)255; };
    L.chunk_log2 = n < 12 ? n : 12;
    L.chunks_log2 = n - L.chunk_log2;
    size_t off = 0;
    L.states = off;
    off = align(off + (size_t)(n_traj + 1) * N * amp_bytes(dtype));
    L.ideal2 = off;  // the noiseless run's second state buffer
    off = align(off + (size_t)N * amp_bytes(dtype));
    L.frames = off;
    off = align(off + (size_t)(n_traj + 1) * count * sizeof(uint64_t));
    L.final_frame = off;
    off = align(off + (size_t)(n_traj + 1) * sizeof(uint64_t));
    L.nins = off;
    off = align(off + (size_t)(n_traj + 1) * sizeof(int32_t));
    L.first = off;
    off = align(off + (size_t)(n_traj + 1) * sizeof(int32_t));
    L.pmlist = off;  // probability-mean list (n_traj entries) and its two counts
    off = align(off + (size_t)(n_traj + 2) * sizeof(int32_t));
    L.pzf = off;
    off = align(off + (size_t)(n_traj + 1) * ((size_t)1 << L.chunks_log2) * (n + 3) * sizeof(double));
    L.px = off;
    off = align(off + (size_t)(n_traj + 1) * n * ((size_t)1 << L.chunks_log2) * sizeof(double));
    L.gates = off;
    off = align(off + (size_t)count * sizeof(TGate));
    L.dgates = off;
    off = align(off + (size_t)count * sizeof(DGate));
    L.nm = off;
    off = align(off + (size_t)n_traj * nnoise * 8 * sizeof(double));
    const size_t tv_bytes = (size_t)(n_traj + 1) * count * 8 * sizeof(double);
    L.tables = n >= 12 && tv_bytes <= kTrajTableMax;
    L.tv = off;
    if (L.tables) off = align(off + tv_bytes);
    L.tc = off;
    if (L.tables) off = align(off + (size_t)(n_traj + 1) * count * sizeof(int32_t));
    L.total = off;
    return L;
}

// Expected pass work of a plan for trajectories with insertion probability p
// per slot (gate applications plus a per-pass floor for the state traffic;
// the noiseless run does every pass), used to choose how finely to cut the
// early passes: a trajectory runs every pass from the one holding the first
// gate executed after its first insertion.
static double traj_plan_cost(const std::vector<DPass> &passes, const std::vector<DGate> &dg, const qs_gate *gates, int count, double p,
                             int n_traj) {
    constexpr double kFloor = 14.5;  // one pass's read+write of a state, in gate applications (measured, 16 qubits)
    const int np = (int)passes.size();
    std::vector<int> after(count + 1, np);  // after[g]: earliest pass holding a gate of the list beyond g - 1
    for (int k = 0; k < np; ++k)
        for (int i = passes[k].gate_begin; i < passes[k].gate_begin + passes[k].gate_count; ++i) after[dg[i].gidx] = k;
    for (int g = count - 1; g >= 0; --g) after[g] = std::min(after[g], after[g + 1]);
    std::vector<double> tail(np + 1, 0.0);
    for (int k = np - 1; k >= 0; --k) tail[k] = tail[k + 1] + passes[k].gate_count + kFloor;
    double surv = 1.0, e = 0.0;
    for (int g = 0; g < count; ++g) {
        const int slots = gates[g].kind == QS_G_NOISE ? 0 : gates[g].kind == QS_G_1Q ? 1 : 2;
        const double pins = 1.0 - std::pow(1.0 - p, slots);
        e += surv * pins * tail[after[g + 1]];
        surv *= 1.0 - pins;
    }
    return n_traj * e + tail[0];
}

// Compiled trajectory passes, kept per (plan structure, device) for the
// process: a trajectory run is one call, and repeated runs of one circuit
// reuse the code without generating its source again (the key is the plan's
// structure, from which the source is a function: pass tiles and each plan
// gate's kind, slots, sweep and folding marks, not its values).  At most
// kMaxTrajModules are kept; beyond that the device is synchronised and the
// least recently used module unloaded.
struct TrajModule {
    hipModule_t mod = nullptr;
    std::vector<hipFunction_t> fn;
    uint64_t last_use = 0;
};
constexpr size_t kMaxTrajModules = 16;
static std::mutex g_traj_mu;
static uint64_t g_traj_clock = 0;
static auto *g_traj_mods = new std::map<std::pair<std::string, int>, TrajModule>();  // never destroyed (process exit)

static std::string traj_plan_key(const std::vector<DPass> &passes, const std::vector<DGate> &dg, int dtype) {
    std::string k;
    auto add = [&](const void *p, size_t n) { k.append((const char *)p, n); };
    add(&dtype, sizeof dtype);
    for (const DPass &P : passes) {
        add(&P.tb, sizeof P.tb);
        add(&P.nrest, sizeof P.nrest);
        add(P.T, sizeof P.T);
        add(&P.gate_begin, sizeof P.gate_begin);
        add(&P.gate_count, sizeof P.gate_count);
    }
    for (const DGate &d : dg) add(&d, offsetof(DGate, nidx));  // kind .. run: everything the source depends on
    return k;
}

// Functions of the plan's compiled passes; `make_src` runs only when they
// are not cached.  Fails (the caller then interprets) if it returns "".
static int traj_functions(const std::string &plan_key, const std::function<std::string()> &make_src, int np, std::vector<hipFunction_t> &out) {
    int dev = 0;
    QS_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_traj_mu);
    auto key = std::make_pair(plan_key, dev);
    auto it = g_traj_mods->find(key);
    if (it == g_traj_mods->end()) {
        const std::string src = make_src();
        if (src.empty()) return QS_ERR_UNSUPPORTED;
        JitFns jf;
        if (int rc = jit_block_functions(src, np, dev, jf, "qs_tpass")) return rc;
        if (g_traj_mods->size() >= kMaxTrajModules) {
            auto lru = g_traj_mods->begin();
            for (auto j = g_traj_mods->begin(); j != g_traj_mods->end(); ++j)
                if (j->second.last_use < lru->second.last_use) lru = j;
            (void)hipDeviceSynchronize();
            (void)hipModuleUnload(lru->second.mod);
            g_traj_mods->erase(lru);
        }
        TrajModule m;
        m.mod = jf.mod;
        m.fn = jf.fn;
        it = g_traj_mods->emplace(key, std::move(m)).first;
    }
    it->second.last_use = ++g_traj_clock;
    out = it->second.fn;
    return QS_OK;
}

template <typename R, int TBMAX>
static int traj_run_t(int n, int dtype, const qs_gate *gates, int count, u64 basis, int n_traj, double p, double inv_T1, double inv_T2, u64 seed,
                      const qs_traj_out *out, char *ws, hipStream_t st) {
    const int nnoise = count_noise(gates, count);
    const TrajLayout L = traj_layout(n, dtype, count, n_traj, nnoise);
    const u64 N = 1ull << n;
    // SWAP gates at the end of a list without noise gates are not simulated:
    // they become the read-outs' qubit relabelling (QPerm).
    QPerm perm{};
    int count_exec = count;
    if (nnoise == 0) {
        while (count_exec > 1 && gates[count_exec - 1].kind == QS_G_SWAP) --count_exec;
        if (count_exec < count) {
            perm.active = 1;
            for (int q = 0; q < kTrajMaxQubits; ++q) perm.src[q] = (uint8_t)q;
            for (int k = count_exec; k < count; ++k) std::swap(perm.src[gates[k].q0], perm.src[gates[k].q1]);
        }
    }
    std::vector<DPass> passes;
    std::vector<DGate> dg;
    make_plan(n, dtype, TBMAX, gates, count_exec, passes, dg);
    bool noisy_gates = false;
    for (int k = 0; k < count; ++k)
        if (gates[k].kind == QS_G_NOISE && gates[k].u[0] > 0.0 && (inv_T1 > 0.0 || inv_T2 > 0.0)) noisy_gates = true;
    // Sparse insertions: cut the first pass's stretch of the list into up to
    // four shorter passes when the expected work drops (noise gates make every
    // trajectory run every pass, so they keep the plan).
    if (!noisy_gates && p > 0.0 && p < 1.0 && !passes.empty()) {
        const int L = passes[0].gate_count;
        double best = traj_plan_cost(passes, dg, gates, count, p, n_traj);
        for (int parts = 2; parts <= 4 && L >= 2 * parts; ++parts) {
            std::vector<DPass> p2;
            std::vector<DGate> d2;
            make_plan(n, dtype, TBMAX, gates, count_exec, p2, d2, (L + parts - 1) / parts, L);
            const double c = traj_plan_cost(p2, d2, gates, count, p, n_traj);
            if (c < best) {
                best = c;
                passes.swap(p2);
                dg.swap(d2);
            }
        }
    }
    // A one-qubit gate followed (execution order) by a noise gate on its qubit
    // takes the noise matrix into its own (pad0 = 1); the noise gate is then
    // skipped (pad0 = 2).
    for (size_t i = 0; nnoise && i + 1 < dg.size(); ++i)
        if (dg[i].kind == QS_G_1Q && dg[i + 1].kind == QS_G_NOISE && dg[i + 1].q0 == dg[i].q0) {
            dg[i].pad0 = 1;
            dg[i + 1].pad0 = 2;
            ++i;
        }
    // dg holds every simulated gate once, in execution order (dg[i].gidx: its
    // list index); each pass applies a slice of it.
    // The device copy carries each gate's first draw slot and its execution
    // position in the plan in its pad field (16 bits each; count for the
    // trailing SWAPs, which are never executed).
    std::vector<qs_gate> gl(gates, gates + count);
    for (int k = 0; k < count; ++k) gl[k].pad = count << 16;
    for (size_t i = 0; i < dg.size(); ++i) gl[dg[i].gidx].pad = (int)i << 16;
    for (int k = 0, slot = 0; k < count; ++k) {
        gl[k].pad |= slot;
        slot += gates[k].kind == QS_G_NOISE ? 0 : gates[k].kind == QS_G_1Q ? 1 : 2;
    }
    QS_HIP(hipMemcpyAsync(ws + L.gates, gl.data(), (size_t)count * sizeof(TGate), hipMemcpyHostToDevice, st));
    QS_HIP(hipMemcpyAsync(ws + L.dgates, dg.data(), dg.size() * sizeof(DGate), hipMemcpyHostToDevice, st));
    QS_HIP(hipStreamSynchronize(st));  // host arrays are released when this call returns
    u32 thr = 0;
    if (p >= 1.0) thr = 0xFFFFFFFFu;
    else if (p > 0.0) thr = (u32)floor(p * 4294967296.0);
    uint64_t *frames = (uint64_t *)(ws + L.frames), *final_frame = (uint64_t *)(ws + L.final_frame);
    int32_t *nins = (int32_t *)(ws + L.nins), *first_gate = (int32_t *)(ws + L.first);
    hipLaunchKernelGGL(k_traj_frames, dim3((n_traj + kFrameWaves) / kFrameWaves), dim3(64 * kFrameWaves), 0, st, (const TGate *)(ws + L.gates),
                       count, n_traj, thr,
                       (u32)seed, (u32)(seed >> 32), frames, final_frame, nins, first_gate, out->counts, out->log, out->log ? out->log_cap : 0,
                       noisy_gates ? 1 : 0, perm, n);
    QS_LAUNCH_CHECK("traj_frames");
    double *nm = (double *)(ws + L.nm);
    if (nnoise) {
        const u64 work = (u64)n_traj * count;
        hipLaunchKernelGGL(k_traj_noise_mats, dim3(grid_for(work, 256)), dim3(256), 0, st, (const DGate *)(ws + L.dgates), count, n_traj, nnoise,
                           (u32)seed, (u32)(seed >> 32), inv_T1, inv_T2, nm);
        QS_LAUNCH_CHECK("traj_noise_mats");
    }
    cx<R> *states = (cx<R> *)(ws + L.states);
    const int T1 = n_traj + 1;
    // The noiseless run alternates between its state slot and ideal2 so that
    // its last pass writes the slot the read-outs use.
    cx<R> *ibuf[2] = {states + (u64)n_traj * N, (cx<R> *)(ws + L.ideal2)};
    const int np = (int)passes.size();
    // Compiled passes (jit_block.hip) when the workspace holds the gate
    // tables and every pass has a full tile; QSIM_TRAJ_PATH=interp keeps the
    // interpreter kernel.
    std::vector<hipFunction_t> jfn;
    if (L.tables && !(getenv("QSIM_TRAJ_PATH") && std::string(getenv("QSIM_TRAJ_PATH")) == "interp")) {
        if (traj_functions(traj_plan_key(passes, dg, dtype), [&] { return jit_traj_source(passes, dg, dtype); }, np, jfn) != QS_OK) jfn.clear();
    }
    if (!jfn.empty()) {
        R *tv = (R *)(ws + L.tv);
        int32_t *tc = (int32_t *)(ws + L.tc);
        const int ng = (int)dg.size();
        hipLaunchKernelGGL(k_traj_vals<R>, dim3(grid_for((u64)T1 * ng, 256)), dim3(256), 0, st, (const DGate *)(ws + L.dgates), ng,
                           (const uint64_t *)frames, count, (const int32_t *)nins, n_traj, (const double *)nm, nnoise, tv, tc);
        QS_LAUNCH_CHECK("traj_vals");
        for (int k = 0; k < np; ++k) {
            const u64 blocks = (u64)T1 << passes[k].nrest;
            const cx<R> *in = k == 0 ? nullptr : ibuf[(np - k) & 1];
            cx<R> *outb = ibuf[(np - 1 - k) & 1];
            void *a_states = states, *a_tv = tv, *a_tc = tc, *a_nins = nins, *a_first = first_gate, *a_in = (void *)in, *a_out = outb;
            unsigned long long a_N = N, a_basis = basis;
            unsigned a_ng = (unsigned)ng;
            int a_fp = k == 0 ? 1 : 0, a_nt = n_traj;
            void *args[] = {&a_states, &a_N, &a_tv, &a_tc, &a_ng, &a_fp, &a_basis, &a_nins, &a_first, &a_nt, &a_in, &a_out};
            QS_HIP(hipModuleLaunchKernel(jfn[k], (unsigned)blocks, 1, 1, kTileThreads, 1, 1, 0, st, args, nullptr));
        }
    } else {
        for (int k = 0; k < np; ++k) {
            const DPass &P = passes[k];
            const int tiles_log2 = P.nrest;
            const u64 blocks = (u64)T1 << tiles_log2;
            const cx<R> *in = k == 0 ? nullptr : ibuf[(np - k) & 1];
            cx<R> *outb = ibuf[(np - 1 - k) & 1];
            hipLaunchKernelGGL((k_traj_pass<R, TBMAX>), dim3((unsigned)blocks), dim3(kTileThreads), 0, st, states, N, tiles_log2, P,
                               (const DGate *)(ws + L.dgates), (const uint64_t *)frames, count, k == 0 ? 1 : 0, basis, (const int32_t *)nins,
                               (const int32_t *)first_gate, n_traj, (const double *)nm, nnoise, in, outb);
            QS_LAUNCH_CHECK("traj_pass");
        }
    }
    double *pzf = (double *)(ws + L.pzf), *px = (double *)(ws + L.px);
    const int chunks = 1 << L.chunks_log2;
    const double *diag = out->diag_val ? out->diag : nullptr;
    if (out->z || out->fid || diag) {
        const u64 blocks = (u64)T1 << L.chunks_log2;
        if (out->fid)
            hipLaunchKernelGGL((k_traj_zf<R, true>), dim3((unsigned)blocks), dim3(kBlock), 0, st, (const cx<R> *)states, n, L.chunk_log2, L.chunks_log2,
                               (const uint64_t *)final_frame, (const int32_t *)nins, n_traj, diag, pzf, perm);
        else
            hipLaunchKernelGGL((k_traj_zf<R, false>), dim3((unsigned)blocks), dim3(kBlock), 0, st, (const cx<R> *)states, n, L.chunk_log2, L.chunks_log2,
                               (const uint64_t *)final_frame, (const int32_t *)nins, n_traj, diag, pzf, perm);
        QS_LAUNCH_CHECK("traj_zf");
    }
    if (out->x) {
        const u64 blocks = ((u64)T1 * n) << L.chunks_log2;
        hipLaunchKernelGGL(k_traj_x<R>, dim3((unsigned)blocks), dim3(kBlock), 0, st, (const cx<R> *)states, n, L.chunk_log2, L.chunks_log2,
                           (const int32_t *)nins, n_traj, px);
        QS_LAUNCH_CHECK("traj_x");
    }
    if (out->z || out->x || out->fid || diag) {
        const int work = n_traj * (2 * n + 2);
        hipLaunchKernelGGL(k_traj_final, dim3((work + 255) / 256), dim3(256), 0, st, (const double *)pzf, (const double *)px, n, chunks, n_traj,
                           (const uint64_t *)final_frame, (const int32_t *)nins, out->z, out->x, out->fid, diag ? out->diag_val : nullptr,
                           perm);
        QS_LAUNCH_CHECK("traj_final");
    }
    if (out->prob_mean) {
        int32_t *pml = (int32_t *)(ws + L.pmlist), *pmc = pml + n_traj;
        hipLaunchKernelGGL(k_traj_pm_list, dim3(1), dim3(1024), 0, st, n_traj, (const uint64_t *)final_frame, (const int32_t *)nins, pml, pmc);
        QS_LAUNCH_CHECK("traj_prob_mean");
        hipLaunchKernelGGL(k_traj_prob_mean<R>, dim3((unsigned)((N + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, (const cx<R> *)states, N, n_traj,
                           (const uint64_t *)final_frame, (const int32_t *)nins, (const int32_t *)pml, (const int32_t *)pmc, out->prob_mean,
                           perm, n);
        QS_LAUNCH_CHECK("traj_prob_mean");
    }
    return QS_OK;
}

int validate_gates(int n, const qs_gate *gates, int count, bool allow_noise);

static int traj_run_any(int n, int dtype, const qs_gate *gates, int count, u64 basis_index, int n_traj, const qs_noise &nz, u64 seed,
                        const qs_traj_out *out, void *ws, size_t ws_bytes, void *stream) {
    if (dtype != QS_C64 && dtype != QS_C128) return fail(QS_ERR_DTYPE, "dtype must be QS_C64 or QS_C128");
    if (n < 1 || n > kTrajMaxQubits) return fail(QS_ERR_ARG, "trajectories need 1 <= n <= 20");
    if (count < 1 || count > kTrajMaxGates || n_traj < 1) return fail(QS_ERR_ARG, "bad gate or trajectory count");
    if (!out || !ws) return fail(QS_ERR_ARG, "null output struct or workspace");
    if (out->log && out->log_cap < 1) return fail(QS_ERR_ARG, "log_cap must be >= 1 with a log buffer");
    if (out->diag_val && !out->diag) return fail(QS_ERR_ARG, "diag_val needs the diagonal observable");
    if (basis_index >= (1ull << n)) return fail(QS_ERR_ARG, "basis index >= 2^n");
    if (!(nz.p_depol >= 0.0 && nz.p_depol <= 1.0)) return fail(QS_ERR_ARG, "p must be in [0, 1]");
    if (!(nz.T1 > 0.0) || !(nz.T2 > 0.0) || !(nz.T2 <= 2.0 * nz.T1)) return fail(QS_ERR_ARG, "need T1 > 0 and 0 < T2 <= 2 T1");
    if (int rc = validate_gates(n, gates, count, true)) return rc;
    if (ws_bytes < traj_layout(n, dtype, count, n_traj, count_noise(gates, count)).total)
        return fail(QS_ERR_SIZE, "trajectory workspace too small");
    const double inv_T1 = nz.T1 < INFINITY ? 1.0 / nz.T1 : 0.0, inv_T2 = nz.T2 < INFINITY ? 1.0 / nz.T2 : 0.0;
    hipStream_t st = (hipStream_t)stream;
    // Tiles of 12 qubits for both types (64 KiB of LDS for c128, 32 KiB for
    // c64): with many small states, c64 gains more from twice the resident
    // workgroups per CU than from the wider tile a single state uses.
    return dtype == QS_C128
               ? traj_run_t<double, 12>(n, dtype, gates, count, basis_index, n_traj, nz.p_depol, inv_T1, inv_T2, seed, out, (char *)ws, st)
               : traj_run_t<float, 12>(n, dtype, gates, count, basis_index, n_traj, nz.p_depol, inv_T1, inv_T2, seed, out, (char *)ws, st);
}

}  // namespace qs

using namespace qs;

QS_API int qs_traj_workspace_bytes(int n, int dtype, int count, int n_traj, size_t *bytes) {
    if (!bytes) return fail(QS_ERR_ARG, "null output");
    if (dtype != QS_C64 && dtype != QS_C128) return fail(QS_ERR_DTYPE, "dtype must be QS_C64 or QS_C128");
    if (n < 1 || n > kTrajMaxQubits) return fail(QS_ERR_ARG, "trajectories need 1 <= n <= 20");
    if (count < 1 || count > kTrajMaxGates || n_traj < 1) return fail(QS_ERR_ARG, "bad gate or trajectory count");
    *bytes = traj_layout(n, dtype, count, n_traj, 0).total;
    return QS_OK;
}

QS_API int qs_traj_noise_workspace_bytes(int n, int dtype, const qs_gate *gates, int count, int n_traj, size_t *bytes) {
    if (!bytes || !gates) return fail(QS_ERR_ARG, "null output or gate list");
    if (dtype != QS_C64 && dtype != QS_C128) return fail(QS_ERR_DTYPE, "dtype must be QS_C64 or QS_C128");
    if (n < 1 || n > kTrajMaxQubits) return fail(QS_ERR_ARG, "trajectories need 1 <= n <= 20");
    if (count < 1 || count > kTrajMaxGates || n_traj < 1) return fail(QS_ERR_ARG, "bad gate or trajectory count");
    *bytes = traj_layout(n, dtype, count, n_traj, count_noise(gates, count)).total;
    return QS_OK;
}

QS_API int qs_traj_run(int n, int dtype, const qs_gate *gates, int count, uint64_t basis_index, int n_traj, double p_depol, uint64_t seed,
                       const qs_traj_out *out, void *ws, size_t ws_bytes, void *stream) {
    try {
        for (int k = 0; gates && k < count && k < kTrajMaxGates; ++k)
            if (gates[k].kind == QS_G_NOISE) return fail(QS_ERR_ARG, "noise gates need qs_traj_run_noise");
        const qs_noise nz{p_depol, INFINITY, INFINITY};
        return traj_run_any(n, dtype, gates, count, basis_index, n_traj, nz, seed, out, ws, ws_bytes, stream);
    } catch (...) {
        return fail(QS_ERR_UNSUPPORTED, "unexpected internal error");
    }
}

QS_API int qs_traj_run_noise(int n, int dtype, const qs_gate *gates, int count, uint64_t basis_index, int n_traj, const qs_noise *noise,
                             uint64_t seed, const qs_traj_out *out, void *ws, size_t ws_bytes, void *stream) {
    try {
        if (!noise) return fail(QS_ERR_ARG, "null noise model");
        return traj_run_any(n, dtype, gates, count, basis_index, n_traj, *noise, seed, out, ws, ws_bytes, stream);
    } catch (...) {
        return fail(QS_ERR_UNSUPPORTED, "unexpected internal error");
    }
}
