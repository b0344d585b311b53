// QAOA pass plans and batched launches, shared by the single-graph entry
// point (qaoa.hip) and the pool (pool.hip).
#pragma once

#include <vector>

#include "common.h"

namespace qs {

constexpr int kQMaxEdges = 128;

// Pass flags.  FIRST: the cost phase exp(-i gamma_1 C) at the start, on the
// uniform state generated in registers.  PHASE_END: exp(-i gamma_{l+1} C) at
// the end (one qubit group per layer).  MERGE: the pass continues into the
// next layer on the same qubit group: exp(-i gamma_{l+1} C), then the RX
// gates of layer l+1 on the group.  LAST: the pass also accumulates E.
enum { QF_FIRST = 1, QF_PHASE_END = 2, QF_LAST = 4, QF_MERGE = 8 };

// Per (pass, tile) partial sums of the backward: 0 = gamma of the phase at the
// end or in the middle of the pass, 1 = beta of the pass's layer, 2 = gamma_1
// (first pass), 3 = beta of the next layer (merged passes).
constexpr int kQSlots = 4;

// Edge classes by where the endpoints sit for a thread map: thread-index bit
// ("t"), register-index bit ("j"), or a qubit fixed per tile ("r").
enum { EC_TT = 0, EC_TR, EC_TJ, EC_JJ, EC_JR, EC_RR, EC_N };

struct QEdge {
    uint8_t a, b, wi, pad;
};

// One pass.  Edge lists are classified for the three register layouts of
// the register-tiled kernels (list 0 also serves the LDS kernels).
struct QPass {
    int tb, nrest, layer, flags, pidx;
    uint32_t rx_mask;  // tile bits that receive RX
    int use_l2;        // register-tiled kernels: upper lane bits take RX in the third layout
    int lay_mid;       // register-tiled forward kernel: the layout its first mixer ends in
    alignas(4) uint8_t T[16];     // read as 32-bit words on the device
    alignas(4) uint8_t rest[40];
    int32_t cnt[3][EC_N];  // 32-bit: read with scalar loads at a run-time layout index
    QEdge e[3][kQMaxEdges];
};

struct QWeights {
    double w[kQMaxEdges];
};

// np: passes per circuit.
struct QGeom {
    int n, p, P, tb, G, glog, num_edges, weighted, np;
};

// Which (pass, slot) partial sums make up each output of the final
// reduction: component c < 2p (gamma_1..gamma_p, beta_1..beta_p) sums items
// start[c] .. start[c+1]-1, item = pass << 2 | slot, in pass order.
constexpr int kQMaxP = 64, kQMaxItems = 512;
struct QMap {
    uint16_t start[2 * kQMaxP + 1];
    uint16_t item[kQMaxItems];
};

// Where circuit c of a launch keeps its data: ws + c * circ_bytes + offset
// (offsets < 0 mean "absent").  Single-graph launches: its angles are
// theta + c * 2p and its outputs slot c.  Pooled launches: it is circuit
// circ_map[c0 + c] of the pool (angles and outputs at that index), and its
// pass-k descriptor is passes[((c0 + c) / sets) * np + k].
struct QBatch {
    char *ws;
    u64 circ_bytes;
    long long in_off, out_off, lam_off, part_off, epart_off;
    const double *theta;
    const QPass *passes;
    const int32_t *circ_map;
    int c0, k, sets, np;
};

// Tile shape: TB tile qubits handled by 2^TT threads; r contiguous low qubits
// in every higher-group tile.  rt: register-tiled kernels (n >= 10).
struct QShape {
    int TB, TT, r;
};

struct QPlan {
    QShape shape;
    bool rt;
    QGeom geo;
    std::vector<QPass> passes;   // forward order (geo.np passes)
    std::vector<uint8_t> merged; // per pass: a merged pass (its own kernel instantiation)
    QMap map;
    QWeights W;
};

// Per-circuit workspace layout (byte offsets; -1 = unused).
struct QLayout {
    long long ckpt, lam, part, epart;
    size_t bytes;
};

int build_qplan(int n, int p, int num_edges, const int32_t *edges, const double *w, QShape shape, QPlan &plan);
QLayout qaoa_layout(const QGeom &g, int with_grad);
int launch_qaoa_batch(const QPlan &plan, const double *theta, int nb, double *E_out, double *grad_out, char *ws, size_t circ_bytes, hipStream_t st);
// nb circuits starting at B.c0 of a pooled size class (unit weights).
int launch_qaoa_pooled(const QPlan &proto, const QBatch &B, int nb, double *E_out, double *grad_out, hipStream_t st);
int check_edges(int n, int ne, const int32_t *edges);
// Shape with the fewest passes for n qubits (QSIM_QAOA_TB / QSIM_QAOA_R override).
QShape qaoa_default_shape(int n);
// Candidate shapes the pool's autotuner times.
std::vector<QShape> qaoa_candidate_shapes(int n);
int qaoa_passes_per_layer(int n, QShape s);

}  // namespace qs
