/*
 * qsim.h — C-ABI of the MI355X state-vector simulator (libqsim_hip.so).
 *
 * The operation set follows the paper's Software description: a register of n
 * qubits holding 2^n complex amplitudes is initialised, evolved by one-qubit
 * gates and by two-qubit gates of the controlled form, and read out through
 * probabilities, Pauli expectations and measurement statistics; the "pool of
 * multiple states" runs many related circuits (variational parameters or noise
 * realisations) side by side.
 *
 * Conventions for every call
 *   - Amplitude i, i = sum_q i_q 2^q, qubit 0 = least-significant bit
 *     (Software description, eq. 1; the three-qubit figure's vector order).
 *   - Amplitudes are interleaved (re, im): 16 bytes each for QS_C128
 *     (double), 8 bytes for QS_C64 (float).  Reductions always accumulate in
 *     FP64, also for QS_C64.
 *   - A one-qubit gate is u[8] = {re00, im00, re01, im01, re10, im10, re11,
 *     im11}, row = output index (eq. 3).  For QS_C64 it is rounded to float.
 *     Unitarity is not checked.
 *   - Ownership: device memory (state buffers, outputs, workspaces) belongs to
 *     the caller.  The library borrows raw device pointers and a hipStream_t
 *     passed as void*; it never frees them.  A qs_state handle owns only its
 *     own metadata and a small device scratch area for partial sums and gate
 *     plans, released by qs_state_destroy.
 *   - All device work is asynchronous and ordered on the handle's stream.
 *     Outputs land in caller-provided DEVICE buffers; read them after
 *     qs_sync or a stream synchronisation.  Kernel faults surface at qs_sync
 *     or at a later call as QS_ERR_HIP.
 *   - Every call returns a status; no C++ exception crosses the ABI.  The
 *     text of the last error of the calling thread is qs_last_error().
 *   - Host-side arrays (edges, weights, gate lists, descriptors) are read
 *     during the call only; the library keeps no pointer to them.
 */
#ifndef QSIM_H
#define QSIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define QS_OK 0
#define QS_ERR_ARG (-1)         /* qubit out of range, c == t, index >= 2^n, null pointer, bad count */
#define QS_ERR_DTYPE (-2)       /* dtype not QS_C64 / QS_C128, or states of different dtype */
#define QS_ERR_SIZE (-3)        /* buffer or workspace smaller than required, or n above the limit */
#define QS_ERR_HIP (-4)         /* HIP runtime error (text in qs_last_error) */
#define QS_ERR_UNSUPPORTED (-5) /* combination not implemented */

/* Amplitude types. */
#define QS_C64 1
#define QS_C128 2

/* Largest register on one device: 2^34 * 16 B = 256 GiB (c128), 2^35 * 8 B (c64). */
#define QS_MAX_QUBITS_C128 34
#define QS_MAX_QUBITS_C64 35

typedef struct qs_state qs_state;

/* Gate record for qs_apply_block and qs_traj_run (80 bytes, 8-byte aligned). */
typedef struct qs_gate {
    int32_t kind; /* QS_G_* */
    int32_t q0;   /* 1Q: target; C1Q: control; DIAG2 / SWAP: first qubit */
    int32_t q1;   /* C1Q: target; DIAG2 / SWAP: second qubit; unused for 1Q */
    int32_t pad;  /* ignored */
    double u[8];  /* 1Q / C1Q: the 2x2 matrix; DIAG2: d00, d01, d10, d11 (re, im) with
                     entry index 2*bit(q1) + bit(q0); SWAP: unused */
} qs_gate;

#define QS_G_1Q 1    /* eq. (3) on qubit q0 */
#define QS_G_C1Q 2   /* U on target q1 iff control q0 is |1> (controlled form, Software description) */
#define QS_G_DIAG2 3 /* diagonal two-qubit phase, e.g. CZ or a controlled phase */
#define QS_G_SWAP 4  /* exchange qubits q0 and q1 */
#define QS_G_NOISE 5 /* stochastic noise gate on q0 for the duration u[0] (qs_traj_run_noise only; the
                        noiseless reference run treats it as the identity) */

/* ---------------------------------------------------------------- state */

/* Borrow dev_buf (>= 2^n amplitudes of dtype) as an n-qubit register used on
 * `stream` (a hipStream_t; NULL = the null stream).  1 <= n <= QS_MAX_QUBITS_*.
 * Paper: the QubitRegister declaration with its number of qubits.
 * Allocates a small device scratch area (partial sums, plan storage).
 * Errors: QS_ERR_ARG (null buf/out, n < 1), QS_ERR_DTYPE, QS_ERR_SIZE
 * (buf_bytes < 2^n * amplitude size, n too large), QS_ERR_HIP. */
int qs_state_create(int n, int dtype, void *dev_buf, size_t buf_bytes, void *stream, qs_state **out);

/* Release the handle and its scratch (not dev_buf).  Synchronises the stream. */
int qs_state_destroy(qs_state *s);

/* Change the stream later calls are ordered on. */
int qs_state_set_stream(qs_state *s, void *stream);

/* Wait for all work queued on the handle's stream; reports kernel faults. */
int qs_sync(qs_state *s);

/* Text of the last error on the calling thread ("" if none).  Valid until the
 * thread's next failing call. */
const char *qs_last_error(void);

/* ---------------------------------------------------------------- initialisation */

/* |index>.  Paper: Initialize("base", index).  QS_ERR_ARG if index >= 2^n. */
int qs_init_basis(qs_state *s, uint64_t index);

/* Balanced superposition H^{(x)n}|0> (all amplitudes 2^{-n/2}).  Paper:
 * Software description, "Scope and basic use" (initialisation as the balanced
 * superposition of all computational basis states). */
int qs_init_uniform(qs_state *s);

/* Seeded random normalised state: amplitude i = (2u-1) + i(2v-1), u and v the
 * 53-bit uniforms from Philox4x32-10 (key = seed, counter = (i_lo, i_hi, 1, 0),
 * words (0,1) and (2,3)), then divided by the state's 2-norm (FP64).  The
 * paper mentions random initialisation without a distribution; this is the
 * library's definition. */
int qs_init_random(qs_state *s, uint64_t seed);

/* ---------------------------------------------------------------- gates */

/* One-qubit gate on qubit q (eq. 3).  QS_ERR_ARG if q outside [0, n) or u NULL. */
int qs_apply_1q(qs_state *s, int q, const double u[8]);

/* Controlled one-qubit gate: u on target t iff control c is |1>
 * (e.g. ApplyCPauliX(c, t)).  QS_ERR_ARG if c == t or either is out of range. */
int qs_apply_c1q(qs_state *s, int c, int t, const double u[8]);

/* Two-qubit diagonal: amplitude i *= d[2*bit_q1(i) + bit_q0(i)], d as 4
 * interleaved complex numbers (CZ, controlled phase).  q0 != q1. */
int qs_apply_diag2(qs_state *s, int q0, int q1, const double d[8]);

/* SWAP of qubits a != b. */
int qs_apply_swap(qs_state *s, int a, int b);

/* Dense k-qubit gate, 1 <= k <= 5 (the Software description's gate action
 * generalised from eq. (3)'s pairs to groups of 2^k amplitudes): qubits is a
 * host array of k distinct qubits; U_dev is DEVICE memory holding the
 * 2^k x 2^k matrix row-major as interleaved (re, im) doubles, row = output,
 * and bit m of a row/column index is the value of qubits[m].  For every
 * group of indices that differ only in those bits the 2^k amplitudes are
 * replaced by U times them (computed in FP64; rounded to float for c64).
 * U_dev must be 16-byte aligned and stay valid until the stream has run the
 * gate. */
int qs_apply_kq(qs_state *s, const int32_t *qubits, int k, const double *U_dev);

/* Projective measurement of qubit q onto a given outcome (0 or 1): amplitudes
 * whose bit q differs become 0, the others are divided by sqrt(P), P = the sum
 * of their |a_i|^2 before the call (FP64, fixed-order reduction).  If P = 0
 * the whole state becomes 0.  prob_dev: device double receiving P, or NULL. */
int qs_collapse(qs_state *s, int q, int outcome, double *prob_dev);

/* Born-rule measurement of qubit q: u = u53(x0, x1) of Philox4x32-10(key =
 * seed, counter = (q, 0, 6, 0)); the outcome is 1 iff u < P1 / (P0 + P1)
 * (both sums in FP64), then the state collapses as in qs_collapse.  The
 * decision stays on the device: outcome_dev (device int32) and prob_dev
 * (device double, the outcome's probability) receive it, either may be NULL. */
int qs_measure(qs_state *s, int q, uint64_t seed, int32_t *outcome_dev, double *prob_dev);

/* Fused block: the same result as applying gates[0..count) one after the
 * other (up to rounding).  Paper: Software description, "Scope and basic
 * use" (custom multi-qubit operations built from the register's internals;
 * here a list of one- and two-qubit gates applied as one operation).  The library groups the gates into passes whose
 * targets fit one on-chip tile, moving a gate ahead of earlier ones when it
 * commutes with them (disjoint qubits, or both diagonal) and that saves
 * passes, and runs each pass as one read+write of the state.  Plans
 * are cached per gate list (content-keyed) in the handle; the first call with
 * a new list builds and uploads the plan synchronously, later calls with the
 * same list only launch kernels (so they may be captured in a hipGraph).
 * QS_ERR_ARG on an unknown kind (QS_G_NOISE included: noise gates belong to
 * trajectories) or a bad qubit. */
int qs_apply_block(qs_state *s, const qs_gate *gates, int count);

/* Number of read+write passes of the state that qs_apply_block takes for this
 * gate list on an n-qubit register of this dtype (host-only planning; no
 * device is touched).  *passes = 0 for count = 0.  QS_ERR_ARG / QS_ERR_DTYPE /
 * QS_ERR_SIZE as for qs_state_create and qs_apply_block. */
int qs_block_passes(int n, int dtype, const qs_gate *gates, int count, int *passes);

/* QAOA cost layer: amplitude k *= exp(-i gamma C(k)),
 * C(k) = sum over edges (u,v) of w_uv [k_u != k_v]  (w NULL = unit weights).
 * edges: host int32 [2*num_edges], 0 <= u, v < n, u != v; num_edges <= 256.
 * Paper: the Max-Cut Hamiltonian of the Particle Swarm / QAOA section, and
 * the footnote of "Scope and basic use" on the QAOA-specialised methods (one
 * diagonal operation on the whole register per layer). */
int qs_apply_cut_phase(qs_state *s, const int32_t *edges, const double *w, int num_edges, double gamma);

/* ---------------------------------------------------------------- read-outs (device outputs) */

/* P(qubit q = 1) = sum_{i: i_q = 1} |a_i|^2 into out_dev[0].  Paper: GetProbability. */
int qs_prob_one(qs_state *s, int q, double *out_dev);

/* <Z_q> = sum_i (-1)^{i_q} |a_i|^2 for q = 0..n-1 into out_dev[0..n)
 * (= 1 - 2 P(q = 1) for a normalised state), in one pass over the state.
 * Paper: "Scope and basic use" (<Z> from the probability of qubit q in |1>). */
int qs_expect_z_all(qs_state *s, double *out_dev);

/* sum_i |a_i|^2 into out_dev[0]. */
int qs_norm2(qs_state *s, double *out_dev);

/* <C> = sum_k C(k) |a_k|^2 for the cut counter of qs_apply_cut_phase.
 * Paper: Particle Swarm / QAOA section (the objective is the expectation of
 * the Max-Cut Hamiltonian after the circuit). */
int qs_expect_cut(qs_state *s, const int32_t *edges, const double *w, int num_edges, double *out_dev);

/* sum_k d_k |a_k|^2 for a real diagonal observable d_dev (device, 2^n doubles).
 * Paper: "Scope and basic use" (expectation values of multi-qubit
 * observables; a diagonal one weights each basis state's probability). */
int qs_expect_diag(qs_state *s, const double *d_dev, double *out_dev);

/* <psi|P|psi> for the Pauli product with X on bits only in xmask, Z on bits
 * only in zmask and Y on bits in both; out_dev[0] = re, out_dev[1] = im
 * (zero up to rounding, as P is Hermitian).  Masks must be < 2^n.
 * Paper: "Scope and basic use" (expectation values of products of Pauli
 * matrices). */
int qs_expect_pauli(qs_state *s, uint64_t xmask, uint64_t zmask, double *out_dev);

/* <a|b> = sum_i conj(a_i) b_i into out_dev[0..2) (re, im).  Same n and dtype;
 * the work is ordered on a's stream. */
int qs_inner(qs_state *a, qs_state *b, double *out_dev);

/* Computational-basis sampling (paper: "Scope and basic use", measurement
 * outcomes drawn from the state-dependent distribution): shot s draws
 * u_s = 53-bit uniform of
 * Philox4x32-10 (key = seed, counter = (s_lo, s_hi, 2, 0), words 0 and 1) and
 * returns the smallest index i with CDF(i) > u_s, the CDF summed in FP64;
 * u_s at or above the total returns the last index of nonzero probability.
 * out_dev: device uint64 [shots].  The library's CDF rounding differs from a
 * sequential sum only within ~1e-15 of bin boundaries. */
int qs_sample(qs_state *s, int64_t shots, uint64_t seed, uint64_t *out_dev);

/* qs_sample for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops, harnesses that forbid hipMalloc): the same
 * draws as qs_sample on a register given by pointer (dev_buf: 2^n amplitudes
 * of dtype, buf_bytes its size), without a state handle.  The partial sums
 * (chunk sums and their prefix, at most 2 * 2^18 + 1 doubles) live in a fixed
 * 4 MiB device array inside the library, one copy per device, held until the
 * process ends; this call allocates nothing.  All calls on one device share
 * that array: calls that may overlap on one device (different streams or
 * host threads) race and must be serialised by the caller.  Errors:
 * QS_ERR_DTYPE; QS_ERR_SIZE for n above QS_MAX_QUBITS_* or a short buffer;
 * QS_ERR_ARG for n < 1, null pointers or shots outside [0, 2^32]. */
int qs_sample_noalloc(int n, int dtype, const void *dev_buf, size_t buf_bytes, int64_t shots, uint64_t seed, uint64_t *out_dev,
                      void *stream);

/* ---------------------------------------------------------------- QAOA Max-Cut with adjoint gradient */

/* |psi(theta)> = prod_{l=1..p} exp(-i beta_l B) exp(-i gamma_l C) H^{(x)n}|0>,
 * B = sum_j X_j, C the cut counter; theta = [gamma_1..gamma_p, beta_1..beta_p];
 * objective E(theta) = <psi|C|psi> (Particle Swarm / QAOA section). */
typedef struct qs_qaoa_desc {
    int n;                /* qubits, 2 <= n <= 34 */
    int p;                /* layers, 1 <= p <= 64 */
    int num_edges;        /* 1 <= num_edges <= 256 */
    const int32_t *edges; /* host [2*num_edges] */
    const double *w;      /* host [num_edges] or NULL for unit weights */
} qs_qaoa_desc;

/* Device workspace needed by qs_qaoa_run for one angle set (reused across the
 * B sets of a call).  with_grad = 0: forward only. */
int qs_qaoa_workspace_bytes(const qs_qaoa_desc *d, int with_grad, size_t *bytes);

/* For b = 0..B-1: E_dev[b] = E(angles_dev[b*2p .. (b+1)*2p)); if grad_dev is
 * non-NULL, grad_dev[b*2p + k] = dE/dtheta_k by adjoint differentiation
 * (forward pass writing per-pass checkpoints, then a reverse sweep of lambda
 * with the derivative inner products reduced in FP64).  All arrays are
 * device memory; angles are read on the device, so a captured launch can be
 * replayed with new angles written in place.  ws: device workspace of at
 * least qs_qaoa_workspace_bytes.  Computes in complex128.  The host-side plan
 * (tiles, passes, edge classes) is cached by the descriptor's contents, at
 * most 16 problems, least recently used dropped first; it holds no device
 * memory. */
int qs_qaoa_run(const qs_qaoa_desc *d, const double *angles_dev, int B, double *E_dev, double *grad_dev,
                void *ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------- pool of QAOA circuits */

/* Many QAOA instances of uneven size (paper: "Pool of multiple states", each
 * circuit with its own parameters).  The first call captures the launch
 * sequence (per size class, one launch per pass over a batch of circuits)
 * into a hipGraph; later calls replay it with the angles read on the device.  Circuit c = (graph g,
 * angle set a) for g < num_graphs, a < sets_per_graph, c = g*sets_per_graph + a. */
typedef struct qs_pool_desc {
    int num_graphs;
    int sets_per_graph;
    int p;                      /* layers, shared by all circuits */
    const int32_t *n_qubits;    /* host [num_graphs], each in [2, 26] */
    const int32_t *edge_offset; /* host [num_graphs + 1]: edges of graph g are [edge_offset[g], edge_offset[g+1]) */
    const int32_t *edges;       /* host [2 * edge_offset[num_graphs]] */
} qs_pool_desc;

/* Workspace for gradients of one graph's angle sets per launch:
 * sets_per_graph times the bytes of one circuit of the largest size. */
int qs_pool_workspace_bytes(const qs_pool_desc *d, size_t *bytes);

/* Bytes one circuit of the largest size needs (with_grad = 0: forward only,
 * one state; else per-pass checkpoints as well).  A workspace of m times this
 * runs up to m circuits per launch; qs_pool_run accepts any size of at least
 * one circuit. */
int qs_pool_circuit_bytes(const qs_pool_desc *d, int with_grad, size_t *bytes);

/* angles_dev: device [circuits * 2p]; E_dev: device [circuits];
 * grad_dev: device [circuits * 2p] or NULL.  Complex128.  The library keeps
 * the plan of each (descriptor, buffers) combination it has run: the captured
 * graph and the device tables of the passes, at most 32 plans, the least
 * recently used released first. */
int qs_pool_run(const qs_pool_desc *d, const double *angles_dev, double *E_dev, double *grad_dev,
                void *ws, size_t ws_bytes, void *stream);

/* Release the plan qs_pool_run keeps for exactly these arguments (its
 * captured graph and device tables; the caller's buffers are untouched).  Call
 * it before freeing buffers a plan was captured with.  Synchronises the
 * device.  QS_OK also when no such plan exists. */
int qs_pool_release(const qs_pool_desc *d, const double *angles_dev, double *E_dev, double *grad_dev, void *ws,
                    size_t ws_bytes);

/* ---------------------------------------------------------------- Max-Cut optimum and particle swarm */

/* E_exact of each graph of a pool (Particle Swarm / QAOA section: the
 * approximation ratio divides the best <C> by the exact Max-Cut value):
 * max_dev[g] = max over all 2^n bipartitions k of C(k), summed in edge order
 * (unit weights when w is NULL, else w[e] for edge e of the pool's edge
 * list); argmax_dev[g] = the smallest k attaining it (NULL to skip).  Both
 * device arrays of num_graphs entries.  n up to 34; the work is 2^(n-1)
 * cut evaluations per graph (C(k) = C(complement of k)). */
int qs_cut_max(const qs_pool_desc *d, const double *w, double *max_dev, uint64_t *argmax_dev, void *stream);

/* Particle swarm over a pool (Particle Swarm / QAOA section, eq. (4)): graph
 * g has its own swarm of R = sets_per_graph particles; particle k of graph g
 * is pool circuit c = g R + k and its position is that circuit's angle
 * vector (D = 2p coordinates).  All arrays are caller-owned device memory. */
typedef struct qs_pso_swarm {
    double *pos;       /* [G * R * D] positions (the pool's angle vectors) */
    double *vel;       /* [G * R * D] velocities */
    double *pbest;     /* [G * R * D] best position each particle has evaluated */
    double *pbest_val; /* [G * R] <C> at pbest (-inf before the first round) */
    double *gbest;     /* [G * D] best position of each swarm */
    double *gbest_val; /* [G] */
    double *E;         /* [G * R] <C> at the current positions */
} qs_pso_swarm;

typedef struct qs_pso_params {
    double omega, phi_p, phi_g; /* the paper's study: 0.66, 1.6, 0.62 */
    int attract;                /* +1: pulled toward the bests, v += phi r (best - theta)
                                   (the standard form of the cited source); -1: the sign
                                   as printed in eq. (4), v += phi r (theta - best) */
} qs_pso_params;

/* Positions and velocities uniform in [0, 2 pi): coordinate d of particle c
 * takes Philox4x32-10(key = seed, counter = (c, d, 5, 0)) -> (x0..x3),
 * position 2 pi u53(x0, x1), velocity 2 pi u53(x2, x3), u53(lo, hi) =
 * ((hi << 32 | lo) >> 11) 2^-53.  Best values are set to -inf. */
int qs_pso_init(const qs_pool_desc *d, uint64_t seed, const qs_pso_swarm *sw, void *stream);

/* One round after the evaluations sw->E of the current positions: each
 * personal best takes the current position on strict improvement, each
 * swarm's global best the lowest-index particle with the largest personal
 * best if that beats it strictly; history_dev (device [G] or NULL) receives
 * gbest_val.  If move != 0 every particle then takes velocity eq. (4) with
 * scalars r_p = u53(x0, x1), r_g = u53(x2, x3) of Philox4x32-10(key = seed,
 * counter = (c, round, 4, 0)) and position theta + v. */
int qs_pso_step(const qs_pool_desc *d, const qs_pso_params *prm, int round, int move, uint64_t seed,
                const qs_pso_swarm *sw, double *history_dev, void *stream);

/* A whole swarm run on the device: init, then `rounds` rounds of (pool
 * forward evaluation of every particle, qs_pso_step with move = 1 except
 * after the last round).  history_dev: device [rounds * G], row r = the
 * global bests after round r.  ws: the pool workspace (qs_pool_workspace_bytes).
 * No host synchronisation between rounds. */
int qs_pso_run(const qs_pool_desc *d, const qs_pso_params *prm, int rounds, uint64_t seed, const qs_pso_swarm *sw,
               double *history_dev, void *ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------- noise trajectories */

/* Stochastic Pauli insertion unravelling the single-qubit depolarizing
 * channel (1-p) rho + (p/3)(X rho X + Y rho Y + Z rho Z) (paper: noise by
 * stochastic one-qubit gates averaged over the pool).  After each gate, for
 * each qubit it touches (q0, then q1), draw number `slot` of trajectory t is
 * Philox4x32-10(key = seed, counter = (t, slot, 3, 0)); a Pauli is inserted iff
 * x0 < floor(p 2^32), and it is 1 + floor(3 x1 / 2^32) (1 = X, 2 = Y, 3 = Z).
 * Every trajectory starts from |basis_index>. */
typedef struct qs_traj_out {
    double *z;          /* device [n_traj * n]: per-trajectory <Z_q>, or NULL */
    double *x;          /* device [n_traj * n]: per-trajectory <X_q>, or NULL */
    double *fid;        /* device [n_traj]: |<ideal|psi_t>|^2, ideal = the noiseless circuit, or NULL */
    double *prob_mean;  /* device [2^n]: trajectory mean of |a_k|^2, or NULL */
    int32_t *counts;    /* device [n_traj]: insertions per trajectory, or NULL */
    uint32_t *log;      /* device [n_traj * log_cap]: (slot << 2 | pauli) records, or NULL */
    int log_cap;
    const double *diag; /* device [2^n] diagonal observable d, or NULL */
    double *diag_val;   /* device [n_traj]: per-trajectory sum_k d_k |a_k|^2 (needs diag), or NULL */
} qs_traj_out;

/* Device workspace for qs_traj_run: n_traj + 2 states (the noiseless reference
 * for the fidelity keeps two, so that trajectories can start from its state
 * after the pass before their first insertion) plus per-gate Pauli frames. */
int qs_traj_workspace_bytes(int n, int dtype, int count, int n_traj, size_t *bytes);

/* gates: host list (1Q, C1Q, DIAG2, SWAP), 1 <= count <= 4096; 1 <= n <= 20;
 * 0 <= p_depol <= 1.  Inserted Paulis are tracked as a per-trajectory Pauli
 * frame (conjugating later gates and undone in the read-outs), so they add no
 * pass over the state.  The gate list is uploaded and the call waits for that
 * copy before returning (not capturable).  Outputs are trajectory-resolved;
 * means and convergence curves are reductions of them. */
int qs_traj_run(int n, int dtype, const qs_gate *gates, int count, uint64_t basis_index, int n_traj,
                double p_depol, uint64_t seed, const qs_traj_out *out, void *ws, size_t ws_bytes, void *stream);

/* Device workspace for qs_traj_run_noise: qs_traj_workspace_bytes plus one
 * 2x2 matrix per (trajectory, noise gate of the list). */
int qs_traj_noise_workspace_bytes(int n, int dtype, const qs_gate *gates, int count, int n_traj, size_t *bytes);

/* Noise models of a trajectory run. */
typedef struct qs_noise {
    double p_depol; /* Pauli insertion probability per touched qubit after each gate, as in qs_traj_run */
    double T1, T2;  /* timescales of the QS_G_NOISE gates: 0 < T2 <= 2 T1, or INFINITY (no decay) */
} qs_noise;

/* qs_traj_run with stochastic noise gates as well (Pool of multiple states:
 * noise by one-qubit rotations with random angles, T1/T2 timescales).  A
 * QS_G_NOISE gate of duration d on qubit q applies R_X(a_x), R_Y(a_y), R_Z(a_z),
 * R_P(a) = exp(-i a P / 2), with independent normal angles of variances d/T1,
 * d/T1 and 2d/T2 - d/T1; averaged over trajectories this scales the qubit's
 * Bloch vector by (e^{-d/T2}, e^{-d/T2}, e^{-d/T1}).  The normals come from
 * Box-Muller on Philox4x32-10(key = seed, counter = (t, gate index, 7, w)),
 * u1 = u53(x0, x1), u2 = u53(x2, x3), r = sqrt(-2 ln(1 - u1)): w = 0 gives
 * a_x = r cos(2 pi u2) and a_y = r sin(2 pi u2) (scaled), w = 1 gives a_z from
 * the cos branch.  Noise gates draw no insertion slots.  With noise gates
 * every trajectory is simulated (none shares the noiseless state). */
int qs_traj_run_noise(int n, int dtype, const qs_gate *gates, int count, uint64_t basis_index, int n_traj,
                      const qs_noise *noise, uint64_t seed, const qs_traj_out *out, void *ws, size_t ws_bytes, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* QSIM_H */
