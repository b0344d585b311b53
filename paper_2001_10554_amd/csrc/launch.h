// Host-side launchers shared between the translation units of libqsim_hip.so.
// Each returns a QS_* status.  They assume arguments were validated by the
// C-ABI layer (api.hip).
#pragma once

#include "common.h"

namespace qs {

// init.hip / gates.hip
int launch_init_basis(qs_state *s, u64 index);
int launch_init_uniform(qs_state *s);
int launch_init_random(qs_state *s, u64 seed);
int launch_apply_1q(qs_state *s, int q, const double *u);
int launch_apply_c1q(qs_state *s, int c, int t, const double *u);
int launch_apply_diag2(qs_state *s, int q0, int q1, const double *d);
int launch_apply_swap(qs_state *s, int a, int b);
int launch_cut_phase(qs_state *s, const Graph &g, const Weights *w, double gamma);
int launch_scale(qs_state *s, const double *factor_dev);

// reduce.hip
enum MarginalMode { kMargNorm = 0, kMargZAll = 1, kMargProbOne = 2, kMargInvSqrt = 3 };
int launch_marginals(qs_state *s, int mode, int q, double *out_dev);
int launch_expect_cut(qs_state *s, const Graph &g, const Weights *w, double *out_dev);
int launch_expect_diag(qs_state *s, const double *d_dev, double *out_dev);
int launch_expect_pauli(qs_state *s, u64 xmask, u64 zmask, double *out_dev);
int launch_inner(qs_state *a, qs_state *b, double *out_dev);
int launch_sample(qs_state *s, int64_t shots, u64 seed, u64 *out_dev);
// Sampling of a register given by pointer: scratch holds at least
// 2 * 2^(n - sample_chunk_bits(n)) + 1 doubles (chunk sums, their prefix, the
// last nonzero chunk), all overwritten before they are read.
int sample_chunk_bits(int n);
int launch_sample_buf(int n, int dtype, const void *buf, double *scratch, hipStream_t st, int64_t shots, u64 seed, u64 *out_dev);

// measure.hip
int launch_measure(qs_state *s, int q, int outcome, u64 seed, int32_t *outcome_dev, double *prob_dev);
int launch_apply_kq(qs_state *s, const int32_t *qubits, int k, const double *U_dev);

// tile.hip
int run_block(qs_state *s, const qs_gate *gates, int count);
void free_plan_cache(qs_state *s);

}  // namespace qs
