// C-ABI entry points of libqsim_hip.so: argument validation, handle
// management and dispatch to the launchers.  No C++ exception leaves this file.
#include <cmath>
#include <cstddef>
#include <new>

#include "launch.h"
#include "tile.h"

#define QS_API extern "C" __attribute__((visibility("default")))

namespace qs {

static_assert(sizeof(qs_gate) == 80 && offsetof(qs_gate, u) == 16, "qs_gate layout is part of the ABI");

static thread_local std::string t_last_error;

void set_error(const std::string &msg) { t_last_error = msg; }

int fail(int code, const std::string &msg) {
    t_last_error = msg;
    return code;
}

int hip_fail(hipError_t e, const char *where) {
    t_last_error = std::string(where) + ": " + hipGetErrorString(e);
    return QS_ERR_HIP;
}

static int check_state(const qs_state *s) {
    if (!s) return fail(QS_ERR_ARG, "null state handle");
    return QS_OK;
}

static int check_qubit(const qs_state *s, int q, const char *what) {
    if (q < 0 || q >= s->n) return fail(QS_ERR_ARG, std::string(what) + " qubit out of range");
    return QS_OK;
}

// Graph arguments are copied into the kernel-argument struct.
int make_graph(int n, const int32_t *edges, const double *w, int ne, Graph &g, Weights &wt) {
    if (!edges || ne < 1 || ne > kMaxEdges) return fail(QS_ERR_ARG, "edges: need 1..256 edges");
    g.ne = ne;
    g.weighted = w != nullptr;
    for (int e = 0; e < ne; ++e) {
        const int a = edges[2 * e], b = edges[2 * e + 1];
        if (a < 0 || b < 0 || a >= n || b >= n || a == b) return fail(QS_ERR_ARG, "edge endpoint out of range or self-loop");
        g.uv[e] = pack_edge(a, b);
        if (w) wt.w[e] = w[e];
    }
    return QS_OK;
}

}  // namespace qs

using namespace qs;

#define QS_GUARD_BEGIN try {
#define QS_GUARD_END                                                   \
    }                                                                  \
    catch (const std::bad_alloc &) {                                   \
        return fail(QS_ERR_SIZE, "host allocation failed");            \
    }                                                                  \
    catch (...) {                                                      \
        return fail(QS_ERR_UNSUPPORTED, "unexpected internal error");  \
    }

QS_API const char *qs_last_error(void) { return t_last_error.c_str(); }

QS_API int qs_state_create(int n, int dtype, void *dev_buf, size_t buf_bytes, void *stream, qs_state **out) {
    QS_GUARD_BEGIN
    if (!out || !dev_buf) return fail(QS_ERR_ARG, "null buffer or output pointer");
    *out = nullptr;
    if (dtype != QS_C64 && dtype != QS_C128) return fail(QS_ERR_DTYPE, "dtype must be QS_C64 or QS_C128");
    if (n < 1) return fail(QS_ERR_ARG, "n must be >= 1");
    const int nmax = dtype == QS_C128 ? QS_MAX_QUBITS_C128 : QS_MAX_QUBITS_C64;
    if (n > nmax) return fail(QS_ERR_SIZE, "n above the per-device limit");
    const size_t need = ((size_t)1 << n) * amp_bytes(dtype);
    if (buf_bytes < need) return fail(QS_ERR_SIZE, "state buffer smaller than 2^n amplitudes");
    if (((uintptr_t)dev_buf) % amp_bytes(dtype)) return fail(QS_ERR_ARG, "state buffer not aligned to the amplitude size");
    auto *s = new qs_state{};
    s->n = n;
    s->dtype = dtype;
    s->buf = dev_buf;
    s->bytes = buf_bytes;
    s->stream = (hipStream_t)stream;
    hipError_t e = hipGetDevice(&s->device);
    if (e == hipSuccess) e = hipMalloc((void **)&s->scratch, kScratchDoubles * sizeof(double));
    if (e != hipSuccess) {
        delete s;
        return hip_fail(e, "qs_state_create");
    }
    s->scratch_doubles = kScratchDoubles;
    *out = s;
    return QS_OK;
    QS_GUARD_END
}

QS_API int qs_state_destroy(qs_state *s) {
    QS_GUARD_BEGIN
    if (!s) return QS_OK;
    (void)hipStreamSynchronize(s->stream);
    free_plan_cache(s);
    (void)hipFree(s->scratch);
    delete s;
    return QS_OK;
    QS_GUARD_END
}

QS_API int qs_state_set_stream(qs_state *s, void *stream) {
    if (int rc = check_state(s)) return rc;
    s->stream = (hipStream_t)stream;
    return QS_OK;
}

QS_API int qs_sync(qs_state *s) {
    if (int rc = check_state(s)) return rc;
    QS_HIP(hipStreamSynchronize(s->stream));
    QS_HIP(hipGetLastError());
    return QS_OK;
}

QS_API int qs_init_basis(qs_state *s, uint64_t index) {
    if (int rc = check_state(s)) return rc;
    if (s->n < 64 && index >= (1ull << s->n)) return fail(QS_ERR_ARG, "basis index >= 2^n");
    return launch_init_basis(s, index);
}

QS_API int qs_init_uniform(qs_state *s) {
    if (int rc = check_state(s)) return rc;
    return launch_init_uniform(s);
}

QS_API int qs_init_random(qs_state *s, uint64_t seed) {
    if (int rc = check_state(s)) return rc;
    return launch_init_random(s, seed);
}

QS_API int qs_apply_1q(qs_state *s, int q, const double u[8]) {
    if (int rc = check_state(s)) return rc;
    if (int rc = check_qubit(s, q, "target")) return rc;
    if (!u) return fail(QS_ERR_ARG, "null matrix");
    return launch_apply_1q(s, q, u);
}

QS_API int qs_apply_c1q(qs_state *s, int c, int t, const double u[8]) {
    if (int rc = check_state(s)) return rc;
    if (int rc = check_qubit(s, c, "control")) return rc;
    if (int rc = check_qubit(s, t, "target")) return rc;
    if (c == t) return fail(QS_ERR_ARG, "control equals target");
    if (!u) return fail(QS_ERR_ARG, "null matrix");
    return launch_apply_c1q(s, c, t, u);
}

QS_API int qs_apply_diag2(qs_state *s, int q0, int q1, const double d[8]) {
    if (int rc = check_state(s)) return rc;
    if (int rc = check_qubit(s, q0, "first")) return rc;
    if (int rc = check_qubit(s, q1, "second")) return rc;
    if (q0 == q1) return fail(QS_ERR_ARG, "diagonal gate needs two distinct qubits");
    if (!d) return fail(QS_ERR_ARG, "null diagonal");
    return launch_apply_diag2(s, q0, q1, d);
}

QS_API int qs_apply_swap(qs_state *s, int a, int b) {
    if (int rc = check_state(s)) return rc;
    if (int rc = check_qubit(s, a, "first")) return rc;
    if (int rc = check_qubit(s, b, "second")) return rc;
    if (a == b) return fail(QS_ERR_ARG, "swap needs two distinct qubits");
    return launch_apply_swap(s, a, b);
}

QS_API int qs_apply_kq(qs_state *s, const int32_t *qubits, int k, const double *U_dev) {
    QS_GUARD_BEGIN
    if (int rc = check_state(s)) return rc;
    if (!qubits || !U_dev) return fail(QS_ERR_ARG, "null qubit list or matrix");
    if ((uintptr_t)U_dev % 16) return fail(QS_ERR_ARG, "matrix must be 16-byte aligned");
    if (k < 1 || k > 5) return fail(QS_ERR_ARG, "k-qubit gates need 1 <= k <= 5");
    if (k > s->n) return fail(QS_ERR_ARG, "more gate qubits than the register has");
    for (int m = 0; m < k; ++m) {
        if (int rc = check_qubit(s, qubits[m], "gate")) return rc;
        for (int j = 0; j < m; ++j)
            if (qubits[j] == qubits[m]) return fail(QS_ERR_ARG, "gate qubits must be distinct");
    }
    return launch_apply_kq(s, qubits, k, U_dev);
    QS_GUARD_END
}

QS_API int qs_collapse(qs_state *s, int q, int outcome, double *prob_dev) {
    if (int rc = check_state(s)) return rc;
    if (int rc = check_qubit(s, q, "measured")) return rc;
    if (outcome != 0 && outcome != 1) return fail(QS_ERR_ARG, "outcome must be 0 or 1");
    return launch_measure(s, q, outcome, 0, nullptr, prob_dev);
}

QS_API int qs_measure(qs_state *s, int q, uint64_t seed, int32_t *outcome_dev, double *prob_dev) {
    if (int rc = check_state(s)) return rc;
    if (int rc = check_qubit(s, q, "measured")) return rc;
    return launch_measure(s, q, -1, seed, outcome_dev, prob_dev);
}

namespace qs {
int validate_gates(int n, const qs_gate *gates, int count, bool allow_noise) {
    if (count < 0) return fail(QS_ERR_ARG, "negative gate count");
    if (count > 0 && !gates) return fail(QS_ERR_ARG, "null gate list");
    for (int k = 0; k < count; ++k) {
        const qs_gate &g = gates[k];
        const bool two = g.kind != QS_G_1Q && g.kind != QS_G_NOISE;
        if (g.kind < QS_G_1Q || g.kind > (allow_noise ? QS_G_NOISE : QS_G_SWAP))
            return fail(QS_ERR_ARG, "gate " + std::to_string(k) + ": unknown kind");
        if (g.kind == QS_G_NOISE && !(g.u[0] >= 0.0 && g.u[0] < INFINITY))
            return fail(QS_ERR_ARG, "gate " + std::to_string(k) + ": noise duration must be finite and >= 0");
        if (g.q0 < 0 || g.q0 >= n || (two && (g.q1 < 0 || g.q1 >= n || g.q1 == g.q0)))
            return fail(QS_ERR_ARG, "gate " + std::to_string(k) + ": qubit out of range or repeated");
    }
    return QS_OK;
}
}  // namespace qs

QS_API int qs_apply_block(qs_state *s, const qs_gate *gates, int count) {
    QS_GUARD_BEGIN
    if (int rc = check_state(s)) return rc;
    if (int rc = validate_gates(s->n, gates, count, false)) return rc;
    return run_block(s, gates, count);
    QS_GUARD_END
}

QS_API int qs_block_passes(int n, int dtype, const qs_gate *gates, int count, int *passes) {
    QS_GUARD_BEGIN
    if (!passes) return fail(QS_ERR_ARG, "null output pointer");
    if (dtype != QS_C64 && dtype != QS_C128) return fail(QS_ERR_DTYPE, "dtype must be QS_C64 or QS_C128");
    if (n < 1) return fail(QS_ERR_ARG, "n must be >= 1");
    if (n > (dtype == QS_C128 ? QS_MAX_QUBITS_C128 : QS_MAX_QUBITS_C64)) return fail(QS_ERR_SIZE, "n above the per-device limit");
    if (int rc = validate_gates(n, gates, count, false)) return rc;
    *passes = block_pass_count(n, dtype, gates, count);
    return QS_OK;
    QS_GUARD_END
}

QS_API int qs_apply_cut_phase(qs_state *s, const int32_t *edges, const double *w, int num_edges, double gamma) {
    if (int rc = check_state(s)) return rc;
    Graph g;
    Weights wt;
    if (int rc = make_graph(s->n, edges, w, num_edges, g, wt)) return rc;
    return launch_cut_phase(s, g, w ? &wt : nullptr, gamma);
}

QS_API int qs_prob_one(qs_state *s, int q, double *out_dev) {
    if (int rc = check_state(s)) return rc;
    if (int rc = check_qubit(s, q, "measured")) return rc;
    if (!out_dev) return fail(QS_ERR_ARG, "null output");
    return launch_marginals(s, kMargProbOne, q, out_dev);
}

QS_API int qs_expect_z_all(qs_state *s, double *out_dev) {
    if (int rc = check_state(s)) return rc;
    if (!out_dev) return fail(QS_ERR_ARG, "null output");
    return launch_marginals(s, kMargZAll, 0, out_dev);
}

QS_API int qs_norm2(qs_state *s, double *out_dev) {
    if (int rc = check_state(s)) return rc;
    if (!out_dev) return fail(QS_ERR_ARG, "null output");
    return launch_marginals(s, kMargNorm, 0, out_dev);
}

QS_API int qs_expect_cut(qs_state *s, const int32_t *edges, const double *w, int num_edges, double *out_dev) {
    if (int rc = check_state(s)) return rc;
    if (!out_dev) return fail(QS_ERR_ARG, "null output");
    Graph g;
    Weights wt;
    if (int rc = make_graph(s->n, edges, w, num_edges, g, wt)) return rc;
    return launch_expect_cut(s, g, w ? &wt : nullptr, out_dev);
}

QS_API int qs_expect_diag(qs_state *s, const double *d_dev, double *out_dev) {
    if (int rc = check_state(s)) return rc;
    if (!out_dev || !d_dev) return fail(QS_ERR_ARG, "null diagonal or output");
    return launch_expect_diag(s, d_dev, out_dev);
}

QS_API int qs_expect_pauli(qs_state *s, uint64_t xmask, uint64_t zmask, double *out_dev) {
    if (int rc = check_state(s)) return rc;
    if (!out_dev) return fail(QS_ERR_ARG, "null output");
    if (s->n < 64 && ((xmask | zmask) >> s->n)) return fail(QS_ERR_ARG, "Pauli mask has bits >= n");
    return launch_expect_pauli(s, xmask, zmask, out_dev);
}

QS_API int qs_inner(qs_state *a, qs_state *b, double *out_dev) {
    if (int rc = check_state(a)) return rc;
    if (int rc = check_state(b)) return rc;
    if (!out_dev) return fail(QS_ERR_ARG, "null output");
    if (a->dtype != b->dtype) return fail(QS_ERR_DTYPE, "states of different dtype");
    if (a->n != b->n) return fail(QS_ERR_ARG, "states of different qubit count");
    return launch_inner(a, b, out_dev);
}

QS_API int qs_sample(qs_state *s, int64_t shots, uint64_t seed, uint64_t *out_dev) {
    if (int rc = check_state(s)) return rc;
    if (shots < 0 || shots > ((int64_t)1 << 32)) return fail(QS_ERR_ARG, "shots must be in [0, 2^32]");
    if (shots > 0 && !out_dev) return fail(QS_ERR_ARG, "null output");
    return launch_sample(s, shots, seed, out_dev);
}
