// Pool of QAOA circuits of uneven size (the paper's pool of states, each
// circuit with its own parameters), run as one captured graph.
//
// The pool's circuits are grouped by qubit count.  Within a size class every
// graph has the same pass structure (only the edge lists differ), so one
// kernel launch per pass covers a whole batch of circuits of the class: block
// (c, tile) reads circuit c's pass descriptor and angle vector from device
// tables.  A batch holds as many circuits as the workspace fits.
//
// Tile size (TB in {10, 11, 12}: 16/32/64 KiB forward tiles) is chosen per
// size class by a small autotuner that times one batch with each candidate
// the first time a class is seen; choices are kept for the process (and in
// the file named by QSIM_AUTOTUNE_CACHE when set).
//
// The first qs_pool_run call for a given descriptor and set of buffers plans,
// tunes, uploads the tables and records the whole launch sequence into a
// hipGraph; later calls replay it with one hipGraphLaunch, reading the angle
// vectors that are then in device memory.
#include <cmath>
#include <cstdio>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "launch.h"
#include "qaoa.h"

#define QS_API extern "C" __attribute__((visibility("default")))

namespace qs {

struct PoolClass {
    int n = 0;
    std::vector<int> graphs;  // pool graph ids in this class
    QPlan proto;              // shape, kernel family and geometry shared by the class
    QPass *dev_passes = nullptr;  // [graph in class][np]
    int32_t *dev_map = nullptr;   // class-local circuit -> pool circuit id
    size_t circ_bytes = 0;
    int np = 0;
};

struct PoolPlan {
    std::vector<PoolClass> classes;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t last_use = 0;
};

static std::mutex g_pool_mu;
static std::map<std::string, PoolPlan> g_pool_plans;
static uint64_t g_pool_clock = 0;
// Plans kept at once; the least recently used one is released beyond this.
constexpr size_t kMaxPoolPlans = 32;

// Frees a plan's captured graph and device tables.  The device is synchronised
// first: a replay or a batch launch of the plan may still be queued.
static void free_pool_plan(PoolPlan &p) {
    (void)hipDeviceSynchronize();
    if (p.exec) (void)hipGraphExecDestroy(p.exec);
    if (p.graph) (void)hipGraphDestroy(p.graph);
    for (PoolClass &C : p.classes) {
        if (C.dev_passes) (void)hipFree(C.dev_passes);
        if (C.dev_map) (void)hipFree(C.dev_map);
        C.dev_passes = nullptr;
        C.dev_map = nullptr;
    }
    p.exec = nullptr;
    p.graph = nullptr;
}
static std::map<std::string, std::pair<int, int>> g_tb_choice;  // "n:p:sets:grad" -> (TB, r)

static std::string tb_key(int n, int p, int sets, bool grad) {
    return std::to_string(n) + ":" + std::to_string(p) + ":" + std::to_string(sets) + ":" + (grad ? "1" : "0");
}

static void load_tb_cache() {
    static bool loaded = false;
    if (loaded) return;
    loaded = true;
    const char *path = getenv("QSIM_AUTOTUNE_CACHE");
    if (!path) return;
    if (FILE *f = fopen(path, "r")) {
        char key[128];
        int tb, r;
        while (fscanf(f, "%127s %d %d", key, &tb, &r) == 3) g_tb_choice[key] = {tb, r};
        fclose(f);
    }
}

static void save_tb_choice(const std::string &key, QShape s) {
    const char *path = getenv("QSIM_AUTOTUNE_CACHE");
    if (!path) return;
    if (FILE *f = fopen(path, "a")) {
        fprintf(f, "%s %d %d\n", key.c_str(), s.TB, s.r);
        fclose(f);
    }
}

static QShape shape_of(int TB, int r) { return QShape{TB, TB >= 12 ? 9 : 8, r}; }

static int check_pool(const qs_pool_desc *d) {
    if (!d) return fail(QS_ERR_ARG, "null pool descriptor");
    if (d->num_graphs < 1 || d->sets_per_graph < 1) return fail(QS_ERR_ARG, "pool needs >= 1 graph and >= 1 angle set");
    if (d->p < 1 || d->p > 64) return fail(QS_ERR_ARG, "pool p must be in [1, 64]");
    if (!d->n_qubits || !d->edge_offset || !d->edges) return fail(QS_ERR_ARG, "null pool arrays");
    if ((long long)d->num_graphs * d->sets_per_graph > (1ll << 30)) return fail(QS_ERR_ARG, "too many pool circuits");
    if (d->edge_offset[0] != 0) return fail(QS_ERR_ARG, "edge_offset[0] must be 0");
    for (int g = 0; g < d->num_graphs; ++g) {
        const int n = d->n_qubits[g];
        if (n < 2 || n > 26) return fail(QS_ERR_ARG, "pool qubit counts must be in [2, 26]");
        const int ne = d->edge_offset[g + 1] - d->edge_offset[g];
        if (int rc = check_edges(n, ne, d->edges + 2 * (size_t)d->edge_offset[g])) return rc;
    }
    return QS_OK;
}

// Build the class's device tables for one tile shape.
static int build_class(const qs_pool_desc *d, PoolClass &C, QShape shape, bool grad) {
    std::vector<QPass> all;
    int max_edges = 0;
    QPlan plan;
    for (int g : C.graphs) {
        const int ne = d->edge_offset[g + 1] - d->edge_offset[g];
        max_edges = ne > max_edges ? ne : max_edges;
        if (int rc = build_qplan(C.n, d->p, ne, d->edges + 2 * (size_t)d->edge_offset[g], nullptr, shape, plan)) return rc;
        all.insert(all.end(), plan.passes.begin(), plan.passes.end());
    }
    C.proto.shape = plan.shape;
    C.proto.rt = plan.rt;
    C.proto.geo = plan.geo;
    C.proto.merged = plan.merged;  // the same pass structure for every graph of the class
    C.proto.map = plan.map;
    C.proto.geo.num_edges = max_edges;  // phase tables cover every graph of the class
    C.proto.passes = plan.passes;  // for the pass flags only (the same for every graph of the class); launches read dev_passes
    C.np = C.proto.geo.np;
    C.circ_bytes = qaoa_layout(C.proto.geo, grad).bytes;
    std::vector<int32_t> map;
    for (int g : C.graphs)
        for (int a = 0; a < d->sets_per_graph; ++a) map.push_back(g * d->sets_per_graph + a);
    if (C.dev_passes) (void)hipFree(C.dev_passes);
    if (C.dev_map) (void)hipFree(C.dev_map);
    QS_HIP(hipMalloc(&C.dev_passes, all.size() * sizeof(QPass)));
    QS_HIP(hipMemcpy(C.dev_passes, all.data(), all.size() * sizeof(QPass), hipMemcpyHostToDevice));
    QS_HIP(hipMalloc(&C.dev_map, map.size() * sizeof(int32_t)));
    QS_HIP(hipMemcpy(C.dev_map, map.data(), map.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    return QS_OK;
}

// All launches of one class, in batches that fit the workspace.
static int run_class(const qs_pool_desc *d, const PoolClass &C, const double *angles, double *E, double *grad, char *ws, size_t ws_bytes,
                     hipStream_t st, int max_circuits = -1) {
    const int total = (int)C.graphs.size() * d->sets_per_graph;
    const int limit = max_circuits > 0 && max_circuits < total ? max_circuits : total;
    const u64 fit = ws_bytes / C.circ_bytes;
    const int per = (int)(fit < (u64)limit ? fit : (u64)limit);
    for (int c0 = 0; c0 < limit; c0 += per) {
        const int nb = limit - c0 < per ? limit - c0 : per;
        QBatch B{};
        B.ws = ws;
        B.circ_bytes = C.circ_bytes;
        B.theta = angles;
        B.passes = C.dev_passes;
        B.circ_map = C.dev_map;
        B.c0 = c0;
        B.sets = d->sets_per_graph;
        B.np = C.np;
        if (int rc = launch_qaoa_pooled(C.proto, B, nb, E, grad, st)) return rc;
    }
    return QS_OK;
}

// Time one batch of the class with each tile-size candidate; keep the fastest.
static int autotune_class(const qs_pool_desc *d, PoolClass &C, const double *angles, double *E, double *grad, char *ws, size_t ws_bytes,
                          hipStream_t st) {
    load_tb_cache();
    const std::string key = tb_key(C.n, d->p, d->sets_per_graph, grad != nullptr);
    auto it = g_tb_choice.find(key);
    if (it != g_tb_choice.end()) return build_class(d, C, shape_of(it->second.first, it->second.second), grad != nullptr);
    const std::vector<QShape> cands = qaoa_candidate_shapes(C.n);
    if (getenv("QSIM_QAOA_TB") || cands.size() == 1) return build_class(d, C, qaoa_default_shape(C.n), grad != nullptr);
    hipEvent_t e0, e1;
    QS_HIP(hipEventCreate(&e0));
    QS_HIP(hipEventCreate(&e1));
    float best = 1e30f;
    QShape best_s = qaoa_default_shape(C.n);
    for (QShape s : cands) {
        if (int rc = build_class(d, C, s, grad != nullptr)) return rc;
        if (ws_bytes < C.circ_bytes) continue;
        const u64 fit = ws_bytes / C.circ_bytes;
        const int probe = (int)(fit < 64 ? fit : 64);
        // warm-up, then one timed batch
        if (int rc = run_class(d, C, angles, E, grad, ws, ws_bytes < C.circ_bytes * probe ? ws_bytes : C.circ_bytes * probe, st, probe)) return rc;
        QS_HIP(hipEventRecord(e0, st));
        if (int rc = run_class(d, C, angles, E, grad, ws, C.circ_bytes * probe, st, probe)) return rc;
        QS_HIP(hipEventRecord(e1, st));
        QS_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        QS_HIP(hipEventElapsedTime(&ms, e0, e1));
        ms /= (float)probe;
        if (ms < best) {
            best = ms;
            best_s = s;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    g_tb_choice[key] = {best_s.TB, best_s.r};
    save_tb_choice(key, best_s);
    return build_class(d, C, best_s, grad != nullptr);
}

static std::string pool_key(const qs_pool_desc *d, const void *angles, const void *E, const void *grad, const void *ws, size_t ws_bytes) {
    std::string k;
    auto add = [&](const void *p, size_t n) { k.append((const char *)p, n); };
    add(&d->num_graphs, sizeof(int));
    add(&d->sets_per_graph, sizeof(int));
    add(&d->p, sizeof(int));
    add(d->n_qubits, sizeof(int32_t) * d->num_graphs);
    add(d->edge_offset, sizeof(int32_t) * (d->num_graphs + 1));
    add(d->edges, sizeof(int32_t) * 2 * (size_t)d->edge_offset[d->num_graphs]);
    const void *ptrs[4] = {angles, E, grad, ws};
    add(ptrs, sizeof(ptrs));
    add(&ws_bytes, sizeof(ws_bytes));
    return k;
}

static size_t max_circ_bytes(const qs_pool_desc *d, bool grad) {
    size_t m = 0;
    for (int g = 0; g < d->num_graphs; ++g) {
        QPlan plan;
        const int ne = d->edge_offset[g + 1] - d->edge_offset[g];
        for (QShape s : qaoa_candidate_shapes(d->n_qubits[g])) {
            if (build_qplan(d->n_qubits[g], d->p, ne, d->edges + 2 * (size_t)d->edge_offset[g], nullptr, s, plan)) continue;  // shape unusable
            const size_t b = qaoa_layout(plan.geo, grad).bytes;
            m = b > m ? b : m;
        }
    }
    return m;
}

}  // namespace qs

using namespace qs;

QS_API int qs_pool_workspace_bytes(const qs_pool_desc *d, size_t *bytes) {
    try {
        if (int rc = check_pool(d)) return rc;
        if (!bytes) return fail(QS_ERR_ARG, "null output");
        *bytes = max_circ_bytes(d, true) * (size_t)d->sets_per_graph;
        return QS_OK;
    } catch (...) {
        return fail(QS_ERR_UNSUPPORTED, "unexpected internal error");
    }
}

QS_API int qs_pool_circuit_bytes(const qs_pool_desc *d, int with_grad, size_t *bytes) {
    try {
        if (int rc = check_pool(d)) return rc;
        if (!bytes) return fail(QS_ERR_ARG, "null output");
        *bytes = max_circ_bytes(d, with_grad != 0);
        return QS_OK;
    } catch (...) {
        return fail(QS_ERR_UNSUPPORTED, "unexpected internal error");
    }
}

QS_API int qs_pool_run(const qs_pool_desc *d, const double *angles_dev, double *E_dev, double *grad_dev, void *ws, size_t ws_bytes, void *stream) {
    try {
        if (int rc = check_pool(d)) return rc;
        if (!angles_dev || !E_dev || !ws) return fail(QS_ERR_ARG, "null angles, energies or workspace");
        if (ws_bytes < max_circ_bytes(d, grad_dev != nullptr)) return fail(QS_ERR_SIZE, "pool workspace smaller than one circuit of the largest size");
        hipStream_t st = (hipStream_t)stream;
        const bool use_graph = !(getenv("QSIM_POOL_GRAPH") && atoi(getenv("QSIM_POOL_GRAPH")) == 0);
        std::lock_guard<std::mutex> lk(g_pool_mu);
        const std::string key = pool_key(d, angles_dev, E_dev, grad_dev, ws, ws_bytes);
        auto it = g_pool_plans.find(key);
        if (it == g_pool_plans.end()) {
            PoolPlan plan;
            std::map<int, PoolClass> by_n;
            for (int g = 0; g < d->num_graphs; ++g) {
                PoolClass &C = by_n[d->n_qubits[g]];
                C.n = d->n_qubits[g];
                C.graphs.push_back(g);
            }
            for (auto &kv : by_n) {
                if (int rc = autotune_class(d, kv.second, angles_dev, E_dev, grad_dev, (char *)ws, ws_bytes, st)) return rc;
                plan.classes.push_back(kv.second);
            }
            if (use_graph) {
                hipStream_t cs;
                QS_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
                QS_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
                int rc = QS_OK;
                for (const PoolClass &C : plan.classes)
                    if (!rc) rc = run_class(d, C, angles_dev, E_dev, grad_dev, (char *)ws, ws_bytes, cs);
                hipGraph_t graph = nullptr;
                const hipError_t ec = hipStreamEndCapture(cs, &graph);
                (void)hipStreamDestroy(cs);
                if (rc) return rc;
                if (ec != hipSuccess) return hip_fail(ec, "pool capture");
                QS_HIP(hipGraphInstantiate(&plan.exec, graph, nullptr, nullptr, 0));
                plan.graph = graph;
            }
            if (g_pool_plans.size() >= kMaxPoolPlans) {
                auto lru = g_pool_plans.begin();
                for (auto j = g_pool_plans.begin(); j != g_pool_plans.end(); ++j)
                    if (j->second.last_use < lru->second.last_use) lru = j;
                free_pool_plan(lru->second);
                g_pool_plans.erase(lru);
            }
            it = g_pool_plans.emplace(key, std::move(plan)).first;
        }
        PoolPlan &plan = it->second;
        plan.last_use = ++g_pool_clock;
        if (plan.exec) {
            QS_HIP(hipGraphLaunch(plan.exec, st));
        } else {
            for (const PoolClass &C : plan.classes)
                if (int rc = run_class(d, C, angles_dev, E_dev, grad_dev, (char *)ws, ws_bytes, st)) return rc;
        }
        return QS_OK;
    } catch (...) {
        return fail(QS_ERR_UNSUPPORTED, "unexpected internal error");
    }
}

QS_API int qs_pool_release(const qs_pool_desc *d, const double *angles_dev, double *E_dev, double *grad_dev, void *ws, size_t ws_bytes) {
    try {
        if (int rc = check_pool(d)) return rc;
        std::lock_guard<std::mutex> lk(g_pool_mu);
        auto it = g_pool_plans.find(pool_key(d, angles_dev, E_dev, grad_dev, ws, ws_bytes));
        if (it == g_pool_plans.end()) return QS_OK;
        free_pool_plan(it->second);
        g_pool_plans.erase(it);
        return QS_OK;
    } catch (...) {
        return fail(QS_ERR_UNSUPPORTED, "unexpected internal error");
    }
}
