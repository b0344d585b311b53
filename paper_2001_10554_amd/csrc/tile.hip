// Fused gate blocks: several consecutive gates applied per read+write pass.
//
// A pass works on tiles.  The pass owns a set T of tb qubits (tb <= 12 for
// c128, 13 for c64, i.e. a 64 KiB tile); each workgroup loads the 2^tb
// amplitudes that share one value of the other n - tb bits into LDS, applies
// every gate of the pass there (one barrier per gate) and writes the tile
// back.  T always contains the lowest qubits so that each load/store
// instruction covers whole 128-byte lines.  A gate can join a pass when its
// target qubits lie in T: one-qubit and controlled gates need their target in
// T (a control outside T is constant over the tile and is resolved per tile);
// diagonal gates need nothing; SWAP needs both qubits in T.
//
// The sequential order of the gate list is kept: a pass takes the longest
// prefix of the remaining gates whose targets fit, so the result equals
// applying the gates one after the other.
#include <algorithm>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "launch.h"
#include "tile.h"

namespace qs {

template <typename R, int TBMAX>
__global__ __launch_bounds__(kTileThreads) void k_tile_pass(cx<R> *__restrict__ psi, DPass P, const DGate *__restrict__ gates) {
    constexpr int NT = kTileThreads, PER = (1 << TBMAX) / NT;
    __shared__ cx<R> sh[1 << TBMAX];
    __shared__ SGate<R> sg[kStage];
    const int tb = P.tb;
    const u64 base = pass_base(P, blockIdx.x);
    tile_load<R, NT, PER, false>(sh, psi, P, base, false, 0);
    __syncthreads();
    if (tb >= 3) {
        run_sweeps<R, NT, ((1 << (TBMAX - 3)) + NT - 1) / NT>(sh, sg, tb, base, gates, P.gate_begin, P.gate_count,
                                                              [](int, const DGate &x, GateVals<R> &gv, int &, int &) {
                                                                  gv = gate_vals<R>(x.kind, x.u);
                                                                  return true;
                                                              });
    } else {
        for (int gi = 0; gi < P.gate_count; ++gi) {
            const DGate &g = gates[P.gate_begin + gi];
            lds_apply_gate<R, NT>(sh, 1ull << tb, base, g.kind, g.p0, g.p1, g.q0, g.q1, 1, g.u);
        }
    }
    tile_store<R, NT, PER, false>(sh, psi, P, base);
}

// ------------------------------------------------------------------ planning

// A plan is keyed by the structure of its gate list (kinds, qubits and the
// exact-value classes the generated code specialises on), not by the values:
// a variational loop that changes angles reuses the plan and its compiled
// code and only uploads the new values.
struct Plan {
    std::vector<DPass> passes;
    std::vector<DGate> dg;        // plan order; gidx = index in the caller's list
    // Run-time compiled passes (empty: the interpreter kernel runs the plan).
    JitFns jit;
    // Device copy of what the kernels read: the gate values, 8 per gate in
    // plan order in the state's type (compiled passes), or the DGate records
    // (interpreter).  Uploads go through a pinned staging buffer with an
    // asynchronous copy on the state's stream, only when the values change.
    void *dev = nullptr;
    void *stage = nullptr;
    std::vector<char> last;       // bytes of the last upload
    hipEvent_t staged = nullptr;  // recorded after the last upload's copy
    uint64_t last_use = 0;
};

// Block plans kept per state; the least recently used one is released beyond this.
constexpr size_t kMaxBlockPlans = 32;

// QSIM_BLOCK_PATH=interp keeps fused blocks on the interpreter kernel (read
// when a plan is built).
static bool jit_wanted() {
    const char *e = getenv("QSIM_BLOCK_PATH");
    return !(e && std::string(e) == "interp");
}

int block_pass_count(int n, int dtype, const qs_gate *g, int count) {
    int tb = tile_bits_max(dtype), low = 0;
    if (jit_wanted()) jit_tile_shape(n, dtype, tb, low);
    std::vector<DPass> passes;
    std::vector<DGate> dg;
    make_plan(n, dtype, tb, g, count, passes, dg, 0, 0, low);
    return (int)passes.size();
}

struct PlanCache {
    std::unordered_map<std::string, Plan> plans;
    uint64_t clock = 0;
};

// The caller has synchronised the state's stream (no kernel of the plan is queued).
static void free_plan(Plan &p) {
    if (p.staged) (void)hipEventSynchronize(p.staged);
    (void)hipFree(p.dev);
    (void)hipHostFree(p.stage);
    if (p.staged) (void)hipEventDestroy(p.staged);
    p.dev = p.stage = nullptr;
    p.staged = nullptr;
    if (p.jit.mod) (void)hipModuleUnload(p.jit.mod);
    p.jit.mod = nullptr;
    p.jit.fn.clear();
}

// Cut a pass's gates into sweeps whose non-diagonal targets span at most 3
// tile bits, padded with the highest free tile bits.  A sweep is filled
// greedily: scanning the pass's remaining gates in order, a gate joins if its
// targets fit and it commutes with every gate it overtakes (disjoint qubits,
// or both diagonal); the sweep's gates keep their relative order.  So
// consecutive gates on changing targets (a one-qubit gate on every qubit
// followed by a CNOT chain) share sweeps that a plain prefix split would
// spread over twice as many.  Each gate keeps its list index (gidx).
static void make_sweeps(int tb, DGate *d, int cnt) {
    auto one = [](const DGate &x) { return x.kind == QS_G_1Q || x.kind == QS_G_NOISE; };
    auto touch = [&](const DGate &x) { return (1ull << x.q0) | (one(x) ? 0ull : 1ull << x.q1); };
    std::vector<DGate> in(d, d + cnt), out;
    std::vector<int> rem(cnt), later;
    for (int i = 0; i < cnt; ++i) rem[i] = i;
    out.reserve(cnt);
    while (!rem.empty()) {
        int gp[3], ng = 0;
        auto has = [&](int p) {
            for (int a = 0; a < ng; ++a)
                if (gp[a] == p) return true;
            return false;
        };
        u64 left_any = 0, left_nondiag = 0;
        const size_t first = out.size();
        later.clear();
        for (int i : rem) {
            const DGate &x = in[i];
            int need[2], nn = 0;
            if (one(x)) need[nn++] = x.p0;
            else if (x.kind == QS_G_C1Q) need[nn++] = x.p1;
            else if (x.kind == QS_G_SWAP) { need[nn++] = x.p0; need[nn++] = x.p1; }
            int fresh = 0;
            for (int a = 0; a < nn; ++a) fresh += !has(need[a]) && !(a == 1 && need[1] == need[0]);
            const bool diag = x.kind == QS_G_DIAG2;
            const bool commutes = (touch(x) & (diag ? left_nondiag : left_any)) == 0;
            if (commutes && ng + fresh <= 3 && out.size() - first < (size_t)kStage) {
                for (int a = 0; a < nn; ++a)
                    if (!has(need[a])) gp[ng++] = need[a];
                out.push_back(x);
            } else {
                later.push_back(i);
                left_any |= touch(x);
                if (!diag) left_nondiag |= touch(x);
            }
        }
        rem.swap(later);
        for (int p = tb - 1; ng < 3 && p >= 0; --p)
            if (!has(p)) gp[ng++] = p;
        std::sort(gp, gp + 3);
        auto slot = [&](int p) -> int8_t {
            for (int a = 0; a < 3; ++a)
                if (gp[a] == p) return (int8_t)a;
            return (int8_t)-1;
        };
        DGate &h = out[first];
        h.run = (int16_t)(out.size() - first);
        for (int a = 0; a < 3; ++a) h.g[a] = (int8_t)gp[a];
        for (size_t t = first; t < out.size(); ++t) {
            out[t].s0 = out[t].p0 >= 0 ? slot(out[t].p0) : (int8_t)-1;
            out[t].s1 = out[t].p1 >= 0 ? slot(out[t].p1) : (int8_t)-1;
            if (t != first) out[t].run = 0;
        }
    }
    std::copy(out.begin(), out.end(), d);
}

// Split the list into passes (see the file comment) and encode each gate's
// qubits as tile-bit positions of its pass.
void make_plan(int n, int dtype, int tile_bits, const qs_gate *g, int count, std::vector<DPass> &passes, std::vector<DGate> &dg, int cap,
               int cap_region, int low_bits) {
    // Tiles of up to 13 bits (the interpreter's 12 for c128, or 13 for its
    // compiled passes with 1024-thread workgroups).
    const int tbmax = std::min(std::min(tile_bits, 13), n);
    const int tblow = low_bits > 0 && low_bits < tbmax ? low_bits : 0;
    // Contiguous low qubits in every tile: 128-byte rows, 256-byte rows for a
    // 13-bit c128 tile.
    auto rows = [&](int tb) { return std::min(dtype == QS_C128 ? (tb > 12 ? 4 : 3) : 4, tb); };
    std::vector<int16_t> nidx(count);
    for (int j = 0, c = 0; j < count; ++j) {
        nidx[j] = (int16_t)c;
        c += g[j].kind == QS_G_NOISE;
    }
    // Gate lists and tile masks of the passes; with commute = false a pass is
    // the longest prefix of the remaining list that fits.
    auto split = [&](bool commute, std::vector<std::vector<int>> &lists, std::vector<u64> &tiles, std::vector<int> &tbs) {
        std::vector<int> rem(count), take, later;
        for (int j = 0; j < count; ++j) rem[j] = j;
        // One pass of tb bits from the remaining gates.
        auto collect = [&](int tb, u64 &T) {
            T = (1ull << rows(tb)) - 1;
            u64 left_any = 0, left_nondiag = 0;  // qubits of the gates left for later passes
            const int placed = count - (int)rem.size();
            const size_t limit = cap > 0 && placed < cap_region ? (size_t)cap : (size_t)count;
            take.clear();
            later.clear();
            for (int j : rem) {
                const qs_gate &x = g[j];
                const bool one = x.kind == QS_G_1Q || x.kind == QS_G_NOISE, diag = x.kind == QS_G_DIAG2;
                const u64 touch = (1ull << x.q0) | (one ? 0ull : 1ull << x.q1);
                u64 need = 0;
                if (one) need = 1ull << x.q0;
                else if (x.kind == QS_G_C1Q) need = 1ull << x.q1;
                else if (x.kind == QS_G_SWAP) need = touch;
                const bool blocked = take.size() >= limit || (commute ? (touch & (diag ? left_nondiag : left_any)) != 0 : !later.empty());
                if (!blocked && __builtin_popcountll(T | need) <= tb) {
                    T |= need;
                    take.push_back(j);
                } else {
                    later.push_back(j);
                    left_any |= touch;
                    if (!diag) left_nondiag |= touch;
                }
            }
        };
        while (!rem.empty()) {
            u64 T;
            int tb = tbmax;
            // With low_bits: a pass whose targets all lie among the lowest
            // low_bits qubits keeps that smaller, contiguous tile.
            if (tblow) {
                collect(tblow, T);
                if ((T >> tblow) == 0) tb = tblow;
            }
            if (tb == tbmax) collect(tbmax, T);
            lists.push_back(take);
            tiles.push_back(T);
            tbs.push_back(tb);
            rem.swap(later);
        }
    };
    // Reordering pays only where it saves passes: with as many passes, the
    // list-order split keeps the early passes short, which trajectories
    // starting from the noiseless run's state prefer.
    std::vector<std::vector<int>> lists, lists_c;
    std::vector<u64> tiles, tiles_c;
    std::vector<int> tbs, tbs_c;
    split(false, lists, tiles, tbs);
    split(true, lists_c, tiles_c, tbs_c);
    if (lists_c.size() < lists.size()) {
        lists.swap(lists_c);
        tiles.swap(tiles_c);
        tbs.swap(tbs_c);
    }
    for (size_t pi = 0; pi < lists.size(); ++pi) {
        const std::vector<int> &take = lists[pi];
        u64 T = tiles[pi];
        // Fill the tile up to its size with the lowest unused qubits.
        for (int q = 0; q < n && __builtin_popcountll(T) < tbs[pi]; ++q) T |= 1ull << q;
        DPass P{};
        P.tb = 0;
        int pos[64];
        for (int q = 0; q < n; ++q) {
            if ((T >> q) & 1) {
                pos[q] = P.tb;
                P.T[P.tb++] = (uint8_t)q;
            } else {
                pos[q] = -1;
                P.rest[P.nrest++] = (uint8_t)q;
            }
        }
        for (int k = 0; k < 16; ++k) {
            u64 o = 0;
            const u64 m = (u64)k * kTileThreads;
            for (int b = 0; b < P.tb; ++b)
                if ((m >> b) & 1) o |= 1ull << P.T[b];
            P.hi[k] = o;
        }
        P.gate_begin = (int)dg.size();
        P.gate_count = (int)take.size();
        for (int j : take) {
            DGate d{};
            d.kind = g[j].kind;
            d.q0 = (int8_t)g[j].q0;
            const bool one = g[j].kind == QS_G_1Q || g[j].kind == QS_G_NOISE;
            d.q1 = (int8_t)(one ? 0 : g[j].q1);
            d.p0 = (int8_t)pos[g[j].q0];
            d.p1 = (int8_t)(one ? -1 : pos[g[j].q1]);
            memcpy(d.u, g[j].u, sizeof(d.u));
            d.s0 = d.s1 = -1;
            d.nidx = nidx[j];
            d.gidx = j;
            dg.push_back(d);
        }
        if (P.tb >= 3) make_sweeps(P.tb, dg.data() + P.gate_begin, P.gate_count);
        passes.push_back(P);
    }
}

static std::mutex g_plan_mu;

static std::string structure_key(const qs_state *s, const qs_gate *gates, int count, bool jit) {
    std::string key;
    auto add = [&](int32_t v) { key.append((const char *)&v, sizeof v); };
    add(s->n);
    add(s->dtype);
    add(jit);
    for (int i = 0; i < count; ++i) {
        add(gates[i].kind);
        add(gates[i].q0);
        add(gates[i].kind == QS_G_1Q ? -1 : gates[i].q1);
        add(gate_value_class(gates[i].kind, gates[i].u));
    }
    return key;
}

// Bytes the plan's kernels read for this gate list (values in plan order).
static std::vector<char> plan_bytes(const Plan &p, const qs_gate *gates, int dtype) {
    std::vector<char> out;
    if (!p.jit.fn.empty()) {
        const size_t rs = dtype == QS_C128 ? sizeof(double) : sizeof(float);
        out.resize(p.dg.size() * 8 * rs);
        for (size_t i = 0; i < p.dg.size(); ++i)
            for (int k = 0; k < 8; ++k) {
                const double u = gates[p.dg[i].gidx].u[k];
                if (dtype == QS_C128) memcpy(out.data() + (8 * i + k) * rs, &u, rs);
                else {
                    const float f = (float)u;
                    memcpy(out.data() + (8 * i + k) * rs, &f, rs);
                }
            }
    } else {
        std::vector<DGate> dg = p.dg;
        for (DGate &d : dg) memcpy(d.u, gates[d.gidx].u, sizeof d.u);
        out.resize(dg.size() * sizeof(DGate));
        memcpy(out.data(), dg.data(), out.size());
    }
    return out;
}

int run_block(qs_state *s, const qs_gate *gates, int count) {
    if (count == 0) return QS_OK;
    const bool want_jit = jit_wanted();
    const std::string key = structure_key(s, gates, count, want_jit);
    std::lock_guard<std::mutex> lk(g_plan_mu);
    if (!s->plan_cache) s->plan_cache = new PlanCache();
    auto *cache = (PlanCache *)s->plan_cache;
    auto it = cache->plans.find(key);
    if (it == cache->plans.end()) {
        if (cache->plans.size() >= kMaxBlockPlans) {
            auto lru = cache->plans.begin();
            for (auto j = cache->plans.begin(); j != cache->plans.end(); ++j)
                if (j->second.last_use < lru->second.last_use) lru = j;
            QS_HIP(hipStreamSynchronize(s->stream));  // its kernels may still be queued
            free_plan(lru->second);
            cache->plans.erase(lru);
        }
        Plan p;
        int jtb = tile_bits_max(s->dtype), jlow = 0;
        if (want_jit) jit_tile_shape(s->n, s->dtype, jtb, jlow);
        make_plan(s->n, s->dtype, jtb, gates, count, p.passes, p.dg, 0, 0, jlow);
        const std::string src = want_jit ? jit_block_source(p.passes, p.dg, s->dtype) : std::string();
        std::vector<unsigned> nt;
        for (const DPass &P : p.passes) nt.push_back((unsigned)jit_threads(s->dtype, P.tb));
        if (src.empty() || jit_block_functions(src, (int)p.passes.size(), s->device, p.jit, "qs_pass", nt) != QS_OK) {
            p.jit = JitFns{};
            // The interpreter runs tiles of tile_bits_max bits only (make_plan appends).
            if (jtb != tile_bits_max(s->dtype) || jlow) {
                p.passes.clear();
                p.dg.clear();
                make_plan(s->n, s->dtype, tile_bits_max(s->dtype), gates, count, p.passes, p.dg);
            }
        }
        const size_t nb = plan_bytes(p, gates, s->dtype).size();
        QS_HIP(hipMalloc(&p.dev, nb));
        if (hipHostMalloc(&p.stage, nb, hipHostMallocDefault) != hipSuccess) {
            free_plan(p);
            return fail(QS_ERR_HIP, "hipHostMalloc of the plan's staging buffer failed");
        }
        if (hipEventCreateWithFlags(&p.staged, hipEventDisableTiming) != hipSuccess) {
            free_plan(p);
            return fail(QS_ERR_HIP, "hipEventCreate failed");
        }
        it = cache->plans.emplace(key, std::move(p)).first;
    }
    Plan &plan = it->second;
    plan.last_use = ++cache->clock;
    std::vector<char> bytes = plan_bytes(plan, gates, s->dtype);
    if (bytes != plan.last) {
        QS_HIP(hipEventSynchronize(plan.staged));  // the previous upload has left the staging buffer
        memcpy(plan.stage, bytes.data(), bytes.size());
        QS_HIP(hipMemcpyAsync(plan.dev, plan.stage, bytes.size(), hipMemcpyHostToDevice, s->stream));
        QS_HIP(hipEventRecord(plan.staged, s->stream));
        plan.last.swap(bytes);
    }
    if (!plan.jit.fn.empty()) {
        for (size_t pi = 0; pi < plan.passes.size(); ++pi) {
            unsigned ntiles = 1u << plan.passes[pi].nrest;
            const unsigned grid = std::min(ntiles, plan.jit.max_blocks[pi]);
            void *psi = s->buf, *vals = plan.dev;
            void *args[] = {&psi, &vals, &ntiles};
            QS_HIP(hipModuleLaunchKernel(plan.jit.fn[pi], grid, 1, 1, plan.jit.threads[pi], 1, 1, 0, s->stream, args, nullptr));
        }
        return QS_OK;
    }
    for (const DPass &P : plan.passes) {
        const unsigned grid = 1u << P.nrest;
        if (s->dtype == QS_C128)
            hipLaunchKernelGGL((k_tile_pass<double, 12>), dim3(grid), dim3(kTileThreads), 0, s->stream, (cx<double> *)s->buf, P,
                               (const DGate *)plan.dev);
        else
            hipLaunchKernelGGL((k_tile_pass<float, 13>), dim3(grid), dim3(kTileThreads), 0, s->stream, (cx<float> *)s->buf, P,
                               (const DGate *)plan.dev);
        QS_LAUNCH_CHECK("tile_pass");
    }
    return QS_OK;
}

size_t block_plan_count(const qs_state *s) { return s->plan_cache ? ((const PlanCache *)s->plan_cache)->plans.size() : 0; }

void free_plan_cache(qs_state *s) {
    if (!s->plan_cache) return;
    auto *cache = (PlanCache *)s->plan_cache;
    for (auto &kv : cache->plans) free_plan(kv.second);
    delete cache;
    s->plan_cache = nullptr;
}

}  // namespace qs
