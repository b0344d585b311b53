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

struct Plan {
    std::vector<DPass> passes;
    DGate *dev_gates = nullptr;
};

struct PlanCache {
    std::unordered_map<std::string, Plan> plans;
};

// Cut a pass's gates into sweeps: maximal runs whose non-diagonal targets
// span at most 3 tile bits, padded with the lowest free tile bits.
static void make_sweeps(int tb, DGate *d, int cnt) {
    int i = 0;
    while (i < cnt) {
        int gp[3], ng = 0;
        auto has = [&](int p) {
            for (int a = 0; a < ng; ++a)
                if (gp[a] == p) return true;
            return false;
        };
        int j = i;
        for (; j < cnt; ++j) {
            int need[2], nn = 0;
            const int k = d[j].kind;
            if (k == QS_G_1Q || k == QS_G_NOISE) need[nn++] = d[j].p0;
            else if (k == QS_G_C1Q) need[nn++] = d[j].p1;
            else if (k == QS_G_SWAP) { need[nn++] = d[j].p0; need[nn++] = d[j].p1; }
            int fresh = 0;
            for (int a = 0; a < nn; ++a) fresh += !has(need[a]) && !(a == 1 && need[1] == need[0]);
            if (ng + fresh > 3 || j - i == kStage) break;
            for (int a = 0; a < nn; ++a)
                if (!has(need[a])) gp[ng++] = need[a];
        }
        for (int p = 0; ng < 3 && p < tb; ++p)
            if (!has(p)) gp[ng++] = p;
        std::sort(gp, gp + 3);
        auto slot = [&](int p) -> int8_t {
            for (int a = 0; a < 3; ++a)
                if (gp[a] == p) return (int8_t)a;
            return (int8_t)-1;
        };
        d[i].run = (int16_t)(j - i);
        for (int a = 0; a < 3; ++a) d[i].g[a] = (int8_t)gp[a];
        for (int t = i; t < j; ++t) {
            d[t].s0 = d[t].p0 >= 0 ? slot(d[t].p0) : (int8_t)-1;
            d[t].s1 = d[t].p1 >= 0 ? slot(d[t].p1) : (int8_t)-1;
        }
        i = j;
    }
}

// Split the list into passes (see the file comment) and encode each gate's
// qubits as tile-bit positions of its pass.
void make_plan(int n, int dtype, int tile_bits, const qs_gate *g, int count, std::vector<DPass> &passes, std::vector<DGate> &dg, int cap,
               int cap_region) {
    const int tbmax = std::min(std::min(tile_bits, tile_bits_max(dtype)), n);
    const int r = std::min(dtype == QS_C128 ? 3 : 4, tbmax);  // contiguous low qubits: 128-byte rows
    std::vector<int16_t> nidx(count);
    for (int j = 0, c = 0; j < count; ++j) {
        nidx[j] = (int16_t)c;
        c += g[j].kind == QS_G_NOISE;
    }
    // Gate lists and tile masks of the passes; with commute = false a pass is
    // the longest prefix of the remaining list that fits.
    auto split = [&](bool commute, std::vector<std::vector<int>> &lists, std::vector<u64> &tiles) {
        std::vector<int> rem(count), take, later;
        for (int j = 0; j < count; ++j) rem[j] = j;
        while (!rem.empty()) {
            u64 T = (1ull << r) - 1;
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
                if (!blocked && __builtin_popcountll(T | need) <= tbmax) {
                    T |= need;
                    take.push_back(j);
                } else {
                    later.push_back(j);
                    left_any |= touch;
                    if (!diag) left_nondiag |= touch;
                }
            }
            lists.push_back(take);
            tiles.push_back(T);
            rem.swap(later);
        }
    };
    // Reordering pays only where it saves passes: with as many passes, the
    // list-order split keeps the early passes short, which trajectories
    // starting from the noiseless run's state prefer.
    std::vector<std::vector<int>> lists, lists_c;
    std::vector<u64> tiles, tiles_c;
    split(false, lists, tiles);
    split(true, lists_c, tiles_c);
    if (lists_c.size() < lists.size()) {
        lists.swap(lists_c);
        tiles.swap(tiles_c);
    }
    for (size_t pi = 0; pi < lists.size(); ++pi) {
        const std::vector<int> &take = lists[pi];
        u64 T = tiles[pi];
        // Fill the tile up to tbmax with the lowest unused qubits.
        for (int q = 0; q < n && __builtin_popcountll(T) < tbmax; ++q) T |= 1ull << q;
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

int run_block(qs_state *s, const qs_gate *gates, int count) {
    if (count == 0) return QS_OK;
    std::string key((const char *)gates, (size_t)count * sizeof(qs_gate));
    key.append((const char *)&s->n, sizeof(int));
    key.append((const char *)&s->dtype, sizeof(int));
    Plan *plan = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_plan_mu);
        if (!s->plan_cache) s->plan_cache = new PlanCache();
        auto *cache = (PlanCache *)s->plan_cache;
        auto it = cache->plans.find(key);
        if (it == cache->plans.end()) {
            Plan p;
            std::vector<DGate> dg;
            make_plan(s->n, s->dtype, tile_bits_max(s->dtype), gates, count, p.passes, dg);
            QS_HIP(hipMalloc(&p.dev_gates, dg.size() * sizeof(DGate)));
            QS_HIP(hipMemcpy(p.dev_gates, dg.data(), dg.size() * sizeof(DGate), hipMemcpyHostToDevice));
            it = cache->plans.emplace(std::move(key), std::move(p)).first;
        }
        plan = &it->second;
    }
    for (const DPass &P : plan->passes) {
        const unsigned grid = 1u << P.nrest;
        if (s->dtype == QS_C128)
            hipLaunchKernelGGL((k_tile_pass<double, 12>), dim3(grid), dim3(kTileThreads), 0, s->stream, (cx<double> *)s->buf, P, plan->dev_gates);
        else
            hipLaunchKernelGGL((k_tile_pass<float, 13>), dim3(grid), dim3(kTileThreads), 0, s->stream, (cx<float> *)s->buf, P, plan->dev_gates);
        QS_LAUNCH_CHECK("tile_pass");
    }
    return QS_OK;
}

void free_plan_cache(qs_state *s) {
    if (!s->plan_cache) return;
    auto *cache = (PlanCache *)s->plan_cache;
    for (auto &kv : cache->plans) (void)hipFree(kv.second.dev_gates);
    delete cache;
    s->plan_cache = nullptr;
}

}  // namespace qs
