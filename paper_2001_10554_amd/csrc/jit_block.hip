// Fused-block passes as straight-line code generated per plan and compiled at
// run time (hiprtc).
//
// The interpreter kernel (k_tile_pass) decides at run time, gate by gate,
// which kind of gate a staged record holds and which register slots it
// touches; the compiler has to keep one register assignment for the group's
// amplitudes across every branch, and it does so with copies at every merge.
// Here the plan's structure (tile qubits, sweeps, each gate's kind, slots and
// control position) is written out as source, so every gate becomes its plain
// arithmetic on named values: a general 2x2 gate is its 16 multiply-adds per
// pair, a permutation gate (X, CNOT, SWAP with the control in the group) only
// renames values, and a diagonal entry equal to 1 costs nothing.  Gate values
// stay data: the kernel reads them from a table (scalar loads), so a plan with
// new angles but the same structure reuses the compiled code.
//
// Each workgroup is persistent: it walks tiles blockIdx.x, + gridDim.x, ...
// and prefetches the next tile's amplitudes into registers while the current
// tile's sweeps run, so the HBM stream overlaps the arithmetic.  Every pass
// has its own tile size (complex128: 12 bits for a tile of the lowest qubits,
// 13 bits with longer rows for the others), workgroup size and LDS swizzle;
// workgroup barriers sit only between LDS phases whose wavefront footprints
// differ, and a pass over one contiguous stretch of the state streams it
// non-temporally.
#include <hip/hiprtc.h>

#include <cstdio>
#include <cstdlib>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "launch.h"
#include "tile.h"

namespace qs {

namespace {

std::string S(long long v) { return std::to_string(v); }

std::string hex(u64 v) {
    char b[32];
    snprintf(b, sizeof b, "0x%llxull", (unsigned long long)v);
    return b;
}

// sum over b < nb of ((x >> b) & 1) << map[b], with runs of consecutive
// positions mapped to consecutive bits as one shift-and-mask each.
std::string deposit(const std::string &x, const uint8_t *map, int nb) {
    std::string e;
    int b = 0;
    while (b < nb) {
        int len = 1;
        while (b + len < nb && map[b + len] == map[b] + len) ++len;
        const u64 mask = len >= 64 ? ~0ull : ((1ull << len) - 1);
        const std::string term = "(((" + x + ") >> " + S(b) + ") & " + hex(mask) + ") << " + S(map[b]);
        e += (e.empty() ? "(" : " | (") + term + ")";
        b += len;
    }
    return e.empty() ? std::string("0ull") : e;
}

enum Cls { kGeneral, kPermX, kDiagonal, kIdentity };

// Structure of a 2x2 matrix, decided on its exact entries.
Cls classify(const double *u) {
    const bool off0 = u[2] == 0 && u[3] == 0 && u[4] == 0 && u[5] == 0;
    if (off0 && u[0] == 1 && u[1] == 0 && u[6] == 1 && u[7] == 0) return kIdentity;
    if (off0) return kDiagonal;
    if (u[0] == 0 && u[1] == 0 && u[6] == 0 && u[7] == 0 && u[2] == 1 && u[3] == 0 && u[4] == 1 && u[5] == 0) return kPermX;
    return kGeneral;
}

// Entry e of a diagonal two-qubit gate: 1 = exactly 1, -1 = exactly -1, 0 = other.
int diag_entry_class(const double *u, int e) {
    const double re = u[2 * e], im = u[2 * e + 1];
    return re == 1 && im == 0 ? 1 : (re == -1 && im == 0 ? -1 : 0);
}

// A value source for one bit of an amplitude's index within a sweep: a
// compile-time constant (a group slot), a per-lane bool, or a uniform bool.
struct Bit {
    int konst = -1;    // 0 / 1 when known for amplitude j
    std::string var;   // otherwise the bool expression's variable
};

struct Gen {
    int dtype;
    int G;          // groups of 8 per thread
    bool traj = false;  // trajectory passes: values per trajectory (every gate general), C1Q control value from tcv
    std::string o;
    int uid = 0;
    std::string fresh(const char *p) { return std::string(p) + S(uid++); }
    std::string U(int gi, int k) const { return "vv[" + S(8 * gi + k) + "]"; }

    // Bit of amplitude j of group g for tile position p / slot s / qubit q.
    Bit bit(int j, int s, int p, int q, std::vector<std::string> &lane_vars, std::string &uni_var, int g) {
        Bit b;
        if (s >= 0) {
            b.konst = (j >> s) & 1;
        } else if (p >= 0) {
            if (lane_vars[g].empty()) {
                lane_vars[g] = fresh("c");
                o += "      const bool " + lane_vars[g] + " = ((m" + S(g) + " >> " + S(p) + ") & 1u) != 0u;\n";
            }
            b.var = lane_vars[g];
        } else {
            if (uni_var.empty()) {
                uni_var = fresh("w");
                o += "      const bool " + uni_var + " = ((base >> " + S(q) + ") & 1ull) != 0ull;\n";
            }
            b.var = uni_var;
        }
        return b;
    }

    // The pair (names[j], names[k]) under a 2x2 gate of class c with values
    // of plan gate gi, applied only where `cond` holds ("" = always).
    void pair(std::string &x, std::string &y, Cls c, int gi, const std::string &cond) {
        if (c == kIdentity) return;
        if (c == kPermX) {
            if (cond.empty()) {
                std::swap(x, y);
            } else {
                const std::string a = fresh("x"), b = fresh("x");
                o += "      const C " + a + " = " + cond + " ? " + y + " : " + x + ";\n";
                o += "      const C " + b + " = " + cond + " ? " + x + " : " + y + ";\n";
                x = a;
                y = b;
            }
            return;
        }
        const std::string a = fresh("x"), b = fresh("x");
        if (c == kDiagonal) {
            o += "      const C " + a + " = cm(" + x + ", " + U(gi, 0) + ", " + U(gi, 1) + ");\n";
            o += "      const C " + b + " = cm(" + y + ", " + U(gi, 6) + ", " + U(gi, 7) + ");\n";
        } else {
            o += "      const C " + a + " = row(" + U(gi, 0) + ", " + U(gi, 1) + ", " + U(gi, 2) + ", " + U(gi, 3) + ", " + x + ", " + y + ");\n";
            o += "      const C " + b + " = row(" + U(gi, 4) + ", " + U(gi, 5) + ", " + U(gi, 6) + ", " + U(gi, 7) + ", " + x + ", " + y + ");\n";
        }
        if (cond.empty()) {
            x = a;
            y = b;
        } else {
            const std::string a2 = fresh("x"), b2 = fresh("x");
            o += "      const C " + a2 + " = " + cond + " ? " + a + " : " + x + ";\n";
            o += "      const C " + b2 + " = " + cond + " ? " + b + " : " + y + ";\n";
            x = a2;
            y = b2;
        }
    }

    // One gate of a sweep on every group of the thread.
    void gate(const DGate &d, int gi, std::vector<std::vector<std::string>> &nm) {
        std::vector<std::string> lane0(G), lane1(G);
        std::string uni0, uni1;
        if (d.kind == QS_G_1Q || (traj && d.kind == QS_G_NOISE)) {
            if (traj && d.pad0 == 2) return;  // a noise gate folded into the gate before it
            const Cls c = traj ? kGeneral : classify(d.u);
            for (int g = 0; g < G; ++g)
                for (int j = 0; j < 8; ++j)
                    if (!((j >> d.s0) & 1)) pair(nm[g][j], nm[g][j | (1 << d.s0)], c, gi, "");
        } else if (d.kind == QS_G_C1Q) {
            const Cls c = traj ? kGeneral : classify(d.u);
            // Trajectories: the control value the gate fires on (an X in the
            // frame on the control flips it) is per trajectory.
            std::string cv;
            if (traj) {
                cv = fresh("v");
                o += "      const bool " + cv + " = tcv[" + S(gi) + "] != 0;\n";
            }
            for (int g = 0; g < G; ++g)
                for (int j = 0; j < 8; ++j) {
                    if ((j >> d.s1) & 1) continue;
                    const Bit b = bit(j, d.s0, d.p0, d.q0, lane0, uni0, g);
                    std::string cond;
                    if (!traj) {
                        if (b.konst == 0) continue;
                        cond = b.konst == 1 ? "" : b.var;
                    } else if (b.konst >= 0) {
                        cond = b.konst ? cv : "!" + cv;
                    } else {
                        cond = "(" + b.var + " == " + cv + ")";
                    }
                    pair(nm[g][j], nm[g][j | (1 << d.s1)], c, gi, cond);
                }
        } else if (d.kind == QS_G_DIAG2) {
            // Entry index 2 b1 + b0; entries equal to 1 are skipped, -1 negates
            // (blocks only: a trajectory's frame permutes the entries).
            auto entry_cls = [&](int e) { return traj ? 0 : diag_entry_class(d.u, e); };
            for (int g = 0; g < G; ++g)
                for (int j = 0; j < 8; ++j) {
                    const Bit b0 = bit(j, d.s0, d.p0, d.q0, lane0, uni0, g);
                    const Bit b1 = bit(j, d.s1, d.p1, d.q1, lane1, uni1, g);
                    std::string &x = nm[g][j];
                    const std::string y = fresh("x");
                    if (b0.konst >= 0 && b1.konst >= 0) {
                        const int e = 2 * b1.konst + b0.konst, ec = entry_cls(e);
                        if (ec == 1) continue;
                        if (ec == -1) o += "      const C " + y + " = -" + x + ";\n";
                        else o += "      const C " + y + " = cm(" + x + ", " + U(gi, 2 * e) + ", " + U(gi, 2 * e + 1) + ");\n";
                    } else {
                        // Select the entry's parts with the runtime bits.
                        auto pick = [&](int part) {
                            auto ent = [&](int e) { return U(gi, 2 * e + part); };
                            auto over0 = [&](int hi) {
                                if (b0.konst >= 0) return ent(2 * hi + b0.konst);
                                return "(" + b0.var + " ? " + ent(2 * hi + 1) + " : " + ent(2 * hi) + ")";
                            };
                            if (b1.konst >= 0) return over0(b1.konst);
                            return "(" + b1.var + " ? " + over0(1) + " : " + over0(0) + ")";
                        };
                        o += "      const C " + y + " = cm(" + x + ", " + pick(0) + ", " + pick(1) + ");\n";
                    }
                    x = y;
                }
        } else if (d.kind == QS_G_SWAP) {
            const int a = d.s0, b = d.s1;
            for (int g = 0; g < G; ++g)
                for (int j = 0; j < 8; ++j)
                    if (((j >> a) & 1) && !((j >> b) & 1)) std::swap(nm[g][j], nm[g][j ^ (1 << a) ^ (1 << b)]);
        }
    }
};

}  // namespace

int gate_value_class(int kind, const double *u) {
    if (kind == QS_G_1Q || kind == QS_G_C1Q) return (int)classify(u);
    if (kind == QS_G_DIAG2) {
        int c = 0;
        for (int e = 0; e < 4; ++e) c |= (diag_entry_class(u, e) + 1) << (2 * e);
        return c;
    }
    return 0;
}

void jit_tile_shape(int n, int dtype, int &tile_bits, int &low_bits) {
    // QSIM_JIT_TB=12 or 13: one tile size for every pass (for comparisons).
    static const int env_tb = [] {
        const char *e = getenv("QSIM_JIT_TB");
        return e ? atoi(e) : 0;
    }();
    tile_bits = tile_bits_max(dtype);
    low_bits = 0;
    if (dtype != QS_C128 || n < kJitMixedMinQubits || env_tb == 12) return;
    tile_bits = 13;
    if (env_tb != 13) low_bits = 12;
}

int jit_threads(int dtype, int tile_bits) { return dtype == QS_C128 && tile_bits == 13 ? 1024 : kTileThreads; }

// Source of one kernel per pass (qs_pass0, qs_pass1, ...) for passes whose
// tile is full (tb = a tile size the generator supports).  Returns "" if a
// pass does not qualify (the caller then uses the interpreter).
std::string jit_block_source(const std::vector<DPass> &passes, const std::vector<DGate> &dg, int dtype) {
    // Code-shape knobs (for tuning runs): QSIM_JIT_PREFETCH=0 loads each tile
    // straight into LDS instead of prefetching the next one into registers;
    // QSIM_JIT_WAVES=w asks the compiler to fit w waves per SIMD (0: no limit).
    auto env = [](const char *k, int dflt) {
        const char *e = getenv(k);
        return e ? atoi(e) : dflt;
    };
    const bool prefetch = env("QSIM_JIT_PREFETCH", 1) != 0;
    // QSIM_JIT_BARRIERS=1: a workgroup barrier between every two LDS phases
    // (see wave_pos below).
    const bool all_barriers = env("QSIM_JIT_BARRIERS", 0) != 0;
    // QSIM_JIT_INREGS=0: always load tiles with the top three tile bits as
    // register bits (see in_grp below).
    const bool in_regs = env("QSIM_JIT_INREGS", 1) != 0;
    const int waves = env("QSIM_JIT_WAVES", 4);
    // QSIM_JIT_ORDER=k (k > 0): the tile counter's first k bits go to the k
    // lowest non-tile qubits and its other bits to the remaining non-tile
    // qubits from the highest down, so that the tiles in flight at one time
    // spread over distant parts of the state instead of one contiguous stretch.
    const int order_k = env("QSIM_JIT_ORDER", 0);
    // QSIM_JIT_XCD=1: workgroup b (on XCD b mod 8) starts at tile
    // (b mod 8) * (grid / 8) + b / 8, so that neighbouring tiles run on one
    // XCD at the same time.
    const bool xcd = env("QSIM_JIT_XCD", 0) != 0;
    // Non-temporal state loads and stores for passes whose tile is one
    // contiguous stretch of the state (tile bit b = qubit b), ordinary ones
    // for the others.  Measured on a 30-qubit register, one pass with
    // register-renaming gates: 12-bit contiguous tiles 6.76 -> 6.33 ms, 13-bit
    // tiles of 256-byte rows 7.20 -> 8.57 ms.  QSIM_JIT_NT=0 / 1 forces
    // ordinary / non-temporal accesses for every pass.
    const int nt_mode = env("QSIM_JIT_NT", -1);
    bool nt = false;  // set per pass
    auto ld = [&](const std::string &addr) { return nt ? "__builtin_nontemporal_load(psi + (" + addr + "))" : "psi[" + addr + "]"; };
    auto stv = [&](const std::string &addr, const std::string &v) {
        return nt ? "__builtin_nontemporal_store(" + v + ", psi + (" + addr + "));\n" : "psi[" + addr + "] = " + v + ";\n";
    };
    static const int kSwz128[12] = {1, 2, 4, 8, 15, 12, 9, 3, 6, 14, 6, 0};
    static const int kSwz128w[13] = {1, 2, 4, 8, 15, 11, 13, 4, 8, 11, 5, 8, 6};
    static const int kSwz64[13] = {1, 2, 4, 8, 16, 31, 26, 22, 1, 0, 14, 9, 20};
    const int SB = dtype == QS_C128 ? 4 : 5;
    auto supported = [&](int tb) { return dtype == QS_C128 ? tb == 12 || tb == 13 : tb == 13; };
    auto pattern = [&](int tb) { return dtype == QS_C128 ? (tb == 13 ? kSwz128w : kSwz128) : kSwz64; };
    bool used[14] = {};
    for (const DPass &P : passes) {
        if (!supported(P.tb)) return "";
        used[P.tb] = true;
    }
    Gen gen;
    gen.dtype = dtype;
    std::string &o = gen.o;
    o += dtype == QS_C128 ? "typedef double R;\n" : "typedef float R;\n";
    o += "typedef __attribute__((address_space(4))) const R CR;\n";
    o += "typedef R C __attribute__((ext_vector_type(2)));\n"
         "__device__ __forceinline__ C row(R a, R b, R c, R d, C x, C y) {\n"
         "  C r; r.x = a * x.x - b * x.y + c * y.x - d * y.y; r.y = a * x.y + b * x.x + c * y.y + d * y.x; return r; }\n"
         "__device__ __forceinline__ C cm(C x, R a, R b) { C r; r.x = a * x.x - b * x.y; r.y = a * x.y + b * x.x; return r; }\n"
         "__device__ __forceinline__ unsigned ins(unsigned x, int b) { return ((x >> b) << (b + 1)) | (x & ((1u << b) - 1u)); }\n"
         "#define LDS(off) (*(C *)((char *)sh + (off)))\n";
    // LDS accesses take the swizzled slot as a byte offset, so that an access
    // at (group base) ^ (constant) is one XOR (the shift to bytes is applied
    // to the base once and folded into the constants).
    const int SH = dtype == QS_C128 ? 4 : 3;
    // LDS slot of tile index m: m ^ hsw(m), hsw XOR-ing a fixed pattern into
    // the low SB bits for each set bit of m at or above SB (a bijection).  The
    // b128 (c128) / b64 (c64) accesses of 16 / 32 lanes are served together;
    // with these patterns the lanes of every sweep whose group bits are three
    // consecutive tile bits (and of the load/store layout) reach 2^SB distinct
    // slots modulo 2^SB, i.e. distinct banks (found by search over all
    // patterns; 189 of the 220 possible group-bit triples of a 12-bit c128
    // tile, 251 of 286 for a 13-bit one).
    // (one function per tile size: hsw12, hsw13)
    for (int tb = 12; tb <= 13; ++tb) {
        if (!used[tb]) continue;
        o += "__device__ __forceinline__ unsigned hsw" + S(tb) + "(unsigned m) {\n  unsigned h = 0u;\n";
        for (int p = SB; p < tb; ++p)
            if (pattern(tb)[p]) o += "  h ^= ((m >> " + S(p) + ") & 1u) ? " + S(pattern(tb)[p]) + "u : 0u;\n";
        o += "  return h;\n}\n";
    }
    for (size_t pi = 0; pi < passes.size(); ++pi) {
        const DPass &P = passes[pi];
        // This pass's tile size, workgroup size and swizzle.
        const int TB = P.tb, NT = jit_threads(dtype, TB), TS = 1 << TB, PER = TS / NT;
        int TTB = 0;  // thread bits
        while ((1 << TTB) < NT) ++TTB;
        if ((1 << TTB) != NT || PER < 8 || PER % 8 || TTB < 6) return "";
        const int *swz_pat = pattern(TB);
        auto hsw = [&](u32 m) {
            u32 h = 0;
            for (int p = SB; p < TB; ++p)
                if ((m >> p) & 1) h ^= (u32)swz_pat[p];
            return h;
        };
        const std::string HSW = "hsw" + S(TB);
        gen.G = (TS / 8) / NT;
        {
            bool contiguous = true;
            for (int b = 0; b < TB; ++b) contiguous = contiguous && P.T[b] == b;
            nt = nt_mode >= 0 ? nt_mode != 0 : contiguous;
        }
        o += "extern \"C\" __global__ void __launch_bounds__(" + S(NT) + ")";
        if (waves > 0) o += " __attribute__((amdgpu_waves_per_eu(" + S(waves) + ")))";
        o += " qs_pass" + S((long long)pi) + "(C *__restrict__ psi, const R *__restrict__ v, unsigned ntiles) {\n";
        o += "  __shared__ C sh[" + S(TS) + "];\n";
        o += "  const unsigned t = threadIdx.x, st = (t ^ " + HSW + "(t)) << " + S(SH) + ";\n";
        o += "  const unsigned long long dt = " + deposit("(unsigned long long)t", P.T, TTB) + ";\n";
        std::vector<u64> hi(PER);
        for (int k = 0; k < PER; ++k) {
            u64 off = 0;
            for (int b = TTB; b < TB; ++b)
                if (((u64)k << TTB >> b) & 1) off |= 1ull << P.T[b];
            hi[k] = off;
        }
        // Sweeps of the pass: (first gate, run, group bits).
        struct Sw {
            int begin, run, g0, g1, g2;
        };
        std::vector<Sw> sw;
        for (int gi = P.gate_begin; gi < P.gate_begin + P.gate_count; gi += dg[gi].run)
            sw.push_back({gi, dg[gi].run, dg[gi].g[0], dg[gi].g[1], dg[gi].g[2]});
        // Load and store layouts.  By default the top three tile bits are the
        // register bits (thread t, register k: tile index t + NT k).  Loads
        // use the first sweep's group bits instead when they all lie above
        // the tile's contiguous row (so a wavefront still reads whole rows)
        // and a thread holds one group: the first sweep then runs on the
        // loaded registers, without the tile's first trip through LDS and its
        // barrier.  Stores use the last sweep's group bits on the same terms.
        const int row_bits = dtype == QS_C128 ? (TB > 12 ? 4 : 3) : 4;
        auto own_layout = [&](const Sw &w) {
            return in_regs && gen.G == 1 && w.g0 >= row_bits && !(w.g0 == TB - 3 && w.g1 == TB - 2 && w.g2 == TB - 1);
        };
        const bool in_first = !sw.empty() && own_layout(sw.front());
        const bool out_last = !sw.empty() && own_layout(sw.back());
        std::vector<u64> hio(8, 0);
        if (out_last) {
            const Sw &f = sw.back();
            uint8_t q[16];
            int nq = 0;
            for (int p = 0; p < TB; ++p)
                if (p != f.g0 && p != f.g1 && p != f.g2) q[nq++] = P.T[p];
            o += "  const unsigned long long dto = " + deposit("(unsigned long long)t", q, nq) + ";\n";
            for (int k = 0; k < 8; ++k)
                hio[k] = ((k & 1) ? 1ull << P.T[f.g0] : 0) | ((k & 2) ? 1ull << P.T[f.g1] : 0) | ((k & 4) ? 1ull << P.T[f.g2] : 0);
        }
        std::vector<u64> hii = hi;
        if (in_first) {
            const Sw &f = sw.front();
            uint8_t q[16];
            int nq = 0;
            for (int p = 0; p < TB; ++p)
                if (p != f.g0 && p != f.g1 && p != f.g2) q[nq++] = P.T[p];
            o += "  const unsigned long long dti = " + deposit("(unsigned long long)t", q, nq) + ";\n";
            for (int k = 0; k < PER; ++k)
                hii[k] = ((k & 1) ? 1ull << P.T[f.g0] : 0) | ((k & 2) ? 1ull << P.T[f.g1] : 0) | ((k & 4) ? 1ull << P.T[f.g2] : 0);
        } else {
            o += "  const unsigned long long dti = dt;\n";
        }
        uint8_t rest_order[40];
        for (int b = 0; b < P.nrest; ++b) rest_order[b] = P.rest[b];
        if (order_k > 0 && order_k < P.nrest)
            for (int b = order_k; b < P.nrest; ++b) rest_order[b] = P.rest[P.nrest - 1 - (b - order_k)];
        const std::string dep_tile = deposit("(unsigned long long)tile", rest_order, P.nrest);
        const std::string dep_next = deposit("(unsigned long long)nx", rest_order, P.nrest);
        o += "  C pre[" + S(PER) + "];\n";
        if (xcd)
            o += "  unsigned tile = (gridDim.x & 7u) ? blockIdx.x : (blockIdx.x & 7u) * (gridDim.x >> 3) + (blockIdx.x >> 3);\n";
        else
            o += "  unsigned tile = blockIdx.x;\n";
        if (prefetch) {
            o += "  if (tile < ntiles) {\n    const unsigned long long b0 = " + dep_tile + ";\n";
            for (int k = 0; k < PER; ++k) o += "    pre[" + S(k) + "] = " + ld("b0 | dti | " + hex(hii[k])) + ";\n";
            o += "  }\n";
        }
        const size_t body_at = o.size();  // the loop header goes here
        // Opaque copies of the thread index and the value table per tile, so
        // that the sweeps' LDS addresses and gate values are formed where they
        // are used instead of being hoisted out of the loop, which would hold
        // every sweep's addresses in registers at once.  The table is read
        // through the constant address space: its uniform entries then come
        // from scalar loads, which do not share the vector-memory counter
        // with the prefetch and the stores (a generic pointer gives flat
        // loads, and every sweep would wait for the whole prefetch).
        o += "    unsigned tl = t; asm volatile(\"\" : \"+v\"(tl));\n";
        o += "    CR *vv; { unsigned long long a_ = (unsigned long long)v; asm volatile(\"\" : \"+s\"(a_)); vv = (CR *)a_; }\n";
        o += "    const unsigned long long base = " + dep_tile + ";\n";
        // A sweep whose group bits are the tile's top three positions holds
        // exactly the amplitudes of the load/store layout (thread t, register
        // k: tile index t + 512 k): the first such sweep runs on the loaded
        // registers and the last one stores its registers, each saving one
        // trip through LDS and a barrier.  (The first sweep also runs on the
        // loaded registers with the load layout of in_first.)
        auto on_top = [&](const Sw &w) { return w.g0 == TB - 3 && w.g1 == TB - 2 && w.g2 == TB - 1; };
        const bool first_regs = !sw.empty() && (on_top(sw.front()) || in_first);
        const bool last_regs = !sw.empty() && (on_top(sw.back()) || out_last);
        auto hi_of = [&](u32 mhigh) {  // state offset of the tile bits of mhigh above the thread bits
            u64 off = 0;
            for (int b = TTB; b < TB; ++b)
                if ((mhigh >> b) & 1) off |= 1ull << P.T[b];
            return off;
        };
        auto grp_off = [&](const Sw &w, int j) {
            return ((u32)(j & 1) << w.g0) | ((u32)((j >> 1) & 1) << w.g1) | ((u32)((j >> 2) & 1) << w.g2);
        };
        // Tile positions that select the wavefront in an LDS phase (a sweep, or
        // w = nullptr: the load/store layout, thread t and register k at tile
        // index t + NT k): thread bits 6..TTB-1 land on the non-group
        // positions of ranks 6..TTB-1.  Where two consecutive phases have the
        // same positions, every wavefront reads only slots it wrote itself;
        // LDS runs one wavefront's instructions in order, so a wavefront-level
        // fence replaces the workgroup barrier there.
        auto wave_pos = [&](const Sw *w) {
            u32 h = 0;
            for (int p = 0, rank = 0; p < TB; ++p) {
                if (w && (p == w->g0 || p == w->g1 || p == w->g2)) continue;
                if (rank >= 6 && rank < TTB) h |= 1u << p;
                ++rank;
            }
            return h;
        };
        auto sync = [&](const char *ind, u32 from, u32 to) {
            if (all_barriers || from != to) o += std::string(ind) + "__syncthreads();\n";
            else
                o += std::string(ind) + "__builtin_amdgcn_fence(__ATOMIC_RELEASE, \"wavefront\"); __builtin_amdgcn_wave_barrier(); "
                                        "__builtin_amdgcn_fence(__ATOMIC_ACQUIRE, \"wavefront\");\n";
        };
        const u32 h_io = wave_pos(nullptr);
        // Layout of the first LDS access of the next tile.
        const u32 h_next_tile = first_regs ? wave_pos(&sw.front()) : h_io;
        auto issue_prefetch = [&]() {
            if (!prefetch) return;
            o += "    { const unsigned nx = tile + gridDim.x;\n      if (nx < ntiles) {\n        const unsigned long long nb = " + dep_next + ";\n";
            for (int k = 0; k < PER; ++k) o += "        pre[" + S(k) + "] = " + ld("nb | dti | " + hex(hii[k])) + ";\n";
            o += "      }\n    }\n";
        };
        if (!prefetch)
            for (int k = 0; k < PER; ++k) o += "    pre[" + S(k) + "] = " + ld("base | dti | " + hex(hii[k])) + ";\n";
        if (!first_regs) {
            for (int k = 0; k < PER; ++k) o += "    LDS(st ^ " + S(((u32)(k * NT) ^ hsw((u32)(k * NT))) << SH) + "u) = pre[" + S(k) + "];\n";
            if (sw.empty()) o += "    __syncthreads();\n";
            else sync("    ", h_io, wave_pos(&sw.front()));
            issue_prefetch();
        }
        for (size_t si = 0; si < sw.size(); ++si) {
            const Sw &w = sw[si];
            const bool from_regs = si == 0 && first_regs, to_global = si + 1 == sw.size() && last_regs;
            o += "    {\n";
            std::vector<std::vector<std::string>> nm(gen.G, std::vector<std::string>(8));
            for (int g = 0; g < gen.G; ++g) {
                o += "      const unsigned m" + S(g) + " = ins(ins(ins(tl + " + S(g * NT) + "u, " + S(w.g0) + "), " + S(w.g1) + "), " + S(w.g2) + ");\n";
                if (!from_regs || !to_global) o += "      const unsigned s" + S(g) + " = (m" + S(g) + " ^ " + HSW + "(m" + S(g) + ")) << " + S(SH) + ";\n";
                for (int j = 0; j < 8; ++j) {
                    nm[g][j] = gen.fresh("x");
                    if (from_regs)  // register k of the load layout holds amplitude k of the group
                        o += "      const C " + nm[g][j] + " = pre[" + S(in_first ? j : (g * NT + grp_off(w, j)) >> TTB) + "];\n";
                    else
                        o += "      const C " + nm[g][j] + " = LDS(s" + S(g) + " ^ " + S((grp_off(w, j) ^ hsw(grp_off(w, j))) << SH) + "u);\n";
                }
            }
            for (int r = 0; r < w.run; ++r) gen.gate(dg[w.begin + r], w.begin + r, nm);
            if (to_global && out_last) {  // register j of the store layout: amplitude j of the group
                for (int j = 0; j < 8; ++j) o += "      " + stv("base | dto | " + hex(hio[j]), nm[0][j]);
            } else if (to_global) {
                for (int g = 0; g < gen.G; ++g)
                    for (int j = 0; j < 8; ++j)
                        o += "      " + stv("base | dt | " + hex(hi_of((u32)(g * NT) + grp_off(w, j))), nm[g][j]);
            } else {
                for (int g = 0; g < gen.G; ++g)
                    for (int j = 0; j < 8; ++j) o += "      LDS(s" + S(g) + " ^ " + S((grp_off(w, j) ^ hsw(grp_off(w, j))) << SH) + "u) = " + nm[g][j] + ";\n";
            }
            // The next LDS phase: the next sweep, the stores from LDS in the
            // load/store layout, or the next tile's first write.
            const u32 h_after = si + 1 < sw.size() ? wave_pos(&sw[si + 1]) : to_global ? h_next_tile : h_io;
            sync("      ", wave_pos(&w), h_after);
            o += "    }\n";
            if (from_regs) issue_prefetch();
        }
        if (sw.empty()) {  // a pass without gates: copy the tile back
            for (int k = 0; k < PER; ++k) o += "    " + stv("base | dt | " + hex(hi[k]), "LDS(st ^ " + S(((u32)(k * NT) ^ hsw((u32)(k * NT))) << SH) + "u)");
            o += "    __syncthreads();\n";
        } else if (!last_regs) {
            for (int k = 0; k < PER; ++k) o += "    " + stv("base | dt | " + hex(hi[k]), "LDS(st ^ " + S(((u32)(k * NT) ^ hsw((u32)(k * NT))) << SH) + "u)");
            sync("    ", h_io, h_next_tile);
        }
        o.insert(body_at, "  for (; tile < ntiles; tile += gridDim.x) {\n");
        o += "  }\n}\n";
    }
    return o;
}

// Trajectory passes (one kernel per pass, qs_tpass0, ...): block = (trajectory,
// tile) as in k_traj_pass, with the same early exits (trajectories that share
// the noiseless state or whose first affected gate lies beyond the pass) and
// the same start from the noiseless run's state; gate values and C1Q control
// values come per trajectory from tables (tv: 8 values per plan gate, tcv: 1
// per plan gate) that the frames, noise matrices and folding fill beforehand.
// Tiles of 12 bits for both types.
std::string jit_traj_source(const std::vector<DPass> &passes, const std::vector<DGate> &dg, int dtype) {
    const int TB = 12, TS = 1 << TB, NT = kTileThreads, PER = TS / NT;
    static const int kPat128[12] = {1, 2, 4, 8, 15, 12, 9, 3, 6, 14, 6, 0};
    static const int kPat64[12] = {1, 2, 4, 8, 16, 31, 25, 21, 27, 25, 1, 30};
    const int SB = dtype == QS_C128 ? 4 : 5;
    const int *pat = dtype == QS_C128 ? kPat128 : kPat64;
    auto hsw = [&](u32 m) {
        u32 h = 0;
        for (int p = SB; p < TB; ++p)
            if ((m >> p) & 1) h ^= (u32)pat[p];
        return h;
    };
    Gen gen;
    gen.dtype = dtype;
    gen.G = 1;
    gen.traj = true;
    std::string &o = gen.o;
    o += dtype == QS_C128 ? "typedef double R;\n" : "typedef float R;\n";
    o += "typedef R C __attribute__((ext_vector_type(2)));\n"
         "__device__ __forceinline__ C row(R a, R b, R c, R d, C x, C y) {\n"
         "  C r; r.x = a * x.x - b * x.y + c * y.x - d * y.y; r.y = a * x.y + b * x.x + c * y.y + d * y.x; return r; }\n"
         "__device__ __forceinline__ C cm(C x, R a, R b) { C r; r.x = a * x.x - b * x.y; r.y = a * x.y + b * x.x; return r; }\n"
         "__device__ __forceinline__ unsigned ins(unsigned x, int b) { return ((x >> b) << (b + 1)) | (x & ((1u << b) - 1u)); }\n"
         "#define LDS(off) (*(C *)((char *)sh + (off)))\n";
    const int SH = dtype == QS_C128 ? 4 : 3;  // LDS slots as byte offsets (as in the block passes)
    o += "__device__ __forceinline__ unsigned hsw(unsigned m) {\n  unsigned h = 0u;\n";
    for (int p = SB; p < TB; ++p)
        if (pat[p]) o += "  h ^= ((m >> " + S(p) + ") & 1u) ? " + S(pat[p]) + "u : 0u;\n";
    o += "  return h;\n}\n";
    for (size_t pi = 0; pi < passes.size(); ++pi) {
        const DPass &P = passes[pi];
        if (P.tb != TB) return "";
        o += "extern \"C\" __global__ void __launch_bounds__(" + S(NT) + ") qs_tpass" + S((long long)pi) +
             "(C *__restrict__ states, unsigned long long N, const R *__restrict__ tv, const int *__restrict__ tc, unsigned ngates,"
             " int first_pass, unsigned long long basis, const int *__restrict__ nins, const int *__restrict__ first, int n_traj,"
             " const C *ideal_in, C *ideal_out) {\n";
        o += "  __shared__ C sh[" + S(TS) + "];\n";
        o += "  const unsigned tile = blockIdx.x & " + S((1u << P.nrest) - 1) + "u;\n";
        o += "  const unsigned t = blockIdx.x >> " + S(P.nrest) + ";\n";
        o += "  if (!(t == (unsigned)n_traj || nins[t] > 0)) return;\n";
        o += "  const bool ideal = t == (unsigned)n_traj;\n";
        o += "  const int g1 = ideal ? 0 : first[t];\n";
        o += "  if (!ideal && g1 >= " + S(P.gate_begin + P.gate_count) + ") return;\n";
        o += "  const bool from_ideal = ideal || g1 >= " + S(P.gate_begin) + ";\n";
        o += "  C *psi = ideal ? ideal_out : states + (unsigned long long)t * N;\n";
        o += "  const C *src = from_ideal ? ideal_in : psi;\n";
        o += "  const bool fill = from_ideal && first_pass != 0;\n";
        o += "  const R *__restrict__ vv = tv + (unsigned long long)t * ngates * 8u;\n";
        o += "  const int *__restrict__ tcv = tc + (unsigned long long)t * ngates;\n";
        o += "  const unsigned tl = threadIdx.x, st = (tl ^ hsw(tl)) << " + S(SH) + ";\n";
        o += "  const unsigned long long dt = " + deposit("(unsigned long long)tl", P.T, 9) + ";\n";
        o += "  const unsigned long long base = " + deposit("(unsigned long long)tile", P.rest, P.nrest) + ";\n";
        std::vector<u64> hi(PER);
        for (int k = 0; k < PER; ++k) {
            u64 off = 0;
            for (int b = 9; b < TB; ++b)
                if (((u64)k << 9 >> b) & 1) off |= 1ull << P.T[b];
            hi[k] = off;
        }
        struct Sw {
            int begin, run, g0, g1, g2;
        };
        std::vector<Sw> sw;
        for (int gi = P.gate_begin; gi < P.gate_begin + P.gate_count; gi += dg[gi].run)
            sw.push_back({gi, dg[gi].run, dg[gi].g[0], dg[gi].g[1], dg[gi].g[2]});
        auto on_top = [&](const Sw &w) { return w.g0 == TB - 3 && w.g1 == TB - 2 && w.g2 == TB - 1; };
        // Load and store layouts as in the block passes: the first / last
        // sweep's group bits serve as register bits when they lie above the
        // tile's contiguous row.
        const int row_bits = dtype == QS_C128 ? 3 : 4;
        auto own_layout = [&](const Sw &w) { return w.g0 >= row_bits && !on_top(w); };
        const bool in_first = !sw.empty() && own_layout(sw.front());
        const bool out_last = !sw.empty() && own_layout(sw.back());
        auto group_layout = [&](const Sw &f, const char *name, std::vector<u64> &h) {
            uint8_t q[16];
            int nq = 0;
            for (int p = 0; p < TB; ++p)
                if (p != f.g0 && p != f.g1 && p != f.g2) q[nq++] = P.T[p];
            o += "  const unsigned long long " + std::string(name) + " = " + deposit("(unsigned long long)tl", q, nq) + ";\n";
            h.assign(8, 0);
            for (int k = 0; k < 8; ++k)
                h[k] = ((k & 1) ? 1ull << P.T[f.g0] : 0) | ((k & 2) ? 1ull << P.T[f.g1] : 0) | ((k & 4) ? 1ull << P.T[f.g2] : 0);
        };
        std::vector<u64> hii = hi, hio;
        if (in_first) group_layout(sw.front(), "dti", hii);
        else o += "  const unsigned long long dti = dt;\n";
        if (out_last) group_layout(sw.back(), "dto", hio);
        o += "  C pre[" + S(PER) + "];\n";
        for (int k = 0; k < PER; ++k) {
            const std::string idx = "(base | dti | " + hex(hii[k]) + ")";
            o += "  if (fill) { pre[" + S(k) + "].x = " + idx + " == basis ? (R)1 : (R)0; pre[" + S(k) + "].y = (R)0; }\n";
            o += "  else pre[" + S(k) + "] = __builtin_nontemporal_load(src + " + idx + ");\n";
        }
        const bool first_regs = !sw.empty() && (on_top(sw.front()) || in_first);
        const bool last_regs = !sw.empty() && (on_top(sw.back()) || out_last);
        auto grp_off = [&](const Sw &w, int j) {
            return ((u32)(j & 1) << w.g0) | ((u32)((j >> 1) & 1) << w.g1) | ((u32)((j >> 2) & 1) << w.g2);
        };
        auto hi_of = [&](u32 mhigh) {
            u64 off = 0;
            for (int b = 9; b < TB; ++b)
                if ((mhigh >> b) & 1) off |= 1ull << P.T[b];
            return off;
        };
        // Workgroup barriers only where the wavefront-selecting tile positions
        // of consecutive LDS phases differ (as in the block passes).
        auto wave_pos = [&](const Sw *w) {
            u32 h = 0;
            for (int p = 0, rank = 0; p < TB; ++p) {
                if (w && (p == w->g0 || p == w->g1 || p == w->g2)) continue;
                if (rank >= 6 && rank < 9) h |= 1u << p;
                ++rank;
            }
            return h;
        };
        auto sync = [&](const char *ind, u32 from, u32 to) {
            if (from != to) o += std::string(ind) + "__syncthreads();\n";
            else
                o += std::string(ind) + "__builtin_amdgcn_fence(__ATOMIC_RELEASE, \"wavefront\"); __builtin_amdgcn_wave_barrier(); "
                                        "__builtin_amdgcn_fence(__ATOMIC_ACQUIRE, \"wavefront\");\n";
        };
        const u32 h_io = wave_pos(nullptr);
        if (!first_regs) {
            for (int k = 0; k < PER; ++k) o += "  LDS(st ^ " + S(((u32)(k * NT) ^ hsw((u32)(k * NT))) << SH) + "u) = pre[" + S(k) + "];\n";
            if (sw.empty()) o += "  __syncthreads();\n";
            else sync("  ", h_io, wave_pos(&sw.front()));
        }
        for (size_t si = 0; si < sw.size(); ++si) {
            const Sw &w = sw[si];
            const bool from_regs = si == 0 && first_regs, to_global = si + 1 == sw.size() && last_regs;
            o += "  {\n";
            std::vector<std::vector<std::string>> nm(1, std::vector<std::string>(8));
            o += "      const unsigned m0 = ins(ins(ins(tl, " + S(w.g0) + "), " + S(w.g1) + "), " + S(w.g2) + ");\n";
            if (!from_regs || !to_global) o += "      const unsigned s0 = (m0 ^ hsw(m0)) << " + S(SH) + ";\n";
            for (int j = 0; j < 8; ++j) {
                nm[0][j] = gen.fresh("x");
                if (from_regs)  // register k of the load layout holds amplitude k of the group
                    o += "      const C " + nm[0][j] + " = pre[" + S(in_first ? j : grp_off(w, j) >> 9) + "];\n";
                else
                    o += "      const C " + nm[0][j] + " = LDS(s0 ^ " + S((grp_off(w, j) ^ hsw(grp_off(w, j))) << SH) + "u);\n";
            }
            for (int r = 0; r < w.run; ++r) gen.gate(dg[w.begin + r], w.begin + r, nm);
            if (to_global) {
                for (int j = 0; j < 8; ++j)
                    o += "      __builtin_nontemporal_store(" + nm[0][j] + ", psi + (base | " +
                         (out_last ? "dto | " + hex(hio[j]) : "dt | " + hex(hi_of(grp_off(w, j)))) + "));\n";
            } else {
                for (int j = 0; j < 8; ++j) o += "      LDS(s0 ^ " + S((grp_off(w, j) ^ hsw(grp_off(w, j))) << SH) + "u) = " + nm[0][j] + ";\n";
                sync("      ", wave_pos(&w), si + 1 < sw.size() ? wave_pos(&sw[si + 1]) : h_io);
            }
            o += "  }\n";
        }
        if (sw.empty() || !last_regs)
            for (int k = 0; k < PER; ++k)
                o += "  __builtin_nontemporal_store(LDS(st ^ " + S(((u32)(k * NT) ^ hsw((u32)(k * NT))) << SH) + "u), psi + (base | dt | " + hex(hi[k]) + "));\n";
        o += "}\n";
    }
    return o;
}

// ------------------------------------------------------------------ compile and load

namespace {

// Compiled plan sources (code objects, host memory), kept for reuse: a new
// state or a released plan with the same structure loads the code again
// without compiling.  Beyond kMaxJitSources the least recently used source is
// dropped.  Device residency belongs to the plans: each plan loads its own
// module and unloads it when it is released.
struct JitCode {
    std::vector<char> code;
    uint64_t last_use = 0;
};
constexpr size_t kMaxJitSources = 64;
std::mutex g_jit_mu;
uint64_t g_jit_clock = 0;
std::unordered_map<std::string, JitCode> g_jit;

int compile(const std::string &src, std::vector<char> &code) {
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, src.c_str(), "qsim_block.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS)
        return fail(QS_ERR_UNSUPPORTED, "hiprtcCreateProgram failed");
    const char *opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
    const hiprtcResult r = hiprtcCompileProgram(prog, (int)(sizeof opts / sizeof opts[0]), opts);
    if (r != HIPRTC_SUCCESS) {
        size_t n = 0;
        hiprtcGetProgramLogSize(prog, &n);
        std::string log(n, '\0');
        if (n) hiprtcGetProgramLog(prog, &log[0]);
        hiprtcDestroyProgram(&prog);
        return fail(QS_ERR_UNSUPPORTED, "hiprtc compile of a block plan failed: " + log.substr(0, 2000));
    }
    size_t n = 0;
    hiprtcGetCodeSize(prog, &n);
    code.resize(n);
    hiprtcGetCode(prog, code.data());
    hiprtcDestroyProgram(&prog);
    return QS_OK;
}

}  // namespace

int jit_block_functions(const std::string &src, int npass, int device, JitFns &out, const char *prefix,
                        const std::vector<unsigned> &threads) {
    std::vector<char> code;
    {
        std::lock_guard<std::mutex> lk(g_jit_mu);
        auto it = g_jit.find(src);
        if (it == g_jit.end()) {
            JitCode c;
            if (int rc = compile(src, c.code)) return rc;
            if (g_jit.size() >= kMaxJitSources) {
                auto lru = g_jit.begin();
                for (auto j = g_jit.begin(); j != g_jit.end(); ++j)
                    if (j->second.last_use < lru->second.last_use) lru = j;
                g_jit.erase(lru);
            }
            it = g_jit.emplace(src, std::move(c)).first;
        }
        it->second.last_use = ++g_jit_clock;
        code = it->second.code;
    }
    JitFns f;
    QS_HIP(hipModuleLoadData(&f.mod, code.data()));
    f.fn.resize(npass);
    f.max_blocks.resize(npass);
    f.threads.assign(npass, (unsigned)kTileThreads);
    for (int p = 0; p < npass && p < (int)threads.size(); ++p) f.threads[p] = threads[p];
    int cus = 0;
    hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    for (int p = 0; p < npass && e == hipSuccess; ++p) {
        const std::string name = prefix + S(p);
        e = hipModuleGetFunction(&f.fn[p], f.mod, name.c_str());
        int nb = 0;
        if (e == hipSuccess) e = hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f.fn[p], (int)f.threads[p], 0);
        f.max_blocks[p] = (unsigned)std::max(1, nb) * (unsigned)std::max(1, cus);
    }
    if (e != hipSuccess) {
        (void)hipModuleUnload(f.mod);
        return hip_fail(e, "loading a compiled block plan");
    }
    out = std::move(f);
    return QS_OK;
}

}  // namespace qs
