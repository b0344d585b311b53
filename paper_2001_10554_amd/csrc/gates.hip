// Streaming kernels: state initialisation and single gates applied as one
// read+write pass over the amplitudes that the gate touches.
//
// A one-qubit gate (eq. 3) couples amplitude i (bit q clear) with i + 2^q and
// nothing else, so every pair is independent.  Pair k of the 2^{n-1} pairs is
// i0 = k with a zero inserted at bit q; consecutive lanes take consecutive k,
// so for q >= 6 a wavefront touches two contiguous 1 KiB runs (c128) and for
// q < 6 the two partners of a lane sit in the same 128-byte line.  Each thread
// keeps PPT pairs in flight to cover HBM latency.
#include "launch.h"
#include "vec.h"

namespace qs {

// ------------------------------------------------------------------ initialisation
//
// One amplitude per thread up to 2^31 amplitudes: every wavefront writes one
// contiguous 1 KiB run (c128) and retires.  For these write-only streams that
// form measured 6.9 TB/s against 5.2 TB/s for a 65536-block grid-stride loop
// and 6.0 TB/s for four amplitudes per thread.  A launch holds fewer than 2^32
// work-items, so larger registers loop over 2^31-amplitude strides.

template <typename R> __global__ __launch_bounds__(kBlock) void k_fill_basis(cx<R> *psi, u64 N, u64 index) {
    for (u64 i = (u64)blockIdx.x * kBlock + threadIdx.x; i < N; i += (u64)gridDim.x * kBlock) {
        cx<R> v;
        v.x = (i == index) ? (R)1 : (R)0;
        v.y = (R)0;
        psi[i] = v;
    }
}

template <typename R> __global__ __launch_bounds__(kBlock) void k_fill_uniform(cx<R> *psi, u64 N, double amp) {
    cx<R> v;
    v.x = (R)amp;
    v.y = (R)0;
    for (u64 i = (u64)blockIdx.x * kBlock + threadIdx.x; i < N; i += (u64)gridDim.x * kBlock) psi[i] = v;
}

// Unnormalised draw: (2u - 1) + i (2v - 1), u, v from Philox(seed; i_lo, i_hi, tag, 0).
template <typename R> __global__ __launch_bounds__(kBlock) void k_fill_random(cx<R> *psi, u64 N, u32 k0, u32 k1) {
    for (u64 i = (u64)blockIdx.x * kBlock + threadIdx.x; i < N; i += (u64)gridDim.x * kBlock) {
        const Philox4 x = philox4x32_10((u32)i, (u32)(i >> 32), kTagInitRandom, 0u, k0, k1);
        cx<R> v;
        v.x = (R)(2.0 * u53(x.v[0], x.v[1]) - 1.0);
        v.y = (R)(2.0 * u53(x.v[2], x.v[3]) - 1.0);
        psi[i] = v;
    }
}

// psi *= 1 / sqrt(*norm_dev), factor read on the device (stream-ordered).
template <typename R> __global__ __launch_bounds__(kBlock) void k_scale_inv_sqrt(cx<R> *psi, u64 N, const double *norm_dev) {
    const double f = 1.0 / sqrt(*norm_dev);
    for (u64 i = (u64)blockIdx.x * kBlock + threadIdx.x; i < N; i += (u64)gridDim.x * kBlock) {
        cx<R> v = psi[i];
        v.x = (R)((double)v.x * f);
        v.y = (R)((double)v.y * f);
        psi[i] = v;
    }
}

static unsigned stream_grid(u64 N) {
    const u64 g = (N + kBlock - 1) / kBlock, cap = 1ull << 23;  // 2^23 * 256 = 2^31 work-items
    return (unsigned)(g < cap ? g : cap);
}

int launch_init_basis(qs_state *s, u64 index) {
    const u64 N = 1ull << s->n;
    if (s->dtype == QS_C128)
        hipLaunchKernelGGL(k_fill_basis<double>, dim3(stream_grid(N)), dim3(kBlock), 0, s->stream, (cx<double> *)s->buf, N, index);
    else
        hipLaunchKernelGGL(k_fill_basis<float>, dim3(stream_grid(N)), dim3(kBlock), 0, s->stream, (cx<float> *)s->buf, N, index);
    QS_LAUNCH_CHECK("init_basis");
    return QS_OK;
}

int launch_init_uniform(qs_state *s) {
    const u64 N = 1ull << s->n;
    const double amp = 1.0 / sqrt((double)N);
    if (s->dtype == QS_C128)
        hipLaunchKernelGGL(k_fill_uniform<double>, dim3(stream_grid(N)), dim3(kBlock), 0, s->stream, (cx<double> *)s->buf, N, amp);
    else
        hipLaunchKernelGGL(k_fill_uniform<float>, dim3(stream_grid(N)), dim3(kBlock), 0, s->stream, (cx<float> *)s->buf, N, amp);
    QS_LAUNCH_CHECK("init_uniform");
    return QS_OK;
}

int launch_init_random(qs_state *s, u64 seed) {
    const u64 N = 1ull << s->n;
    const u32 k0 = (u32)seed, k1 = (u32)(seed >> 32);
    if (s->dtype == QS_C128)
        hipLaunchKernelGGL(k_fill_random<double>, dim3(stream_grid(N)), dim3(kBlock), 0, s->stream, (cx<double> *)s->buf, N, k0, k1);
    else
        hipLaunchKernelGGL(k_fill_random<float>, dim3(stream_grid(N)), dim3(kBlock), 0, s->stream, (cx<float> *)s->buf, N, k0, k1);
    QS_LAUNCH_CHECK("init_random");
    // Normalise: FP64 norm into the handle's result slot, then scale on device.
    double *norm = s->scratch + kScratchDoubles - 8;
    int rc = launch_marginals(s, kMargNorm, 0, norm);
    if (rc != QS_OK) return rc;
    return launch_scale(s, norm);
}

int launch_scale(qs_state *s, const double *norm_dev) {
    const u64 N = 1ull << s->n;
    if (s->dtype == QS_C128)
        hipLaunchKernelGGL(k_scale_inv_sqrt<double>, dim3(stream_grid(N)), dim3(kBlock), 0, s->stream, (cx<double> *)s->buf, N, norm_dev);
    else
        hipLaunchKernelGGL(k_scale_inv_sqrt<float>, dim3(stream_grid(N)), dim3(kBlock), 0, s->stream, (cx<float> *)s->buf, N, norm_dev);
    QS_LAUNCH_CHECK("scale");
    return QS_OK;
}

// ------------------------------------------------------------------ one-qubit gate (eq. 3)

// Block-index remap.  The hardware hands consecutive workgroups to the 8 XCDs
// in turn, so by default all XCDs stream through one common window of the
// state.  With chunk = C > 0, XCD x instead takes runs of C consecutive
// logical blocks (groups of 8C blocks, XCD x owning the x-th run of each
// group); chunk = ~0 gives each XCD one contiguous eighth of the grid.
// blk0: the launch piece's first workgroup (the remap acts within a piece).
__device__ __forceinline__ u64 logical_block(u32 chunk, u64 blk0) {
    const u64 b = blockIdx.x, nb = gridDim.x;
    if (chunk == 0 || (nb & 7)) return blk0 + b;
    if (chunk == ~0u) return blk0 + (b & 7) * (nb >> 3) + (b >> 3);
    const u64 C = chunk;
    if (nb % (8 * C)) return blk0 + b;
    const u64 r = b >> 3;
    return blk0 + (r / C) * (8 * C) + (b & 7) * C + (r % C);
}

// CTRL: a controlled gate whose control qubit c lies inside every 128-byte
// line (c < 3 for c128, c < 4 for c64).  Such a gate touches half of every
// line, so the whole line is moved anyway; these kernels then stream all
// pairs and leave the control-0 ones unchanged, keeping loads and stores
// full-line.
// dlog: the thread's PPT pairs are 2^dlog pairs apart (8: consecutive
// 256-pair slices of one block); a block then covers 256 pairs in each of PPT
// slices of a region of PPT * 2^dlog pairs.  The host uses dlog > 8 only when
// npairs is a multiple of that region.
template <typename R, int PPT, bool NT, bool CTRL = false>
__global__ __launch_bounds__(kBlock) void k_apply_1q(cx<R> *__restrict__ psi, u64 npairs, int q, Mat2<R> u, u32 chunk, int c, int dlog,
                                                     u64 blk0) {
    const u64 s = 1ull << q;
    const u64 lb = logical_block(chunk, blk0);
    const int rlog = dlog - 8;  // blocks per region, log2
    const u64 first = ((lb >> rlog) * PPT << dlog) + ((lb & ((1ull << rlog) - 1)) << 8) + threadIdx.x;
    cx<R> a[PPT], b[PPT];
    u64 i0[PPT];
    if ((lb + 1) * (kBlock * PPT) <= npairs) {
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            i0[j] = insert0(first + ((u64)j << dlog), q);
            a[j] = ld<NT>(psi + i0[j]);
            b[j] = ld<NT>(psi + i0[j] + s);
        }
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            if (!CTRL || ((i0[j] >> c) & 1)) apply2<R>(u, a[j], b[j]);
            st<NT>(psi + i0[j], a[j]);
            st<NT>(psi + i0[j] + s, b[j]);
        }
    } else {
        for (int j = 0; j < PPT; ++j) {
            const u64 k = first + (u64)j * kBlock;
            if (k >= npairs) break;
            const u64 i = insert0(k, q);
            if (CTRL && !((i >> c) & 1)) continue;
            cx<R> x = psi[i], y = psi[i + s];
            apply2<R>(u, x, y);
            psi[i] = x;
            psi[i + s] = y;
        }
    }
}

// Low targets (q < 6): the partner of amplitude i sits in the same wavefront
// when lanes hold consecutive amplitudes, so every load and store instruction
// covers one contiguous 1 KiB (c128) run and the partner arrives by a lane
// shuffle (lane xor 2^q).  Lane with bit q clear computes U00 a + U01 b, the
// other U10 a + U11 b.  Requires 2^n to be a multiple of 256 * APT.
// dlog / chunk: as for the pair kernel (the thread's APT amplitudes are
// 2^dlog apart; chunk remaps blocks to XCD runs).
template <typename R, int APT, bool NT, bool CTRL = false>
__global__ __launch_bounds__(kBlock) void k_apply_1q_lane(cx<R> *__restrict__ psi, int q, Mat2<R> u, int c, int dlog, u32 chunk,
                                                          u64 blk0) {
    const u64 lb = logical_block(chunk, blk0);
    const int rlog = dlog - 8;
    const u64 first = ((lb >> rlog) * APT << dlog) + ((lb & ((1ull << rlog) - 1)) << 8) + threadIdx.x;
    const int lane = threadIdx.x & 63, mask = 1 << q;
    const bool upper = lane & mask;
    // own coefficient (diagonal) and partner coefficient (off-diagonal) of this lane's row
    const R own_re = upper ? u.m[6] : u.m[0], own_im = upper ? u.m[7] : u.m[1];
    const R oth_re = upper ? u.m[4] : u.m[2], oth_im = upper ? u.m[5] : u.m[3];
    cx<R> a[APT];
#pragma unroll
    for (int j = 0; j < APT; ++j) a[j] = ld<NT>(psi + first + ((u64)j << dlog));
#pragma unroll
    for (int j = 0; j < APT; ++j) {
        cx<R> b;
        b.x = __shfl_xor(a[j].x, mask, 64);
        b.y = __shfl_xor(a[j].y, mask, 64);
        cx<R> r;
        r.x = own_re * a[j].x - own_im * a[j].y + oth_re * b.x - oth_im * b.y;
        r.y = own_re * a[j].y + own_im * a[j].x + oth_re * b.y + oth_im * b.x;
        if (CTRL && !(((first + ((u64)j << dlog)) >> c) & 1)) r = a[j];
        st<NT>(psi + first + ((u64)j << dlog), r);
    }
}

// Launch shape of the one-qubit gate.  Defaults come from timing every target
// of a 32-qubit complex128 sweep; environment variables override them for
// tuning runs: QSIM_1Q_PPT pairs per thread 1/2/4; QSIM_1Q_NT non-temporal
// hints 0/1; QSIM_1Q_CHUNK block remap (0 = hardware order, -1 = XCD eighths,
// C = runs of C blocks); QSIM_1Q_LANE lane-shuffle kernel for q < 6, 0/1;
// QSIM_1Q_SPREAD / QSIM_1Q_LSPREAD log2 of the distance between a thread's
// pairs / amplitudes (pair / lane kernel); QSIM_1Q_LCHUNK the lane kernel's
// block remap; QSIM_C1Q_SPREAD the controlled kernel's spread.
struct Shape1q {
    int ppt, nt, lane, dlog, ldlog, cdlog, cppt, qdlog, sdlog;
    u32 chunk, lchunk, cchunk, dchunk;
};

static Shape1q shape_1q() {
    static Shape1q sh = [] {
        auto env = [](const char *k, long dflt) {
            const char *e = getenv(k);
            return e ? atol(e) : dflt;
        };
        Shape1q v;
        v.ppt = (int)env("QSIM_1Q_PPT", 2);
        v.nt = (int)env("QSIM_1Q_NT", 1);
        v.lane = (int)env("QSIM_1Q_LANE", 1);
        v.chunk = (u32)env("QSIM_1Q_CHUNK", 0x7fffffff);  // 0x7fffffff: per-target schedule below
        v.dlog = (int)env("QSIM_1Q_SPREAD", 11);
        v.ldlog = (int)env("QSIM_1Q_LSPREAD", 11);
        // Controlled gates: a thread's quads 2^cdlog apart, per control by
        // default (spread_for_c1q); QSIM_C1Q_SPREAD forces one value.
        v.cdlog = (int)env("QSIM_C1Q_SPREAD", 0);
        // Lane kernel (q < 6): runs of 64 blocks per XCD.  Measured on a
        // 32-qubit complex128 register, two runs: 6.54-6.63 TB/s in hardware
        // order, 6.68-6.70 with runs of 64, 6.66-6.68 with 256, 6.57-6.59
        // with contiguous eighths.
        v.lchunk = (u32)env("QSIM_1Q_LCHUNK", 64);
        v.cppt = (int)env("QSIM_C1Q_PPT", 2);
        v.cchunk = (u32)env("QSIM_C1Q_CHUNK", 0x7fffffff);  // 0x7fffffff: per-control schedule
        v.dchunk = (u32)env("QSIM_QUAD_CHUNK", 0x7fffffff);  // diagonal / SWAP block remap
        v.qdlog = (int)env("QSIM_DIAG_SPREAD", 8);          // two-qubit diagonal spread
        v.sdlog = (int)env("QSIM_SWAP_SPREAD", 11);         // SWAP spread
        return v;
    }();
    return sh;
}

// Per-XCD run length (in blocks of 512 pairs) for target q.  Measured on a
// 32-qubit complex128 sweep (three alternating runs on one box, pairs spread
// 2^11 apart): runs of 64 blocks for q = 6..15 (+30..140 GB/s over 128-256),
// 128 for q = 16 and 256 for q = 17; above, the best length follows q mod 4
// (the address bits in which the two partner streams differ): 64 for q = 2, 3
// mod 4, 32 for q = 1 mod 4, and for q = 0 mod 4 16 at q = 20 but 64 at
// q = 24, 28.
static u32 chunk_for_target(int q) {
    if (q <= 15) return 64;
    if (q == 16) return 128;
    if (q == 17) return 256;
    switch ((q - 20) & 3) {
    case 0: return q == 20 ? 16 : 64;
    case 1: return 32;
    default: return 64;
    }
}

// Spread of the two quads of a diagonal / SWAP thread (2^dlog apart; 8 =
// consecutive 256-quad slices), used when the quad count is a multiple of
// the region it implies.  Measured on a 30-qubit complex128 register: SWAP
// gains 1-4% from 2^11 (SWAP(5,25): 5.39 -> 5.62 TB/s of the touched
// quarters), the diagonal loses 1-2%, so it keeps consecutive slices.
static int quad_spread(int want, u64 nquads) {
    const int dlog = want >= 8 && want < 40 ? want : 8;
    return nquads % (2ull << dlog) ? 8 : dlog;
}

// Controlled gates with the control outside the 128-byte line, diagonal and
// SWAP gates (quads of two qubits): each XCD takes one contiguous eighth of
// the grid.  Measured on a 32-qubit complex128 register against per-target
// XCD runs of 16..256 blocks and hardware order: 6.3-6.6 TB/s for CNOT(c, c+1)
// at every c >= 3 (runs: 5.1-6.2), CZ 6.5 (6.0), SWAP 6.4 (5.6).
static u32 chunk_for_control(int, int) { return ~0u; }

// Per-XCD run length of the controlled gate (with the spreads of
// spread_for_c1q below) for CNOT(c, c+1), c = 3..30; 0 stands for contiguous
// eighths (chunk_for_control).  Measured on a 32-qubit complex128 register,
// two runs of every control with runs of 64, 256, 1024 blocks and eighths;
// the entries follow the DRAM address interleaving and were picked where
// both runs agreed (weakest control 5.67 -> 5.73 TB/s of the touched half;
// c = 25..28: +85..170 GB/s with runs of 64).
static u32 chunk_for_c1q(int c, int t) {
    static const u32 kRun[31] = {0,   0,   0,    64,   256,  1024, 0,  0,  64,  256, 0,  0,   256,  64,  256, 1024,
                                 0,   0,   0,    1024, 1024, 1024, 0,  256, 256, 64, 64, 64,  64,   1024, 1024};
    if (t == c + 1 && c >= 3 && c <= 30 && kRun[c]) return kRun[c];
    return chunk_for_control(c, t);
}

// Spread of the controlled gate's quads (log2 of their distance).  Measured
// per control on a 32-qubit complex128 CNOT(c, c+1) sweep with spreads 2^9..
// 2^13 against consecutive slices: 2^9..2^13 all lift the weakest low control
// (c = 7: 5.46 TB/s consecutive) and 2^11 suits c < 15 best; above, 2^10 is
// best or within noise for most controls (c = 28: 5.66 -> 5.85 TB/s, c = 20,
// 24: +0.08) and 2^13 for c = 3 mod 8 (c = 19: 5.62 -> 5.72, c = 27: 5.59 ->
// 5.67), in step with the DRAM address interleaving.
static int spread_for_c1q(int c, int t) {
    if (t != c + 1 || c < 15) return 11;
    return (c & 7) == 3 ? 13 : 10;
}

template <typename R> static int launch_1q_t(qs_state *s, int q, const double *u) {
    const u64 N = 1ull << s->n, npairs = N >> 1;
    const Mat2<R> m = to_mat<R>(u);
    cx<R> *psi = (cx<R> *)s->buf;
    const Shape1q v = shape_1q();
    const u32 chunk = v.chunk == 0x7fffffffu ? chunk_for_target(q) : v.chunk;
    hipStream_t st = s->stream;
    int dlog = v.dlog >= 8 && v.dlog < 40 ? v.dlog : 8;
    if (npairs % ((u64)v.ppt << dlog)) dlog = 8;
#define PAIR(PPT, NT)                                                                                                                 \
    for_pieces(grid_for(npairs, kBlock * PPT), [&](unsigned g, u64 b0) {                                                                \
        hipLaunchKernelGGL((k_apply_1q<R, PPT, NT>), dim3(g), dim3(kBlock), 0, st, psi, npairs, q, m, chunk, 0, dlog, b0);               \
    })
    if (v.lane && q < 6 && N >= (u64)kBlock * 2) {
        int ldlog = v.ldlog >= 8 && v.ldlog < 40 ? v.ldlog : 8;
        if (N % (2ull << ldlog)) ldlog = 8;
        for_pieces(N / (kBlock * 2), [&](unsigned g, u64 b0) {
            if (v.nt)
                hipLaunchKernelGGL((k_apply_1q_lane<R, 2, true>), dim3(g), dim3(kBlock), 0, st, psi, q, m, 0, ldlog, v.lchunk, b0);
            else
                hipLaunchKernelGGL((k_apply_1q_lane<R, 2, false>), dim3(g), dim3(kBlock), 0, st, psi, q, m, 0, ldlog, v.lchunk, b0);
        });
    } else if (v.nt) {
        if (v.ppt == 1) PAIR(1, true);
        else if (v.ppt == 4) PAIR(4, true);
        else PAIR(2, true);
    } else {
        if (v.ppt == 1) PAIR(1, false);
        else if (v.ppt == 4) PAIR(4, false);
        else PAIR(2, false);
    }
#undef PAIR
    QS_LAUNCH_CHECK("apply_1q");
    return QS_OK;
}

int launch_apply_1q(qs_state *s, int q, const double *u) {
    return s->dtype == QS_C128 ? launch_1q_t<double>(s, q, u) : launch_1q_t<float>(s, q, u);
}

// ------------------------------------------------------------------ controlled one-qubit gate
// Only the 2^{n-2} pairs whose control bit is 1 are read and written.

template <typename R, int PPT>
__global__ __launch_bounds__(kBlock) void k_apply_c1q(cx<R> *__restrict__ psi, u64 nquads, int c, int t, Mat2<R> u, u32 chunk, int dlog,
                                                      u64 blk0) {
    const int lo = c < t ? c : t, hi = c < t ? t : c;
    const u64 sc = 1ull << c, st_ = 1ull << t;
    const u64 lb = logical_block(chunk, blk0);
    const int rlog = dlog - 8;  // the thread's quads are 2^dlog apart (see k_apply_1q)
    const u64 first = ((lb >> rlog) * PPT << dlog) + ((lb & ((1ull << rlog) - 1)) << 8) + threadIdx.x;
    cx<R> a[PPT], b[PPT];
    u64 i0[PPT];
    bool ok[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const u64 k = first + ((u64)j << dlog);
        ok[j] = k < nquads;
        i0[j] = insert0(insert0(k, lo), hi) | sc;
        if (ok[j]) {
            a[j] = ld<true>(psi + i0[j]);
            b[j] = ld<true>(psi + (i0[j] | st_));
        }
    }
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        if (ok[j]) {
            apply2<R>(u, a[j], b[j]);
            st<true>(psi + i0[j], a[j]);
            st<true>(psi + (i0[j] | st_), b[j]);
        }
    }
}

template <typename R> static int launch_c1q_t(qs_state *s, int c, int t, const double *u) {
    const u64 N = 1ull << s->n, nquads = N >> 2;
    const Mat2<R> m = to_mat<R>(u);
    cx<R> *psi = (cx<R> *)s->buf;
    hipStream_t st = s->stream;
    const int line_bits = sizeof(R) == 8 ? 3 : 4;  // amplitudes per 128-byte line
    if (c < line_bits) {
        // Control inside the line: stream every pair of target t with full-line
        // accesses and leave the control-0 pairs unchanged.
        if (t < 6 && N >= (u64)kBlock * 2)
            for_pieces(N / (kBlock * 2), [&](unsigned g, u64 b0) {
                hipLaunchKernelGGL((k_apply_1q_lane<R, 2, true, true>), dim3(g), dim3(kBlock), 0, st, psi, t, m, c, 8, 0u, b0);
            });
        else
            for_pieces(grid_for(N >> 1, kBlock * 2), [&](unsigned g, u64 b0) {
                hipLaunchKernelGGL((k_apply_1q<R, 2, true, true>), dim3(g), dim3(kBlock), 0, st, psi, N >> 1, t, m, chunk_for_target(t), c, 8, b0);
            });
    } else {
        const Shape1q v = shape_1q();
        int dlog = v.cdlog >= 8 && v.cdlog < 40 ? v.cdlog : v.cdlog == 0 ? spread_for_c1q(c, t) : 8;
        const int ppt = v.cppt == 4 ? 4 : 2;
        if (nquads % ((u64)ppt << dlog)) dlog = 8;
        const u32 chunk = v.cchunk == 0x7fffffffu ? chunk_for_c1q(c, t) : v.cchunk;
        for_pieces(grid_for(nquads, kBlock * ppt), [&](unsigned g, u64 b0) {
            if (ppt == 4)
                hipLaunchKernelGGL((k_apply_c1q<R, 4>), dim3(g), dim3(kBlock), 0, st, psi, nquads, c, t, m, chunk, dlog, b0);
            else
                hipLaunchKernelGGL((k_apply_c1q<R, 2>), dim3(g), dim3(kBlock), 0, st, psi, nquads, c, t, m, chunk, dlog, b0);
        });
    }
    QS_LAUNCH_CHECK("apply_c1q");
    return QS_OK;
}

int launch_apply_c1q(qs_state *s, int c, int t, const double *u) {
    return s->dtype == QS_C128 ? launch_c1q_t<double>(s, c, t, u) : launch_c1q_t<float>(s, c, t, u);
}

// ------------------------------------------------------------------ two-qubit diagonal and SWAP
// Both enumerate the 2^{n-2} quads (bits q0, q1 cleared).  A diagonal entry
// equal to exactly 1 is skipped (touch mask), so CZ and controlled phases read
// and write only the |11> quarter of the state.

template <typename R> struct Diag4 {
    R d[8];
};

// Two quads per thread, loads before stores; blocks remapped to XCD runs as
// for the controlled gate.
// dlog: the thread's quads are 2^dlog apart (as for the controlled gate).
template <typename R, int PPT>
__global__ __launch_bounds__(kBlock) void k_apply_diag2(cx<R> *__restrict__ psi, u64 nquads, int q0, int q1, Diag4<R> d, int touch, u32 chunk,
                                                        int dlog, u64 blk0) {
    const int lo = q0 < q1 ? q0 : q1, hi = q0 < q1 ? q1 : q0;
    const u64 lb = logical_block(chunk, blk0);
    const int rlog = dlog - 8;
    const u64 first = ((lb >> rlog) * PPT << dlog) + ((lb & ((1ull << rlog) - 1)) << 8) + threadIdx.x;
    cx<R> v[PPT][4];
    u64 base[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const u64 k = first + ((u64)j << dlog);
        base[j] = insert0(insert0(k, lo), hi);
        if (k < nquads) {
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if ((touch >> e) & 1) v[j][e] = ld<true>(psi + (base[j] | ((u64)(e & 1) << q0) | ((u64)(e >> 1) << q1)));
        }
    }
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        if (first + ((u64)j << dlog) >= nquads) continue;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            if (!((touch >> e) & 1)) continue;
            cx<R> f;
            f.x = d.d[2 * e];
            f.y = d.d[2 * e + 1];
            st<true>(psi + (base[j] | ((u64)(e & 1) << q0) | ((u64)(e >> 1) << q1)), cmul<R>(v[j][e], f));
        }
    }
}

template <typename R, int PPT>
__global__ __launch_bounds__(kBlock) void k_apply_swap(cx<R> *__restrict__ psi, u64 nquads, int a, int b, u32 chunk, int dlog, u64 blk0) {
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    const u64 lb = logical_block(chunk, blk0);
    const int rlog = dlog - 8;
    const u64 first = ((lb >> rlog) * PPT << dlog) + ((lb & ((1ull << rlog) - 1)) << 8) + threadIdx.x;
    cx<R> x[PPT], y[PPT];
    u64 i[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const u64 k = first + ((u64)j << dlog);
        i[j] = insert0(insert0(k, lo), hi);
        if (k < nquads) {
            x[j] = ld<true>(psi + (i[j] | (1ull << a)));
            y[j] = ld<true>(psi + (i[j] | (1ull << b)));
        }
    }
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        if (first + ((u64)j << dlog) >= nquads) continue;
        st<true>(psi + (i[j] | (1ull << a)), y[j]);
        st<true>(psi + (i[j] | (1ull << b)), x[j]);
    }
}

template <typename R> static int launch_diag2_t(qs_state *s, int q0, int q1, const double *d) {
    const u64 nquads = 1ull << (s->n - 2);
    Diag4<R> dd;
    int touch = 0;
    for (int e = 0; e < 4; ++e) {
        dd.d[2 * e] = (R)d[2 * e];
        dd.d[2 * e + 1] = (R)d[2 * e + 1];
        if (!(d[2 * e] == 1.0 && d[2 * e + 1] == 0.0)) touch |= 1 << e;
    }
    if (!touch) return QS_OK;
    const Shape1q v = shape_1q();
    const u32 chunk = v.dchunk == 0x7fffffffu ? chunk_for_control(q0, q1) : v.dchunk;
    const int dlog = quad_spread(v.qdlog, nquads);
    for_pieces(grid_for(nquads, kBlock * 2), [&](unsigned g, u64 b0) {
        hipLaunchKernelGGL((k_apply_diag2<R, 2>), dim3(g), dim3(kBlock), 0, s->stream, (cx<R> *)s->buf, nquads, q0, q1, dd, touch, chunk, dlog,
                           b0);
    });
    QS_LAUNCH_CHECK("apply_diag2");
    return QS_OK;
}

int launch_apply_diag2(qs_state *s, int q0, int q1, const double *d) {
    return s->dtype == QS_C128 ? launch_diag2_t<double>(s, q0, q1, d) : launch_diag2_t<float>(s, q0, q1, d);
}

int launch_apply_swap(qs_state *s, int a, int b) {
    const u64 nquads = 1ull << (s->n - 2);
    const Shape1q v = shape_1q();
    const u32 chunk = v.dchunk == 0x7fffffffu ? chunk_for_control(a, b) : v.dchunk;
    const int dlog = quad_spread(v.sdlog, nquads);
    if (s->dtype == QS_C128)
        for_pieces(grid_for(nquads, kBlock * 2), [&](unsigned g, u64 b0) {
            hipLaunchKernelGGL((k_apply_swap<double, 2>), dim3(g), dim3(kBlock), 0, s->stream, (cx<double> *)s->buf, nquads, a, b, chunk, dlog, b0);
        });
    else
        for_pieces(grid_for(nquads, kBlock * 2), [&](unsigned g, u64 b0) {
            hipLaunchKernelGGL((k_apply_swap<float, 2>), dim3(g), dim3(kBlock), 0, s->stream, (cx<float> *)s->buf, nquads, a, b, chunk, dlog, b0);
        });
    QS_LAUNCH_CHECK("apply_swap");
    return QS_OK;
}

// ------------------------------------------------------------------ QAOA cost layer exp(-i gamma C)
// Unit weights: C(k) is an integer in [0, E]; each block builds the table
// exp(-i gamma c) for c = 0..E in LDS and then streams its amplitudes.
// Weighted edges: the phase is evaluated per amplitude.

template <typename R>
__global__ __launch_bounds__(kBlock) void k_cut_phase(cx<R> *__restrict__ psi, u64 N, Graph g, double gamma) {
    __shared__ double2 tab[kMaxEdges + 1];
    for (int c = threadIdx.x; c <= g.ne; c += kBlock) {
        double sn, cs;
        sincos(gamma * (double)c, &sn, &cs);
        tab[c] = make_double2(cs, -sn);
    }
    __syncthreads();
    for (u64 i = (u64)blockIdx.x * kBlock + threadIdx.x; i < N; i += (u64)gridDim.x * kBlock) {
        const double2 f = tab[cut_count(i, g)];
        cx<R> a = psi[i];
        cx<R> r;
        r.x = (R)(a.x * f.x - a.y * f.y);
        r.y = (R)(a.x * f.y + a.y * f.x);
        psi[i] = r;
    }
}

// Unit weights, chunks of 2^c amplitudes per block: integer cut values from
// cut_split and the phase table e^{-i gamma c}, c = 0..|E|.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_cut_phase_chunk(cx<R> *__restrict__ psi, int c, Graph g, double gamma) {
    __shared__ double2 ph[kMaxEdges + 1];
    __shared__ int tab[1 << kCutLoopBits];
    for (int k = threadIdx.x; k <= g.ne; k += kBlock) {
        double sn, cs;
        sincos(gamma * (double)k, &sn, &cs);
        ph[k] = make_double2(cs, -sn);
    }
    const u64 base = (u64)blockIdx.x << c;
    const u32 t = threadIdx.x;
    int ct, coef[kCutLoopBits];
    cut_split<int, false>(g, nullptr, t, base, c, ct, coef, tab, kBlock);
    __syncthreads();
    // Four loop steps per iteration (c >= 12: at least 16 steps), loads first.
    for (u32 j = 0; j < (1u << (c - 8)); j += 4) {
        cx<R> a[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) a[u] = psi[base + ((u64)(j + u) << 8) + t];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const double2 f = ph[cut_at<int>(ct, coef, tab, j + u)];
            cx<R> r;
            r.x = (R)(a[u].x * f.x - a[u].y * f.y);
            r.y = (R)(a[u].x * f.y + a[u].y * f.x);
            psi[base + ((u64)(j + u) << 8) + t] = r;
        }
    }
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_cut_phase_w(cx<R> *__restrict__ psi, u64 N, Graph g, Weights w, double gamma) {
    for (u64 i = (u64)blockIdx.x * kBlock + threadIdx.x; i < N; i += (u64)gridDim.x * kBlock) {
        double sn, cs;
        sincos(gamma * cut_weighted(i, g, w.w), &sn, &cs);
        cx<R> a = psi[i];
        cx<R> r;
        r.x = (R)(a.x * cs + a.y * sn);
        r.y = (R)(a.y * cs - a.x * sn);
        psi[i] = r;
    }
}

int launch_cut_phase(qs_state *s, const Graph &g, const Weights *w, double gamma) {
    const u64 N = 1ull << s->n;
    u64 blocks = (N + kBlock * 16 - 1) / (kBlock * 16);
    if (blocks > 16384) blocks = 16384;
    const dim3 grid((unsigned)(blocks ? blocks : 1));
    if (w) {
        if (s->dtype == QS_C128)
            hipLaunchKernelGGL(k_cut_phase_w<double>, grid, dim3(kBlock), 0, s->stream, (cx<double> *)s->buf, N, g, *w, gamma);
        else
            hipLaunchKernelGGL(k_cut_phase_w<float>, grid, dim3(kBlock), 0, s->stream, (cx<float> *)s->buf, N, g, *w, gamma);
    } else if (s->n >= 12) {
        int c = s->n - 11 > 12 ? s->n - 11 : 12;  // at most 2048 blocks while the loop fits the table
        if (c > 8 + kCutLoopBits) c = 8 + kCutLoopBits;
        const dim3 cg((unsigned)(N >> c));
        if (s->dtype == QS_C128)
            hipLaunchKernelGGL(k_cut_phase_chunk<double>, cg, dim3(kBlock), 0, s->stream, (cx<double> *)s->buf, c, g, gamma);
        else
            hipLaunchKernelGGL(k_cut_phase_chunk<float>, cg, dim3(kBlock), 0, s->stream, (cx<float> *)s->buf, c, g, gamma);
    } else {
        if (s->dtype == QS_C128)
            hipLaunchKernelGGL(k_cut_phase<double>, grid, dim3(kBlock), 0, s->stream, (cx<double> *)s->buf, N, g, gamma);
        else
            hipLaunchKernelGGL(k_cut_phase<float>, grid, dim3(kBlock), 0, s->stream, (cx<float> *)s->buf, N, g, gamma);
    }
    QS_LAUNCH_CHECK("cut_phase");
    return QS_OK;
}

}  // namespace qs
