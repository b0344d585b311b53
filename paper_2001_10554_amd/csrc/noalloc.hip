// Allocation-free sampling: qs_sample on a register given by pointer, with its
// partial sums in a fixed device array instead of a handle's scratch, for
// callers that cannot allocate device memory (graph capture, serving loops).
//
// The array lives in the code object, so every device the library runs on
// holds one copy until the process ends.  Host code never passes the array's
// name to a kernel: its device address is looked up once per device with
// hipGetSymbolAddress and kept per device.  All calls on one device share the
// array, so calls that overlap on one device (different streams, or several
// host threads) race; calls ordered on one stream do not.  Every element a
// call reads is written earlier in the same call, so nothing needs clearing.
#include <mutex>

#include "launch.h"

#define QS_API extern "C" __attribute__((visibility("default")))

namespace qs {

// Chunk sums and their prefix for at most 2^18 chunks (the chunk count of
// every register size up to the per-device limit), plus the last-chunk slot.
constexpr size_t kNoAllocChunks = (size_t)1 << 18;
constexpr size_t kNoAllocDoubles = 2 * kNoAllocChunks + 64;  // 4 MiB + 512 B

static __device__ __align__(256) double scratch[kNoAllocDoubles];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_dev[kMaxDevices];  // device address of `scratch`, per device

// The calling thread's current device's copy of the array.
static int scratch_on_current_device(double **out) {
    int dev = -1;
    QS_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(QS_ERR_UNSUPPORTED, "device index above the library's limit");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(QS_ERR_HIP, "hipGetSymbolAddress(scratch) returned null");
        g_scratch_dev[dev] = (double *)p;
    }
    *out = g_scratch_dev[dev];
    return QS_OK;
}

}  // namespace qs

using namespace qs;

QS_API int qs_sample_noalloc(int n, int dtype, const void *dev_buf, size_t buf_bytes, int64_t shots, uint64_t seed, uint64_t *out_dev,
                             void *stream) {
    try {
        if (dtype != QS_C64 && dtype != QS_C128) return fail(QS_ERR_DTYPE, "dtype must be QS_C64 or QS_C128");
        if (n < 1) return fail(QS_ERR_ARG, "n must be >= 1");
        const int nmax = dtype == QS_C128 ? QS_MAX_QUBITS_C128 : QS_MAX_QUBITS_C64;
        if (n > nmax) return fail(QS_ERR_SIZE, "n above the per-device limit");
        const size_t chunks = (size_t)1 << (n - sample_chunk_bits(n));
        if (2 * chunks + 1 > kNoAllocDoubles) return fail(QS_ERR_SIZE, "register needs more than the fixed sampling scratch");
        if (!dev_buf) return fail(QS_ERR_ARG, "null state buffer");
        if (buf_bytes < ((size_t)1 << n) * amp_bytes(dtype)) return fail(QS_ERR_SIZE, "state buffer smaller than 2^n amplitudes");
        if (shots < 0 || shots > ((int64_t)1 << 32)) return fail(QS_ERR_ARG, "shots must be in [0, 2^32]");
        if (shots > 0 && !out_dev) return fail(QS_ERR_ARG, "null output");
        double *sc = nullptr;
        if (int rc = scratch_on_current_device(&sc)) return rc;
        return launch_sample_buf(n, dtype, dev_buf, sc, (hipStream_t)stream, shots, seed, out_dev);
    } catch (...) {
        return fail(QS_ERR_UNSUPPORTED, "unexpected internal error");
    }
}
