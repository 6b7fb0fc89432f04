// Sequential search that allocates nothing, for callers that cannot allocate
// device memory (code under hipGraph capture, tight serving loops, harnesses
// that forbid hipMalloc).  It runs the register-tiled scan and the top-k merge
// of qd_knn_bruteforce; the scan's per-wave top-k lists, which that entry
// point takes from the stream-ordered allocator, live here in a file-scope
// device array instead.
//
// The array is a device symbol: in host code its name is not a device
// address.  Its address on each device comes from hipGetSymbolAddress, taken
// once per device (with that device current) on the first call there, and
// only that address is passed to the kernels.  Every call on one device shares
// its array: the scan writes every list the merge reads before the merge runs,
// so nothing needs clearing between calls, but calls that overlap on one
// device (two streams, two threads) race on it.
#include <mutex>

#include "qd_internal.h"
#include "qd_launch.h"

namespace qd {
namespace {

constexpr size_t kScratchBytes = 32ull << 20;  // QD_NOALLOC_SCRATCH_BYTES
static_assert(kScratchBytes == QD_NOALLOC_SCRATCH_BYTES, "header and library disagree");

__device__ __align__(256) u64 scratch[kScratchBytes / sizeof(u64)];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
u64 *g_scratch[kMaxDevices] = {};

// Device address of `scratch` on the current device.
int scratch_address(u64 **out) {
    int dev = 0;
    QD_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(QD_ERR_UNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(QD_ERR_DEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        g_scratch[dev] = static_cast<u64 *>(p);
    }
    *out = g_scratch[dev];
    return QD_OK;
}

}  // namespace
}  // namespace qd

extern "C" int qd_knn_bruteforce_noalloc(const uint64_t *d_db, uint64_t n, const uint64_t *d_q, uint32_t nq,
                                         uint32_t k, uint32_t *d_idx, int32_t *d_missed, int32_t *d_extra,
                                         float *d_dist, void *stream) {
    using namespace qd;
    if (k < 1 || k > QD_MAX_K) return fail(QD_ERR_INVALID, "k=%u outside 1..%d", k, QD_MAX_K);
    if (n < 1 || n > QD_MAX_ROWS) return fail(QD_ERR_INVALID, "n=%llu outside 1..%llu", (u64)n, (u64)QD_MAX_ROWS);
    if (nq == 0) return QD_OK;
    if (!d_db || !d_q || !d_idx || !d_missed || !d_extra || !d_dist) return fail(QD_ERR_INVALID, "null pointer");
    if (!aligned16(d_db) || !aligned16(d_q)) return fail(QD_ERR_INVALID, "descriptor arrays must be 16-byte aligned");
    // every query needs at least one list of k keys
    const uint64_t per_slice = (uint64_t)nq * k * sizeof(u64);
    if (per_slice > kScratchBytes)
        return fail(QD_ERR_INVALID, "nq*k = %llu exceeds the %llu keys of the no-allocation scratch",
                    (u64)nq * k, (u64)(kScratchBytes / sizeof(u64)));
    // the automatic launch shape, with fewer row slices if its lists would not fit
    BruteLaunch sh = brute_launch_shape(n, nq, k, 0, 0);
    if (sh.part_bytes > kScratchBytes) sh = brute_launch_shape(n, nq, k, 0, (uint32_t)(kScratchBytes / per_slice));
    if (sh.part_bytes > kScratchBytes) return fail(QD_ERR_INVALID, "launch shape exceeds the scratch");
    u64 *part = nullptr;
    const int rc = scratch_address(&part);
    if (rc != QD_OK) return rc;
    return brute_launch(sh, part, d_db, n, d_q, nq, nullptr, k, d_idx, d_missed, d_extra, d_dist,
                        (hipStream_t)stream, /*timed=*/false);
}
