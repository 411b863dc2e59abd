// hs_knn_exact_noalloc: the exact k-NN path of hs_knn_exact with its query
// workspace (counters, result pools, candidate slices, per-query tables) in
// one file-scope device array instead of a caller-provided buffer, for
// callers that cannot allocate device memory (code under graph capture,
// tight serving loops).  It runs the same kernels as hs_knn_exact.
//
// Host code never passes the array's name to a kernel or a copy: in host code
// the name is a host-side stand-in.  The array's device address is taken with
// hipGetSymbolAddress once per device, with that device current, on the first
// call there, and kept per device; each GPU holds its own copy of the array
// for the life of the process.  Every call on a GPU shares that GPU's array
// (the kernels clear what must start at zero), so calls that overlap on one
// GPU race.
#include <mutex>

#include "hs_host.h"

namespace {

constexpr int64_t kScratchBytes = (int64_t)128 << 20;  // HS_NOALLOC_SCRATCH_BYTES
constexpr int kMaxDevices = 64;
// candidate-list entries the array must still hold beside the fixed tables
constexpr int64_t kMinCandidates = 4096;

static_assert(kScratchBytes == HS_NOALLOC_SCRATCH_BYTES, "header and library disagree on the scratch size");

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of this device's array (taken once, then cached).
hs_status scratch_of(int device, void** out) {
    if (device < 0 || device >= kMaxDevices) return hs::fail(HS_EINVAL, "device %d out of range", device);
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return hs::fail(HS_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_ptr[device] = p;
    }
    *out = g_ptr[device];
    return HS_OK;
}

// The most candidate-list entries whose workspace layout fits the array.
int64_t fitting_candidates(const hs_index* idx, int32_t Q, int32_t k) {
    int64_t lo = 0, hi = (int64_t)1 << 31;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo + 1) / 2;
        if (hs::ws_layout(idx, Q, k, nullptr, nullptr, mid) <= kScratchBytes) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

}  // namespace

extern "C" {

hs_status hs_knn_exact_noalloc(hs_index* idx, const float* q_dev, int32_t Q, int32_t k, int64_t* ids_dev,
                               float* d2_dev, double* err_dev, void* stats_dev, void* stream) {
    if (!idx) return hs::fail(HS_EINVAL, "idx is NULL");
    if (Q < 0) return hs::fail(HS_EINVAL, "Q=%d < 0", Q);
    if (k < 1 || k > HS_KMAX) return hs::fail(HS_EINVAL, "k=%d out of range [1, %d]", k, HS_KMAX);
    if (Q == 0) return HS_OK;
    if (Q >= (1 << 24)) return hs::fail(HS_EINVAL, "Q=%d: at most 2^24 - 1 queries per call", Q);
    if (!q_dev || !ids_dev || !d2_dev) return hs::fail(HS_EINVAL, "NULL device pointer");
    int device = -1;
    HIP_TRY(hipGetDevice(&device));
    if (device != idx->device)
        return hs::fail(HS_EINVAL, "current device %d is not the index's device %d", device, idx->device);
    const int64_t cand = fitting_candidates(idx, Q, k);
    if (cand < kMinCandidates)
        return hs::fail(HS_EINVAL,
                        "Q=%d, k=%d: the query tables need more than the %lld-byte static scratch holds; "
                        "split the batch or use hs_knn_exact with a workspace",
                        Q, k, (long long)kScratchBytes);
    void* ws = nullptr;
    hs_status s = scratch_of(device, &ws);
    if (s) return s;
    hs::KnnCall c;
    s = hs::knn_prepare(idx, Q, k, ws, kScratchBytes, false, &c, cand);
    if (s) return s;
    hipStream_t st = (hipStream_t)stream;
    auto* stats_out = (hs_query_stats*)stats_dev;
    s = hs::knn_enqueue(c, q_dev, ids_dev, d2_dev, err_dev, stats_out, st, nullptr, nullptr);
    if (s) return s;
    return hs::knn_finish(c, ids_dev, d2_dev, err_dev, stats_out, st, nullptr);
}

}  // extern "C"
