// Internal declarations shared by the host driver (hs_api.cpp) and the
// kernels (hs_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/hs.h"

namespace hs {

constexpr int kCard = 256;          // iSAX alphabet (8-bit symbols)
constexpr int kChunk = 64;          // points per refinement chunk (early-abandon granularity)
constexpr int kTile = 256;          // series per LB_SAX tile = threads per scan workgroup
constexpr uint32_t kInfBits = 0x7f800000u;  // +inf as float bits

// Relative slack on every prune comparison: a bound is compared against
// BSF_k * (1 + kSlack).  It covers float32 rounding of LB_SAX sums and of the
// refined distances (each well below 2e-6 relative).
constexpr double kSlack = 1e-5;

// Pool of candidate results per query: (distance bits << 32 | original id).
constexpr int kPoolMin = 4096;

// Everything a kernel needs to know about an index.
struct IndexView {
    const float* rows;        // [N][stride] leaf-ordered series, zero padded
    const uint32_t* ids;      // [N] original row id of each stored series
    const uint8_t* words;     // [N][wstride] iSAX symbols
    const int64_t* leaf_start;// [L + 1]
    const float4* env;        // [L][w] (mu_min, mu_max, sd_min, sd_max), rounded outward
    const float* beta;        // [257] float32 breakpoints, beta[0] = -inf, beta[256] = +inf
    int64_t N;
    int64_t L;
    int32_t n, w, stride, wstride;
};

// Query-side workspace carved out of the caller's buffer.
struct QueryWs {
    float* qrow;          // [Q][stride] zero-padded queries
    double* qstat;        // [Q][w][2] segment mean / std (FP64)
    float* lut;           // [Q][w][256] LB_SAX table: (n/w) * gap^2, rounded down
    float* lbe;           // [Q][L] LB_EAPCA^2, rounded down
    uint32_t* bsf;        // [Q] float bits of the current BSF_k (monotone, atomicMin)
    uint32_t* pool_cnt;   // [Q]
    uint32_t* flags;      // [Q] bit0 overflow, bit1 skip-sequential, bit2 non-finite query, bit3 redo
    uint32_t* kept;       // [Q] candidate leaves emitted for the main pass
    uint64_t* seed_key;   // [Q] largest (lbE bits, leaf) key among the seed leaves (0 if none)
    uint64_t* pool;       // [Q][P]
    unsigned long long* stats;  // [Q][8]
    uint64_t* items;      // [cap] (q << 32 | leaf)
    uint32_t* counters;   // [4]: 0 items, 1 work counter
    int64_t item_cap;
    int32_t P;
};

struct ScanParams {
    int32_t Q, k;
    float eapca_th;
    int32_t final_pass;
    int32_t n_seed;  // seed leaves per query: min(l_max, L)
};

// kernel launchers (hs_kernels.hip); all asynchronous on `st`
hipError_t launch_series_stats(const float* x, int64_t N, int32_t n, int32_t w, float2* st_out,
                               uint32_t* bad_flag, hipStream_t st);
hipError_t launch_gather_rows(const float* x, const uint32_t* perm, int64_t N, int32_t n, int32_t stride,
                              float* rows, uint32_t* ids, hipStream_t st);
hipError_t launch_words(const IndexView& ix, uint8_t* words, hipStream_t st);
hipError_t launch_envelopes(const IndexView& ix, float4* env, hipStream_t st);

hipError_t launch_query_prep(const IndexView& ix, const float* q, int32_t Q, const QueryWs& ws, hipStream_t st);
hipError_t launch_lb_eapca(const IndexView& ix, int32_t Q, const QueryWs& ws, hipStream_t st);
hipError_t launch_seed_select(const IndexView& ix, int32_t Q, int32_t l_max, const QueryWs& ws, hipStream_t st);
hipError_t launch_emit_main(const IndexView& ix, int32_t Q, bool redo_only, const QueryWs& ws, hipStream_t st);
hipError_t launch_leaf_scan(const IndexView& ix, const ScanParams& sp, const QueryWs& ws, int device_cus,
                            hipStream_t st);
hipError_t launch_merge(const IndexView& ix, const ScanParams& sp, bool redo_only, const QueryWs& ws,
                        int64_t* ids_out, float* d2_out, hs_query_stats* stats_out, hipStream_t st);
hipError_t launch_reset_counters(const QueryWs& ws, hipStream_t st);

}  // namespace hs
