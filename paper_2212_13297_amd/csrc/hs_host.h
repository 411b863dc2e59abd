// Host-side declarations shared by the C ABI implementation (hs_api.cpp) and
// the serving loop (hs_server.cpp).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "hs_internal.h"

struct hs_index {
    hs_params p;
    hs::IndexView view;
    int device = 0;
    int cus = 0;
    int64_t max_leaf = 0;
    int64_t index_bytes = 0;
    // the small tables, inside the caller's index memory
    int64_t* leaf_start_dev = nullptr;
    float4* env_dev = nullptr;
    float* beta_dev = nullptr;
    int64_t* part_start_dev = nullptr;
    uint32_t* part_leaf_dev = nullptr;
    int64_t* part_chunk_dev = nullptr;
    int64_t* chunk_start_dev = nullptr;
    float4* cenv_dev = nullptr;
    int filter_waves = 4;               // wavefronts of the filter kernel (candidate slices)
    std::vector<int64_t> part_start_host;  // [parts + 1] (host copy, for partial low-precision copies)
    hs::ShadowView shadow{};            // low-precision copy (caller-owned memory), kind 0 = none
};

namespace hs {
struct IndexLayout;
}

namespace hs {

// Records the message for hs_last_error (this thread) and returns code.
hs_status fail(hs_status code, const char* fmt, ...);

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess) return hs::fail(HS_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

int64_t align_up(int64_t v, int64_t a);

// Byte offsets of an index's arrays inside the caller's index memory.
struct IndexLayout {
    int64_t rows, ids, words, sig, flag, beta, leaf_start, env, part_start, part_leaf, part_chunk, chunk_start, cenv;
    int64_t scratch;      // the build's scratch (the rows' area when it fits)
    int64_t total;
    int64_t leaf_budget;  // leaves the tables hold
    int64_t chunk_cap;    // chunks (and parts) the tables hold
};
IndexLayout index_layout(int64_t N, const hs_params& p, char* base);

}  // namespace hs

// A streaming build in progress (hs_build_begin .. hs_build_finish).
struct hs_builder {
    hs_index* idx = nullptr;
    hs::IndexLayout lay{};
    hipStream_t st = nullptr;
    char* scratch = nullptr;
    uint32_t* bad = nullptr;     // NaN / Inf flag
    float2* st_dev = nullptr;    // [N][w] segment statistics (first pass)
    uint32_t* pos = nullptr;     // [N] stored position of each series (second pass)
    int stage = 0;               // 0: statistics, 1: rows
    int64_t next_row = 0;
};

namespace hs {

// Device leaf partition (hs_partition.hip).  The statistics [N][w] go into
// partition_stats_buffer(scratch) before the call; on return ids_out holds the
// original id of every stored position and *leaf_starts the sorted leaf starts.
int64_t partition_scratch_bytes(int64_t N, int w, int64_t tau, int64_t budget);
float2* partition_stats_buffer(char* scratch, int64_t N, int w, int64_t tau, int64_t budget);
hs_status partition_device(int64_t N, int w, int64_t tau, int64_t budget, char* scratch, int cus,
                           uint32_t* ids_out, std::vector<int64_t>* leaf_starts, hipStream_t st);

// Query workspace layout for Q queries (bytes; fills *ws when base is given).
// cand_total > 0 fixes the candidate-list entries (otherwise they follow the
// index's cand_per_query).
int64_t ws_layout(const hs_index* idx, int32_t Q, int32_t k, QueryWs* ws, char* base, int64_t cand_total = 0);

struct ScanTimer;

// One k-NN call, validated and laid out in its workspace.
struct KnnCall {
    hs_index* idx = nullptr;
    bool mixed = false;
    int form = kPlain;
    double err_rel = 0.0;
    QueryWs ws{};
    ScanParams sp{};
};

hs_status knn_prepare(hs_index* idx, int32_t Q, int32_t k, void* ws_dev, int64_t ws_bytes, bool mixed, KnnCall* c,
                      int64_t cand_total = 0);
hs_status knn_enqueue(const KnnCall& c, const float* q_dev, int64_t* ids_dev, float* d2_dev, double* err_dev,
                      hs_query_stats* stats_out, hipStream_t st, uint32_t* redo_host, ScanTimer* timer);
hs_status knn_finish(const KnnCall& c, int64_t* ids_dev, float* d2_dev, double* err_dev, hs_query_stats* stats_out,
                     hipStream_t st, ScanTimer* timer);

}  // namespace hs
