// Internal declarations shared by the host driver (hs_api.cpp) and the
// kernels (hs_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/hs.h"

namespace hs {

constexpr int kCard = 256;          // iSAX alphabet (8-bit symbols)
constexpr int kChunk = 64;          // points per refinement chunk (early-abandon granularity)
constexpr int kTile = 256;          // threads per scan / filter / refine workgroup
constexpr int kPartRows = 8192;     // series per work item: leaves are cut into parts of at most this many
constexpr int kChunkRows = 64;      // series per chunk envelope (one wavefront's rows in the filter)
constexpr uint32_t kInfBits = 0x7f800000u;  // +inf as float bits
// result key bound before any result: distance +inf, the largest id
constexpr unsigned long long kInfKey = ((unsigned long long)kInfBits << 32) | 0xffffffffull;
constexpr int kMaxSeedLeaves = 64;  // l_max is clamped to this many leaves in the seed step

// Relative slack on every prune comparison: a bound is compared against
// BSF_k * (1 + kSlack).  It covers float32 rounding of LB_SAX sums and of the
// refined distances (each well below 2e-6 relative).
constexpr double kSlack = 1e-5;

// Pool of candidate results per query: (distance bits << 32 | original id).
constexpr int kPoolMin = 4096;

// query flags
constexpr uint32_t kFlagOverflow = 1;    // the result pool overflowed in this round
constexpr uint32_t kFlagCandLost = 2;    // candidates were dropped (candidate buffer full)
constexpr uint32_t kFlagNonFinite = 4;   // the query holds NaN or Inf
constexpr uint32_t kFlagRedo = 8;        // needs another round
constexpr uint32_t kFlagInRound = 16;    // takes part in the current redo round
constexpr uint32_t kFlagSkipSax = 32;    // skip-sequential path: no LB_SAX filter

// counters[] slots
constexpr int kCtrItems = 0;     // items emitted
constexpr int kCtrWork = 1;      // work-distribution counter of the filter / scan kernels
constexpr int kCtrRedo = 2;      // queries that need another round
constexpr int kCtrNonFinite = 3; // queries with NaN / Inf
constexpr int kCtrCand = 4;      // candidates appended by the filter
constexpr int kCtrRefine = 5;    // work-distribution counter of the refine kernel
constexpr int kCtrOvf = 6;       // entries reserved in the overflow slice
constexpr int kCtrOvfEnd = 7;    // smallest base of an overflow range that did not fit (UINT32_MAX if none):
                                 // overflow entries at or above it were never written
constexpr int kCtrBound = 8;     // 8 slots: the bounding pass's work counter of each XCD
constexpr int kCtrLost = 16;     // queries of the last merge whose candidates were dropped
constexpr int kNumCounters = 17;
constexpr int kStatSlots = 16;   // per-query counters in the workspace (hs_query_stats reads 10)

// Distance forms of the refinement (template argument F of the kernels that
// refine): float32 sum in a fixed order, or compensated float32 (error-free
// transformations on every step, error ~2^-23 relative).
constexpr int kPlain = 0;
constexpr int kComp = 1;

// Low-precision copy of the series (precision form)
constexpr int kShadowBf16 = 1;  // HS_SHADOW_BF16
constexpr int kShadowF16 = 2;   // HS_SHADOW_FP16
constexpr int kBoundQueries = 128;  // queries per workgroup of the bounding pass (4 wavefronts x 32)
constexpr int kBoundRows = 32;      // series per tile of the bounding pass

struct ShadowView {
    const uint16_t* rows;  // [rows_n + kBoundRows][stride] bf16 / fp16 bits of the first rows_n stored series, zero padded
    const float4* norms;   // [N + kBoundRows] (beta, ||x - x~||_2 rounded up, ||x~||^2 rounded down, aug), float32;
                           // beta = ((1 - g) ||x~||^2 - eps^2) / 2 - 3u (||x~||^2 + eps^2), float64, rounded down;
                           // aug: bits of the augmented unit (a*, ebar) as two low-precision values
    int32_t kind;          // kShadowBf16 / kShadowF16
    int64_t rows_n;        // stored series the copy holds: all N, or the first parts_n parts
    int64_t parts_n;       // parts wholly in the copy (the rest take the LB_SAX filter)
};

// Everything a kernel needs to know about an index.
struct IndexView {
    const float* rows;         // [N][stride] leaf-ordered series, zero padded
    const uint32_t* ids;       // [N] original row id of each stored series
    const uint8_t* words;      // [N][wstride] iSAX symbols
    const uint8_t* sig;        // [N][wstride] deviation codes: segment std in [c sig_h, (c + 1) sig_h]
    const int64_t* leaf_start; // [L + 1]
    const float4* env;         // [L][w] (mu_min, mu_max, sd_min, sd_max), rounded outward
    const float* beta;         // [257] float32 breakpoints, beta[0] = -inf, beta[256] = +inf
    const int64_t* part_start; // [parts + 1] rows of part p: [part_start[p], part_start[p + 1])
    const uint32_t* part_leaf; // [parts] leaf of each part
    const int64_t* part_chunk; // [parts] first chunk of each part
    const float4* cenv;        // [chunks][w] chunk envelopes, same layout as env
    int64_t N;
    int64_t L;
    int64_t parts;
    int64_t chunks;
    int32_t n, w, stride, wstride;
    float sig_h;               // width of a deviation code (at most 16 significant bits)
};

// Query-side workspace carved out of the caller's buffer.
struct QueryWs {
    float* qrow;          // [Q][stride] zero-padded queries
    double* qstat;        // [Q][w][2] segment mean / std (FP64)
    float4* qst32;        // [Q][w] float32 intervals holding them: (mu_lo, mu_hi, sd_lo, sd_hi)
    float* lut;           // [Q][w][256] LB_SAX table: (n/w) * gap^2, rounded down
    float* lbe;           // [Q][L] LB_EAPCA^2, rounded down
    // [Q] the smallest k-th result key (d bits << 32 | id) known so far, an
    // upper bound of the final k-th key (monotone, atomicMin); its high word
    // is BSF_k as float bits
    unsigned long long* bkey;
    uint32_t* pool_cnt;   // [Q]
    uint32_t* flags;      // [Q] kFlag* bits
    uint32_t* kept;       // [Q] candidate leaves after the leaf filter
    uint64_t* pool;       // [Q][P]
    unsigned long long* stats;  // [Q][kStatSlots]
    uint64_t* items;      // [item_cap] (q << 32 | part)
    // filter output: one private slice per filter wavefront
    uint32_t* slice_pos;  // [n_slices][slice_cap] stored position of a candidate series
    uint32_t* slice_q;    // [n_slices][slice_cap] its query
    uint32_t* slice_part; // [n_slices][slice_cap] its lower bound by quarters (LB_SAX plus the deviation term, or the precision form's bound in the first): four bytes, the high bytes of fp16 values rounded toward zero
    uint32_t* slice_cnt;  // [n_slices] entries written in each slice
    uint32_t* slice_start;// [n_slices + 1] exclusive prefix of slice_cnt
    uint32_t* counters;   // [kNumCounters]
    // precision form
    uint16_t* qlow;       // [Qpad][stride] low-precision queries (zero rows beyond Q)
    double2* qnorm;       // [Q] (||q~||^2, ||q - q~||_2 rounded up)
    // bounding pass: per part, the queries that keep its leaf
    uint32_t* plist;      // [parts][Q] the part's list, in query order
    uint32_t* pcnt;       // [parts] its length
    uint32_t* pnb;        // [parts + 1] its blocks of kBoundQueries (work items)
    uint32_t* pbo;        // [parts + 2] exclusive prefix of pnb: the part's first work item
    uint32_t* pscan;      // scan scratch
    int32_t Qpad;         // Q rounded up to kBoundQueries
    int64_t item_cap;
    int64_t slice_cap;    // entries per slice
    int64_t ovf_cap;      // entries of the shared overflow slice (slice index n_slices)
    int32_t n_slices;     // all slices; with a partial low-precision copy the
                          // bounding pass writes the upper half, the filter the lower
    int32_t P;
    // batch-union diagnostics (NULL when off): one bit per distinct unit read,
    // raw (series, 64-point chunk) pairs at bit pos * nchunks + c, then
    // series whose word was read at bit word_bit0 + pos, then chunk envelopes
    // at bit env_bit0 + chunk
    uint32_t* ubits;
    int64_t word_bit0, env_bit0;
};

struct ScanParams {
    int32_t Q, k;
    float eapca_th;
    int32_t final_pass;
    int32_t n_seed;     // seed leaves per query: min(l_max, L, kMaxSeedLeaves)
    int32_t seed_rows;  // series refined by the seed step
    // chunk order of the refine: -1 natural order; otherwise log2 of the
    // chunks per quarter of the series (stride = n = 256 2^order_lg, w a
    // multiple of 16)
    int32_t order_lg;
    int64_t emit_part0;   // first part k_emit makes items for (a partial copy's uncovered parts)
    int32_t slice0;       // first slice of the kernel that runs (filter or bounding pass)
    int32_t slices;       // slices it owns
    // abandoning margin: a running distance (any chunk order, either form,
    // plus the cascade's bounds of unread quarters) above fl(limit * marg)
    // proves the pair's result key, its compensated natural-order distance,
    // above the limit.  marg >= (1 + g) / ((1 - u)(1 - e_c)): g bounds the
    // running sum's relative excess over the exact distance (m + 12 roundings
    // for m chunks), e_c the compensated distance's relative error, u = 2^-24
    // the rounding of the product
    float marg;
    // a short candidate list is split into one range per wavefront, of at
    // least this many candidates (the refine sets it per form)
    int32_t min_range;
};

// bits of the batch-union array for an index: raw chunk pairs, words, envelopes
inline int64_t union_bits(const IndexView& ix) {
    return ix.N * (int64_t)(ix.stride / kChunk) + ix.N + ix.chunks;
}

// kernel launchers (hs_kernels.hip); all asynchronous on `st`
hipError_t launch_series_stats(const float* x, int64_t N, int32_t n, int32_t w, float2* st_out,
                               uint32_t* bad_flag, hipStream_t st);
hipError_t launch_gather_rows(const float* x, const uint32_t* perm, int64_t N, int32_t n, int32_t stride,
                              float* rows, hipStream_t st);
// pos[ids[i]] = i
hipError_t launch_inverse_ids(const uint32_t* ids, int64_t N, uint32_t* pos, hipStream_t st);
// rows[pos[row0 + r]] = x[r] (zero padded to stride), r < count
hipError_t launch_scatter_rows(const float* x, int64_t row0, int64_t count, const uint32_t* pos, int32_t n,
                               int32_t stride, float* rows, hipStream_t st);
hipError_t launch_words(const IndexView& ix, uint8_t* words, uint8_t* sig, hipStream_t st);
// Largest segment standard deviation of the statistics (float2 (mean, std)
// each, std >= 0) as float bits, by atomicMax into *out.
hipError_t launch_max_sigma(const float2* st, int64_t count, uint32_t* out, hipStream_t st_);
hipError_t launch_read_probe(const void* buf, int64_t bytes, uint32_t* sink, int device_cus, hipStream_t st);
hipError_t launch_lds_probe(int pattern, int32_t rounds, uint32_t* sink, int device_cus, hipStream_t st);
hipError_t launch_envelopes(const IndexView& ix, const int64_t* starts, int64_t count, float4* env,
                            hipStream_t st);

hipError_t launch_query_prep(const IndexView& ix, const float* q, int32_t Q, const QueryWs& ws, hipStream_t st);
hipError_t launch_lb_eapca(const IndexView& ix, int32_t Q, const QueryWs& ws, hipStream_t st);
hipError_t launch_seed(const IndexView& ix, const ScanParams& sp, const QueryWs& ws, int form, hipStream_t st);
hipError_t launch_emit(const IndexView& ix, const ScanParams& sp, bool redo_only, const QueryWs& ws,
                       hipStream_t st);
// wavefronts the filter launches for this index (one private candidate slice each)
int filter_waves(const IndexView& ix, int device_cus);
hipError_t launch_filter(const IndexView& ix, const ScanParams& sp, const QueryWs& ws, int device_cus,
                         hipStream_t st);
// where each of the filter's slices starts in the candidate list (their concatenation)
hipError_t launch_slice_prefix(const QueryWs& ws, hipStream_t st);
hipError_t launch_refine(const IndexView& ix, const ScanParams& sp, const QueryWs& ws, int device_cus, int form,
                         hipStream_t st);
hipError_t launch_leaf_scan(const IndexView& ix, const ScanParams& sp, const QueryWs& ws, int device_cus, int form,
                            hipStream_t st);
// err_out (may be NULL): err_rel * d2 per result
// counts[0..2] = marked raw chunk pairs, words, envelopes of a batch-union array
hipError_t launch_union_count(const IndexView& ix, const uint32_t* bits, unsigned long long* counts, hipStream_t st);
hipError_t launch_merge(const IndexView& ix, const ScanParams& sp, bool redo_only, const QueryWs& ws,
                        int64_t* ids_out, float* d2_out, double* err_out, double err_rel, hs_query_stats* stats_out,
                        hipStream_t st);

// precision form (hs_precision.hip)
hipError_t launch_shadow(const IndexView& ix, int kind, int64_t nrows, uint16_t* rows, float4* norms,
                         uint32_t* bad_flag, hipStream_t st);
hipError_t launch_query_low(const IndexView& ix, int kind, int32_t Q, const QueryWs& ws, hipStream_t st);
hipError_t launch_bound(const IndexView& ix, const ShadowView& sv, const ScanParams& sp, const QueryWs& ws,
                        int device_cus, hipStream_t st);
// out[i] = in[0] + .. + in[i - 1], out[n] = the total (n + 1 entries); bsum
// holds n / 1024 + 2 entries of scratch
hipError_t launch_exclusive_scan(const uint32_t* in, int64_t n, uint32_t* out, uint32_t* bsum, hipStream_t st);

}  // namespace hs
