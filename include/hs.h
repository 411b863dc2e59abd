/*
 * hs.h -- C ABI of the HIP library for exact data-series k-NN search
 * (filter-and-refine over a collection resident in GPU memory).
 *
 * Method: Hercules (Echihabi et al., PVLDB 15(10), 2022), Sec. 3.4 query
 * answering: a per-leaf LB_EAPCA bound over segment mean/std envelopes, a
 * per-series LB_SAX bound (PAA over w segments against Gaussian breakpoints,
 * alphabet 256), and exact squared-Euclidean refinement with a running k-th
 * best-so-far distance (BSF_k) and early abandoning.
 *
 * Conventions for every entry point:
 *  - Pointers named *_dev are device pointers; pointers without the suffix are
 *    host pointers.  The caller owns and frees every device buffer (input
 *    series, index memory -- which also holds the index's tables and the
 *    build's scratch --, low-precision copy, query workspace, outputs).  The
 *    library owns only opaque host handles (index, server, scheduler) and
 *    calls no device allocator (hs_knn_exact_noalloc's static array aside).
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *    device work is enqueued on it.  hs_build_summaries synchronises the
 *    stream (the leaf partition runs on the host); hs_knn_exact synchronises
 *    it once, at the end, to read the pool-overflow flags (see below).
 *  - Return value: HS_OK (0) or a negative hs_status.  Argument errors are
 *    detected before any work is enqueued.  On failure hs_last_error()
 *    returns a thread-local, NUL-terminated message.  No C++ exception
 *    crosses the ABI.
 *  - Inputs are not z-normalised by the library (the paper normalises data
 *    and queries up front; callers do it).
 */
#ifndef HS_H
#define HS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t hs_status;
#define HS_OK 0
#define HS_EINVAL (-1)   /* invalid argument (sizes, NULL pointers, non-finite input) */
#define HS_ENOMEM (-2)   /* caller-provided buffer too small, or host allocation failed */
#define HS_EHIP (-3)     /* a HIP runtime call failed */
#define HS_EBUSY (-4)    /* no free slot (hs_submit, hs_sched_submit); request already running (hs_cancel) */
#define HS_ECANCEL (-5)  /* status of a completion whose request was withdrawn by hs_cancel */

/* Largest k accepted by hs_knn_exact (the per-workgroup top-k lives in LDS). */
#define HS_KMAX 128

/*
 * Index parameters.
 *  n          series length (points), 1 <= n <= 16384.
 *  w          PAA / iSAX segments, 1 <= w <= 64, w divides n (Sec. 2: PAA
 *             uses equal-length segments; the paper uses 16).
 *  card_bits  bits per iSAX symbol; must be 8 (alphabet 256, Sec. 2).
 *  leaf_size  leaf capacity tau (Sec. 3.2): a node holding more than tau
 *             series is split, unless no H-split separates its series.
 *  l_max      leaves visited by the approximate search that seeds BSF_k
 *             (Sec. 3.4 step 1; the paper's default is 1), 0 <= l_max;
 *             values above 64 are treated as 64.  0 = no seed.
 *  seed_rows  series of those leaves refined by the seed: the ones with the
 *             smallest LB_SAX, at least max(seed_rows, 2k) of them (the
 *             paper refines the whole leaves).  Access-path choice only.
 *  eapca_th   Sec. 3.4 threshold: a query whose leaf pruning ratio is below
 *             it skips the LB_SAX filter and scans its candidate leaves.
 *             Access-path choice only; results do not depend on it.
 *  cand_per_query  candidate-list entries reserved per query in the query
 *             workspace (0 = max(N/8, 4096)).  A query whose LB_SAX
 *             survivors do not fit is answered by the fused filter+refine
 *             kernel instead; results do not depend on it.
 *  build_flags  0, or HS_BUILD_HOST_PARTITION: partition the series on the
 *             host (the reference the device partition is tested against;
 *             needs N * w * 16 bytes of host memory) instead of on the device.
 *             Both give the same leaves and order.
 *  reserved   0.
 * Every field is validated by hs_index_bytes / hs_build_summaries.
 */
#define HS_BUILD_HOST_PARTITION 1
typedef struct {
    int32_t n;
    int32_t w;
    int32_t card_bits;
    int32_t leaf_size;
    int32_t l_max;
    int32_t seed_rows;
    float eapca_th;
    int32_t cand_per_query;
    int32_t build_flags;
    int32_t reserved;
} hs_params;

typedef struct hs_index hs_index; /* opaque, library-owned host handle */

/* Properties of a built index. */
typedef struct {
    int64_t n_series;    /* N */
    int32_t n;           /* series length */
    int32_t w;           /* PAA segments */
    int32_t row_stride;  /* floats per stored row (n rounded up to 64) */
    int32_t word_stride; /* bytes per stored iSAX word (w rounded up to 16) */
    int64_t n_leaves;    /* L */
    int64_t max_leaf;    /* largest leaf (series) */
    int64_t index_bytes; /* device bytes the index occupies */
    int64_t n_chunks;    /* 64-series chunks (each leaf cut from its first series) */
    double sigma_step;   /* width h of the deviation codes: the std of segment i of a stored
                            series lies in [c h, (c + 1) h], c its code (uint8, stored after the
                            words in the same layout) */
} hs_index_info;

/*
 * Device bytes hs_build_summaries needs in `index_mem_dev` for N series:
 * the leaf-ordered copy of the series (the LRDFile analogue, Sec. 3.3),
 * the iSAX words in the same order (the LSDFile analogue), the id map,
 * the leaf, part and chunk tables with their envelopes (sized for at most
 * min(N, 4 ceil(N / leaf_size) + 1024) leaves: the device partition stops
 * splitting nodes into more leaves than that), and the build's scratch,
 * which shares the rows' area when it fits there (it does whenever
 * row_stride * 4 >= w * 16 + 64 bytes or so).  The library allocates no
 * device memory of its own.
 * Errors: HS_EINVAL for N < 1, N >= 2^32, or invalid params.
 */
hs_status hs_index_bytes(int64_t N, const hs_params* params, int64_t* bytes);

/*
 * Build the index over x_dev (float32 [N][n], row-major, read only).
 * Computes per series the EAPCA segment statistics and the iSAX word
 * (Sec. 2), partitions the series into leaves by mean/std midpoint H-splits
 * (Sec. 3.2; see DESIGN notes for the split policy), stores the series in
 * leaf order, and computes every leaf's synopsis (Sec. 3.2, min/max of
 * segment mean and std, rounded outward to float32).
 * The partition runs on the device, level by level (all nodes of one depth
 * together); HS_BUILD_HOST_PARTITION runs it on the host instead.
 * x_dev may be freed after the call returns.  index_mem_dev must hold
 * hs_index_bytes() bytes and stay allocated until hs_index_free.
 * Errors: HS_EINVAL (NULL pointers, bad params, N out of range, non-finite
 * values in x), HS_ENOMEM (index_bytes too small, host memory, or a host
 * partition with more leaves than the tables hold), HS_EHIP.
 */
hs_status hs_build_summaries(const float* x_dev, int64_t N, const hs_params* params,
                             void* index_mem_dev, int64_t index_bytes, void* stream,
                             hs_index** out);

/*
 * Streaming build: the same index as hs_build_summaries, for collections that
 * do not fit in device memory twice (as input and as the leaf-ordered copy).
 * The series arrive in row chunks, twice: first for their segment statistics
 * (the partition's input), then, after hs_build_partition, for their values,
 * which go straight to their stored positions.  Each pass covers rows
 * [0, N) in order (chunk i starts where chunk i - 1 ended), with the same
 * values both times; a chunk's device memory may be reused once the call
 * returns and the stream has passed it (calls are stream-ordered).
 *   hs_build_begin      validates like hs_build_summaries (index memory of
 *                       hs_index_bytes bytes, caller-owned)
 *   hs_build_add_stats  x_dev: float32 [rows][n], rows row0 .. row0 + rows - 1
 *   hs_build_partition  after the first pass; synchronises the stream
 *   hs_build_add_rows   the second pass
 *   hs_build_finish     words and envelopes; returns the index and frees the
 *                       builder
 *   hs_build_abort      frees a builder that will not finish
 * Errors: HS_EINVAL (NULL, chunks out of order or range, a step out of turn,
 * NaN/Inf in the series -- reported by hs_build_partition), HS_ENOMEM,
 * HS_EHIP.  After an error the builder may only be aborted.
 */
typedef struct hs_builder hs_builder;
hs_status hs_build_begin(int64_t N, const hs_params* params, void* index_mem_dev, int64_t index_bytes, void* stream,
                         hs_builder** out);
hs_status hs_build_add_stats(hs_builder* b, const float* x_dev, int64_t row0, int64_t rows);
hs_status hs_build_partition(hs_builder* b);
hs_status hs_build_add_rows(hs_builder* b, const float* x_dev, int64_t row0, int64_t rows);
hs_status hs_build_finish(hs_builder* b, hs_index** out);
hs_status hs_build_abort(hs_builder* b);

/* Properties of a built index (host copy). */
hs_status hs_get_info(const hs_index* idx, hs_index_info* out);

/* Copy the leaf table and the leaf synopses to host memory (synchronous).
 * leaf_start: int64 [L + 1], leaf i holds stored positions
 *             [leaf_start[i], leaf_start[i+1]);
 * env:        float32 [L][w][4] = (mu_min, mu_max, sd_min, sd_max) per
 *             segment (Sec. 3.2 synopsis), rounded outward.
 * Either pointer may be NULL.  Errors: HS_EINVAL, HS_EHIP. */
hs_status hs_get_leaves(const hs_index* idx, int64_t* leaf_start, float* env);

/* Copy the chunk table and the chunk envelopes to host memory (synchronous).
 * Inside a leaf the series are ordered by further mean/std midpoint splits
 * down to 64 series (Sec. 3.2 splitting rule, below the leaf level), and each
 * leaf is cut into consecutive chunks of 64 series from its first one.
 * chunk_start: int64 [n_chunks + 1]; cenv: float32 [n_chunks][w][4], the
 * chunk's (mu_min, mu_max, sd_min, sd_max) per segment, rounded outward.
 * Either pointer may be NULL.  Errors: HS_EINVAL, HS_EHIP. */
hs_status hs_get_chunks(const hs_index* idx, int64_t* chunk_start, float* cenv);

/* Device bytes of query workspace hs_knn_exact needs for Q queries and k. */
hs_status hs_query_workspace_bytes(const hs_index* idx, int32_t Q, int32_t k, int64_t* bytes);

/*
 * Per-query counters written by hs_knn_exact when stats_dev is not NULL
 * (uint64 each).  Byte figures are algorithmic: what the method reads.
 */
typedef struct {
    uint64_t leaves_kept;     /* candidate leaves after LB_EAPCA (seed leaves included) */
    uint64_t rows_filtered;   /* series whose LB_SAX was evaluated */
    uint64_t rows_refined;    /* series whose raw values were read */
    uint64_t chunks_read;     /* 64-point chunks of raw values read (early abandoning stops early) */
    uint64_t path;            /* 0 = LB_SAX path, 1 = skip-sequential (no LB_SAX) */
    uint64_t rounds;          /* refinement rounds (1 unless the candidate pool overflowed) */
    uint64_t candidates;      /* series put on the candidate list (two-stage path): LB_SAX survivors
                                 whose bound with the deviation term also stays within the threshold */
    uint64_t chunks_tested;   /* 64-series chunk envelopes whose LB_EAPCA was evaluated */
    uint64_t rows_bounded;    /* precision form: series of the low-precision copy whose matrix-core
                                 bound was evaluated for this query (0 in the plain form) */
    uint64_t bound_pairs;     /* precision form: series whose dot product with this query the matrix
                                 cores computed (every series of the parts its wavefront took,
                                 padding lanes counted with the wavefront's first query) */
    uint64_t rows_sigma;      /* LB_SAX survivors whose deviation codes were read to add the
                                 deviation term (two-stage path) */
} hs_query_stats;

/*
 * Exact k-NN of Q queries (Sec. 2 k-NN definition; Sec. 3.4 Exact-kNN).
 *  q_dev     float32 [Q][n] queries, row-major.
 *  ws_dev    workspace of at least hs_query_workspace_bytes(idx, Q, k).
 *  ids_dev   int64 [Q][k] out: original row indices of x_dev.
 *  d2_dev    float32 [Q][k] out: squared Euclidean distances, each the
 *            compensated float32 sum of the pair (error-free transformations
 *            on every step, a fixed natural order), so a pair always gets the
 *            same value whatever the batch or the access path.
 *  err_dev   float64 [Q][k] out, or NULL: a-priori bound of |d2 - d| for
 *            each result, d the exact squared distance:
 *            (2^-23 + (4 K + 64) 2^-48) d2 for K = row_stride stored points.
 *  stats_dev hs_query_stats [Q] out, or NULL.
 * Each query's results are sorted by (d2, id) ascending and are the exact k
 * nearest series by d2.  Early abandoning tests a cheaper running sum against
 * the limit times a margin that covers its larger error, so no series whose
 * d2 is within the limit is abandoned.  With d2 within 1.2e-7 relative of d,
 * the id set differs from the exact k-NN only among series whose exact
 * distances lie within 2.4e-7 relative of the k-th.
 * Errors: HS_EINVAL (k < 1, k > HS_KMAX, k > N, Q < 0, Q >= 2^24, NULL
 * pointers, NaN/Inf in a query), HS_ENOMEM (workspace too small), HS_EHIP.
 */
hs_status hs_knn_exact(hs_index* idx, const float* q_dev, int32_t Q, int32_t k, void* ws_dev,
                       int64_t ws_bytes, int64_t* ids_dev, float* d2_dev, double* err_dev, void* stats_dev,
                       void* stream);

/*
 * hs_knn_exact without a workspace argument and without any device memory
 * allocation, for callers that cannot allocate (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  The query
 * workspace lives in a static device array of HS_NOALLOC_SCRATCH_BYTES that
 * the library holds on each GPU it runs on until the process ends.  Same
 * kernels and results as hs_knn_exact (ids, d2, err and stats bit for bit);
 * the candidate list is sized to what the array holds beside the per-query
 * tables, so more queries may take the overflow rounds, which do not change
 * results.  The calling thread's current device must be the index's.  Every
 * call on a GPU shares that GPU's array: calls that overlap on one GPU (other
 * streams or threads) race and must be serialised by the caller.
 * Synchronises the stream once, at the end, like hs_knn_exact.
 * Errors: as hs_knn_exact; HS_EINVAL also when Q queries at this k need more
 * per-query tables than the array holds (split the batch), or when the
 * current device is not the index's.
 */
#define HS_NOALLOC_SCRATCH_BYTES (128LL << 20)
hs_status hs_knn_exact_noalloc(hs_index* idx, const float* q_dev, int32_t Q, int32_t k, int64_t* ids_dev,
                               float* d2_dev, double* err_dev, void* stats_dev, void* stream);

/*
 * Precision form (beside the paper's method; it returns the same exact k-NN).
 * A low-precision copy x~ of every stored series (bf16 or fp16, round to
 * nearest even) replaces LB_SAX as the per-series filter of Sec. 3.4 step 3:
 * a matrix-core pass computes q~.x~ in float32 for every (query, series)
 * pair of the candidate leaves and derives a rigorous lower bound of the
 * squared distance,
 *   LB = max(0, sqrt((1-g)(||q~||^2 + ||x~||^2) - 2 q~.x~) - eps_q - eps_x)^2,
 * eps = ||v - v~||_2, g = K 2^-23 / (1 - K 2^-23) for K = row_stride
 * (float32 accumulation error), evaluated in float64 for every pair that a
 * float32 test with proven margins does not already drop.  Pairs with
 * LB <= BSF_k (1 + 1e-5) are refined from the float32 series with a
 * compensated float32 distance (TwoSum / exact-product transformations).
 */
#define HS_SHADOW_BF16 1
#define HS_SHADOW_FP16 2

/* Device bytes of the low-precision copy of kind HS_SHADOW_*: (R + 32) x
 * row_stride 16-bit values and (R + 32) x 16 bytes of per-series constants
 * (the last 32 rows are zero padding), plus 256 bytes of scratch.  R is the
 * number of stored series the copy holds: all N when shadow_rows < 0 or
 * shadow_rows >= N; otherwise the series of the whole work parts (leaf
 * pieces of at most 8192 series, in stored order) that fit in the first
 * shadow_rows -- a partial copy for collections whose full copy does not fit
 * beside the float32 series.
 * Errors: HS_EINVAL (NULL, unknown kind). */
hs_status hs_shadow_bytes(const hs_index* idx, int32_t kind, int64_t shadow_rows, int64_t* bytes);

/* Build the low-precision copy of (the first R stored series, as for
 * hs_shadow_bytes, of) the index into caller-owned device memory shadow_dev
 * (hs_shadow_bytes bytes, kept allocated until hs_index_free or the next
 * hs_build_shadow).  With a partial copy, hs_knn_mixed bounds the series the
 * copy holds on the matrix cores and filters the others by LB_SAX, both
 * feeding one candidate list refined in the compensated form (same results);
 * the query workspace then holds twice the candidate slices, so
 * hs_query_workspace_bytes is to be taken after this call.
 * Per series it stores x~ in leaf order and four floats:
 * beta (the series' term of the bounding pass's float32 test, computed in
 * float64 from the next two, rounded down), ||x - x~||_2 (float64, stored
 * rounded up), ||x~||^2 (float64, stored rounded down) and, for series of
 * at most 256 points, the augmented unit: two low-precision values (a* in the
 * low 16 bits, ebar >= ||x - x~||_2 in the high 16 bits) that the bounding
 * pass's extra matrix-core step adds, a* covering -(||x~||^2 - eps^2)/2 plus
 * the series' share of the accumulation error bound.  Synchronises the
 * stream.  An index holds one copy; a new
 * call replaces it.
 * Errors: HS_EINVAL (NULL, unknown kind, a value beyond the fp16 range for
 * HS_SHADOW_FP16), HS_ENOMEM (shadow_bytes too small), HS_EHIP. */
hs_status hs_build_shadow(hs_index* idx, int32_t kind, int64_t shadow_rows, void* shadow_dev, int64_t shadow_bytes,
                          void* stream);

/*
 * Exact k-NN of Q queries through the precision form.  Arguments, result
 * keys (the compensated float32 distance d2) and error bounds as for
 * hs_knn_exact (same workspace size): the ids and distances equal
 * hs_knn_exact's.
 * Errors: as hs_knn_exact; HS_EINVAL if the index has no low-precision copy
 * or a query is beyond the fp16 range of an HS_SHADOW_FP16 copy.
 */
hs_status hs_knn_mixed(hs_index* idx, const float* q_dev, int32_t Q, int32_t k, void* ws_dev, int64_t ws_bytes,
                       int64_t* ids_dev, float* d2_dev, double* err_dev, void* stats_dev, void* stream);

/*
 * Serving form (beside the paper's method, which answers one query batch at a
 * time; the paper's interactive workload is a stream of queries arriving
 * asynchronously, Sec. 4.1).  A server holds C indexes ("collections",
 * possibly of different series lengths) and answers requests of any k as
 * they arrive, by continuous batching:
 *  - hs_submit copies the query and queues the request if one of max_slots
 *    slots is free (HS_EBUSY otherwise; the caller retries later);
 *  - a dispatcher thread forms a batch from the head of a collection's queue
 *    whenever one of that collection's streams is idle, and launches the
 *    whole query path for the batch as one HIP graph, captured once per
 *    (stream, batch size, k) and replayed; batches of other collections and
 *    on the collection's other streams keep running on the device meanwhile;
 *  - each stream owns an equal, fixed region of the caller's budget buffer
 *    (budget_bytes / (C * streams_per_coll)) for its batch's query state, so
 *    a batch takes at most as many queries as that region holds (the HBM
 *    budget of admission);
 *  - hs_poll hands out completions.  A request's result is its exact top-k
 *    by (d2, id): the same ids and the same float32 distances as when it is
 *    answered alone (hs_knn_exact / hs_knn_mixed), whatever the mix.
 * forms[c]: 0 = plain path (hs_knn_exact), 1 = precision form (hs_knn_mixed;
 * the collection must have a low-precision copy).  forms may be NULL (all 0).
 * The indexes and the budget buffer must outlive the server.  hs_submit and
 * hs_poll may be called from any thread; the server's own thread makes all
 * HIP calls on the device that was current at hs_server_create.
 */
typedef struct hs_server hs_server;

typedef struct {
    int32_t streams_per_coll; /* streams, and budget regions, per collection (1..8) */
    int32_t max_slots;        /* requests in the server at once (queued + running), >= 1 */
    int32_t max_batch;        /* largest batch, a power of two in [1, 1024] */
    int32_t reserved;         /* 0 */
} hs_server_config;

typedef struct {
    uint64_t tag;            /* the caller's tag */
    int32_t coll;            /* collection */
    int32_t k;               /* neighbours requested */
    hs_status status;        /* HS_OK, HS_ECANCEL (withdrawn), or the error that failed its batch */
    int32_t batch;           /* requests in the batch it ran in */
    double t_submit;         /* seconds on hs_server_now's clock: hs_submit accepted it */
    double t_launch;         /* its batch was launched */
    double t_done;           /* its batch was seen complete */
    int64_t ids[HS_KMAX];    /* first k entries: original row ids, by (d2, id) ascending */
    float d2[HS_KMAX];       /* squared distances (float32; compensated in the precision form) */
    double err[HS_KMAX];     /* a-priori bound of |d2 - d| (as hs_knn_exact's err_dev) */
} hs_completion;

typedef struct {
    int64_t in_system;       /* requests queued or running */
    int64_t batches;         /* batches launched */
    int64_t queries;         /* requests launched */
    int64_t padded_queries;  /* query rows launched (batches run at power-of-two sizes) */
    int64_t graphs;          /* graphs captured */
    int64_t failed;          /* 1 after a device failure (hs_submit then returns HS_EHIP) */
} hs_server_stats;

/* Errors: HS_EINVAL (NULL, C < 1, bad config or form, precision form
 * without a copy), HS_ENOMEM (a region cannot hold one query of some
 * collection, or host memory), HS_EHIP. */
hs_status hs_server_create(hs_index* const* colls, const int32_t* forms, int32_t C, void* budget_dev,
                           int64_t budget_bytes, const hs_server_config* cfg, hs_server** out);
/* q_host: float32 [n] of the collection (copied before return).
 * Errors: HS_EINVAL (collection, k out of [1, min(N, HS_KMAX)], NaN/Inf, or a
 * value beyond the fp16 range for an fp16 precision-form collection),
 * HS_EBUSY (no free slot), HS_EHIP (the server failed earlier). */
hs_status hs_submit(hs_server* srv, int32_t coll, const float* q_host, int32_t k, uint64_t tag);
/* Withdraw a queued request (the oldest one with this tag): its slot is free
 * at once and hs_poll hands out its completion with status HS_ECANCEL (and no
 * results), so every accepted request still completes exactly once.
 * Errors: HS_EBUSY (its batch is already on the device: it completes
 * normally), HS_EINVAL (no request with that tag is queued). */
hs_status hs_cancel(hs_server* srv, uint64_t tag);
/* Up to max completions, oldest first; *got of them written. */
hs_status hs_poll(hs_server* srv, hs_completion* out, int32_t max, int32_t* got);
hs_status hs_server_info(hs_server* srv, hs_server_stats* out);
/* Waits for running batches, drops queued requests, releases the server. */
hs_status hs_server_destroy(hs_server* srv);
/* Seconds on the server's monotonic clock. */
double hs_server_now(void);

/*
 * The server's admission scheduler on its own (host logic, no device calls),
 * for callers that drive their own loop and for testing.  max_q: int32
 * [C][8], the largest batch (0 or a power of two) a stream region of
 * collection c holds when the batch's k falls in bucket b (k <= 2^b).
 * hs_sched_next forms the next batch of (coll, stream) if that stream is idle:
 * FIFO order, as many requests as fit at the batch's k bucket; *count = 0 if
 * none.  tags must hold max_tags >= the largest max_q entry.  The stream stays
 * busy until hs_sched_complete.  hs_sched_submit: HS_EBUSY when max_slots
 * requests are in the system, HS_EINVAL for a k no region holds.
 * hs_sched_cancel withdraws the oldest queued request with the tag (HS_EINVAL
 * if none is queued; a request in a formed batch is not).
 */
typedef struct hs_sched hs_sched;
hs_status hs_sched_create(int32_t C, int32_t streams, int32_t max_slots, const int32_t* max_q, hs_sched** out);
hs_status hs_sched_submit(hs_sched* s, int32_t coll, int32_t k, uint64_t tag);
hs_status hs_sched_next(hs_sched* s, int32_t coll, int32_t stream, int32_t* q_pad, int32_t* k_batch, uint64_t* tags,
                        int32_t max_tags, int32_t* count);
hs_status hs_sched_cancel(hs_sched* s, uint64_t tag);
hs_status hs_sched_complete(hs_sched* s, int32_t coll, int32_t stream);
hs_status hs_sched_in_system(hs_sched* s, int32_t* n);
hs_status hs_sched_destroy(hs_sched* s);

/* Diagnostics.  While enabled, hs_knn_exact and hs_knn_mixed bracket every
 * launch of their scan kernels (the dominant ones) with HIP events on their
 * stream and, after their own final synchronisation, add the elapsed times
 * to process-wide accumulators, one per kind.  Not meant for concurrent
 * calls from several threads. */
#define HS_PROF_FILTER 0 /* LB_SAX filter (Sec. 3.4 step 3) */
#define HS_PROF_REFINE 1 /* refinement of the candidates (step 4) */
#define HS_PROF_FUSED 2  /* fused filter + refinement (overflow fallback) */
#define HS_PROF_BOUND 3  /* matrix-core bounding pass of the precision form */
#define HS_PROF_KINDS 4
hs_status hs_profile_enable(int32_t on);
/* Accumulated milliseconds and launch count of one kind; cleared if reset.
 * Errors: HS_EINVAL for an unknown kind. */
hs_status hs_profile_read(int32_t kind, double* ms, int64_t* launches, int32_t reset);

/* Diagnostics: batch-union counters.  Sec. 4.1 measures the fraction of the
 * data a query accesses; for a batch of queries the units that count are the
 * distinct ones, since a unit read once can serve every query of the batch.
 * While enabled with a caller-owned device bit array (zeroed by the caller,
 * at least hs_union_bytes bytes), hs_knn_exact and hs_knn_mixed mark every
 * distinct unit their filter and refine kernels read (in diagnostic variants
 * of those kernels; the timed ones are not changed; the seed step's reads are
 * not marked):
 *   region 0: (stored series, 64-point chunk) pairs of raw values,
 *   region 1: stored series whose iSAX word was read,
 *   region 2: 64-series chunk envelopes tested.
 * hs_union_count adds the marked units of each region to counts_dev[0..2]
 * (uint64, caller-zeroed), asynchronously on the stream.  Process-wide; not
 * meant for concurrent calls.  hs_union_enable(NULL, 0) turns it off.
 * Errors: HS_EINVAL (NULL, a size that is not a positive multiple of 4);
 * hs_knn_* return HS_ENOMEM while enabled with an array too small for their
 * index. */
hs_status hs_union_bytes(const hs_index* idx, int64_t* bytes);
hs_status hs_union_enable(void* bits_dev, int64_t bytes);
hs_status hs_union_count(const hs_index* idx, const void* bits_dev, uint64_t* counts_dev, void* stream);

/* Diagnostics: the device's achievable read-stream rate, reported beside
 * the nominal HBM peak.  Reads the first `bytes` of device memory buf_dev
 * (a multiple of 16, at least 1 MiB; contents do not matter, only read)
 * once to warm up and then `passes` times, each pass a grid of 8 workgroups
 * per compute unit reading 16-byte units; *ms = event-timed milliseconds of
 * the timed passes.  sink_dev: 4 caller-owned device bytes that the probe may
 * write (it practically never does).  Synchronises the stream.
 * Errors: HS_EINVAL (NULL, bytes or passes out of range), HS_EHIP. */
hs_status hs_read_probe(const void* buf_dev, int64_t bytes, int32_t passes, uint32_t* sink_dev, void* stream,
                        double* ms);

/* Diagnostics: the device's achievable rate of 4-byte LDS table lookups,
 * reported beside the nominal LDS peak for the LB_SAX filter.  Each compute
 * unit runs 4 workgroups of 256 threads; each thread makes `rounds` rounds of
 * 16 lookups into a 16 x 256 float table in LDS, one per row, at the
 * same per-thread symbols every round.  pattern 0: row r at symbol
 * (lane + 7 r) mod 64, so a wavefront's lanes read 64 consecutive words of
 * the row (no bank conflicts); pattern 1: pseudo-random symbols (a hash of
 * thread and row), as the words of unrelated series give.  One warm-up
 * launch, then `passes` timed ones;
 * *lookups_per_s = lookups of the timed launches / their event-timed
 * seconds.  sink_dev: 4 caller-owned device bytes the probe may write (it
 * practically never does).  Synchronises the stream.
 * Errors: HS_EINVAL (NULL, pattern not 0 or 1, rounds outside 1..2^20,
 * passes < 1), HS_EHIP. */
hs_status hs_lds_probe(int32_t pattern, int32_t rounds, int32_t passes, uint32_t* sink_dev, void* stream,
                       double* lookups_per_s);

/* Release the host handle (does not free index_mem_dev). NULL is allowed. */
hs_status hs_index_free(hs_index* idx);

/* Message of the last failure on this thread ("" if none). */
const char* hs_last_error(void);

/* Breakpoints used by the library: beta_1..beta_{card-1} as float32
 * (Phi^-1(j/card), equiprobable N(0,1) regions), written to out[card-1]. */
hs_status hs_breakpoints(int32_t card_bits, float* out);

#ifdef __cplusplus
}
#endif

#endif /* HS_H */
