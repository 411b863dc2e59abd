// Host side of the C ABI declared in include/hs.h: argument checking, device
// memory layout, the leaf partition (host C++), and the query driver that
// enqueues the kernels of hs_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <future>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "hs_host.h"

using namespace hs;

namespace {

thread_local std::string g_err;

std::mutex g_prof_mu;
bool g_prof_on = false;
uint32_t* g_union_bits = nullptr;  // batch-union diagnostics (guarded by g_prof_mu)
int64_t g_union_bytes = 0;
double g_prof_ms[HS_PROF_KINDS] = {};
int64_t g_prof_launches[HS_PROF_KINDS] = {};

}  // namespace

namespace hs {

// Events around the scan-kernel launches while profiling is on.
struct ScanTimer {
    struct Rec {
        hipEvent_t a, b;
        int kind;
    };
    std::vector<Rec> ev;
    bool on = false;
    ScanTimer() {
        std::lock_guard<std::mutex> g(g_prof_mu);
        on = g_prof_on;
    }
    hipError_t begin(hipStream_t st, int kind) {
        if (!on) return hipSuccess;
        Rec r{nullptr, nullptr, kind};
        hipError_t e = hipEventCreate(&r.a);
        if (e != hipSuccess) return e;
        e = hipEventCreate(&r.b);
        if (e != hipSuccess) {
            (void)hipEventDestroy(r.a);
            return e;
        }
        ev.push_back(r);
        return hipEventRecord(r.a, st);
    }
    hipError_t end(hipStream_t st) { return on ? hipEventRecord(ev.back().b, st) : hipSuccess; }
    // after the stream has been synchronised
    void collect() {
        if (!on) return;
        std::lock_guard<std::mutex> g(g_prof_mu);
        for (auto& r : ev) {
            float t = 0.0f;
            if (hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
                g_prof_ms[r.kind] += t;
                g_prof_launches[r.kind] += 1;
            }
        }
    }
    ~ScanTimer() {
        for (auto& r : ev) {
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
    }
};

hs_status fail(hs_status code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int64_t align_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

int32_t row_stride(int32_t n) { return (int32_t)align_up(n, kChunk); }
int32_t word_stride(int32_t w) { return (int32_t)align_up(w, 16); }

hs_status check_params(const hs_params* p) {
    if (!p) return fail(HS_EINVAL, "params is NULL");
    if (p->n < 1 || p->n > 16384) return fail(HS_EINVAL, "n=%d out of range [1, 16384]", p->n);
    if (p->w < 1 || p->w > 64) return fail(HS_EINVAL, "w=%d out of range [1, 64]", p->w);
    if (p->n % p->w) return fail(HS_EINVAL, "w=%d does not divide n=%d", p->w, p->n);
    if (p->card_bits != 8) return fail(HS_EINVAL, "card_bits=%d: only 8 (alphabet 256) is supported", p->card_bits);
    if (p->leaf_size < 1) return fail(HS_EINVAL, "leaf_size=%d must be >= 1", p->leaf_size);
    if (p->l_max < 0) return fail(HS_EINVAL, "l_max=%d must be >= 0", p->l_max);
    if (p->seed_rows < 0) return fail(HS_EINVAL, "seed_rows=%d must be >= 0", p->seed_rows);
    if (!(p->eapca_th >= 0.0f) || !std::isfinite(p->eapca_th)) return fail(HS_EINVAL, "eapca_th must be finite, >= 0");
    if (p->cand_per_query < 0) return fail(HS_EINVAL, "cand_per_query=%d must be >= 0", p->cand_per_query);
    if (p->build_flags & ~HS_BUILD_HOST_PARTITION) return fail(HS_EINVAL, "unknown build_flags 0x%x", p->build_flags);
    if (p->reserved != 0) return fail(HS_EINVAL, "reserved must be 0");
    return HS_OK;
}

// Gaussian breakpoints beta_j = Phi^-1(j / 256), j = 1..255, by bisection on
// Phi(x) = erfc(-x / sqrt 2) / 2 in double precision, rounded to float32.
void compute_breakpoints(float* out255) {
    for (int j = 1; j < kCard; ++j) {
        const double target = (double)j / kCard;
        double lo = -40.0, hi = 40.0;
        for (int it = 0; it < 200; ++it) {
            const double mid = 0.5 * (lo + hi);
            const double phi = 0.5 * std::erfc(-mid / std::sqrt(2.0));
            if (phi < target) lo = mid; else hi = mid;
        }
        out255[j - 1] = (float)(0.5 * (lo + hi));
    }
    out255[kCard / 2 - 1] = 0.0f;  // Phi^-1(1/2) = 0 exactly
}

// ------------------------------------------------------------ leaf builder
//
// Top-down partition by H-splits (Hercules Sec. 3.2): a node with more than
// tau series is split on one segment's mean or std at the midpoint of that
// statistic's [min, max] range over the node; values below the midpoint go
// left.  Policy (the paper defers to DSTree's heuristic without stating it):
// the candidate with the largest segment_length * range^2, lowest segment
// first and mean before std on ties, that leaves both children non-empty.
// The partition is stable, so leaves hold ids in ascending order and the
// final array order is the in-order leaf order.

struct Partition {
    int w = 0;
    int64_t tau = 0;
    float2* st = nullptr;    // [N][w] (mean, std) in current order
    uint32_t* id = nullptr;  // [N] original id in current order
    std::vector<float2> tmp_st;
    std::vector<uint32_t> tmp_id;
    std::mutex mu;
    std::vector<std::pair<int64_t, int64_t>> leaves;

    void add_leaf(int64_t b, int64_t e) {
        std::lock_guard<std::mutex> g(mu);
        leaves.emplace_back(b, e);
    }

    // Below the leaf level the same splits continue down to kChunkRows series
    // (in_leaf): they only order the series inside their leaf, so that the
    // leaf's fixed 64-series chunks hold similar series and get tight chunk
    // envelopes.  Leaves are the nodes that first hold at most tau series.
    void run(int64_t b, int64_t e, int depth, bool in_leaf) {
        while (true) {
            const int64_t cnt = e - b;
            if (!in_leaf && cnt <= tau) {
                add_leaf(b, e);
                in_leaf = true;
            }
            if (in_leaf && cnt <= kChunkRows) return;
            std::vector<float> mn(2 * w, INFINITY), mx(2 * w, -INFINITY);
            for (int64_t r = b; r < e; ++r) {
                const float2* s = st + r * w;
                for (int i = 0; i < w; ++i) {
                    mn[2 * i] = std::min(mn[2 * i], s[i].x);
                    mx[2 * i] = std::max(mx[2 * i], s[i].x);
                    mn[2 * i + 1] = std::min(mn[2 * i + 1], s[i].y);
                    mx[2 * i + 1] = std::max(mx[2 * i + 1], s[i].y);
                }
            }
            // candidates ordered by score desc, then segment, then mean before std
            std::vector<int> order(2 * w);
            for (int c = 0; c < 2 * w; ++c) order[c] = c;
            std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
                const double ra = (double)mx[a] - mn[a], rc = (double)mx[c] - mn[c];
                return ra * ra > rc * rc;  // equal segment lengths: score ~ range^2
            });
            int64_t nl = -1;
            double thr = 0.0;
            int cand = -1;
            for (int c : order) {
                if (!(mx[c] > mn[c])) break;
                thr = ((double)mn[c] + (double)mx[c]) / 2.0;
                int64_t left = 0;
                for (int64_t r = b; r < e; ++r) {
                    const float2 v = st[r * w + c / 2];
                    left += (double)((c & 1) ? v.y : v.x) < thr;
                }
                if (left > 0 && left < cnt) {
                    nl = left;
                    cand = c;
                    break;
                }
            }
            if (cand < 0) {
                if (!in_leaf) add_leaf(b, e);
                return;
            }
            // stable partition through the scratch arrays
            int64_t li = b, ri = b + nl;
            for (int64_t r = b; r < e; ++r) {
                const float2 v = st[r * w + cand / 2];
                const bool goes_left = (double)((cand & 1) ? v.y : v.x) < thr;
                const int64_t dst = goes_left ? li++ : ri++;
                std::memcpy(&tmp_st[dst * w], &st[r * w], sizeof(float2) * w);
                tmp_id[dst] = id[r];
            }
            std::memcpy(&st[b * w], &tmp_st[b * w], sizeof(float2) * w * cnt);
            std::memcpy(&id[b], &tmp_id[b], sizeof(uint32_t) * cnt);
            const int64_t mid = b + nl;
            if (depth < 6 && cnt > (1 << 20)) {
                auto fut = std::async(std::launch::async,
                                      [this, b, mid, depth, in_leaf] { run(b, mid, depth + 1, in_leaf); });
                run(mid, e, depth + 1, in_leaf);
                fut.get();
                return;
            }
            run(b, mid, depth + 1, in_leaf);
            b = mid;  // tail iteration on the right child
            ++depth;
        }
    }
};

void carve(char*& cur, void** out, int64_t bytes) {
    *out = cur;
    cur += align_up(bytes, 256);
}

// Leaves the index's tables are sized for: far above what a midpoint
// partition makes (about 2 N / tau on random walks), and N for tiny leaves.
int64_t leaf_budget(int64_t N, int64_t tau) {
    return std::min<int64_t>(N, 4 * ((N + tau - 1) / tau) + 1024);
}

float bits_to_float_host(uint32_t b) {
    float f;
    std::memcpy(&f, &b, sizeof f);
    return f;
}

// Width h of the deviation codes: the largest segment std, widened by 2^-20
// (the float32 statistics lie within an ulp of the FP64 ones), over 256
// codes, rounded up to 16 significant bits so that c h and (c + 1) h are
// exact in float32 for every code c.  All stds zero: h = 1.
float sigma_step(float smax) {
    const double hh = (double)smax * (1.0 + std::ldexp(1.0, -20)) / 256.0;
    if (!(hh > 0.0) || !std::isfinite(hh)) return 1.0f;
    int e = 0;
    const double m = std::frexp(hh, &e);  // hh = m 2^e, m in [0.5, 1)
    return (float)std::ldexp(std::ceil(m * 65536.0) / 65536.0, e);
}

// Byte offsets inside the caller's index memory (base may be NULL: sizes only).
IndexLayout index_layout(int64_t N, const hs_params& p, char* base) {
    (void)base;
    IndexLayout l{};
    const int64_t stride = row_stride(p.n), wstride = word_stride(p.w);
    l.leaf_budget = leaf_budget(N, p.leaf_size);
    l.chunk_cap = (N + kChunkRows - 1) / kChunkRows + l.leaf_budget;  // each leaf cut from its first series
    int64_t cur = 0;
    auto take = [&](int64_t bytes) {
        const int64_t at = cur;
        cur += align_up(bytes, 256);
        return at;
    };
    const int64_t rows_bytes = N * stride * 4;
    l.rows = take(rows_bytes);
    l.ids = take(N * 4);
    l.words = take(N * wstride);
    l.sig = take(N * wstride);
    l.flag = take(256);
    l.beta = take((kCard + 1) * 4);
    l.leaf_start = take((l.leaf_budget + 1) * 8);
    l.env = take(l.leaf_budget * p.w * 16);
    l.part_start = take((l.chunk_cap + 1) * 8);
    l.part_leaf = take(l.chunk_cap * 4);
    l.part_chunk = take(l.chunk_cap * 8);
    l.chunk_start = take((l.chunk_cap + 1) * 8);
    l.cenv = take(l.chunk_cap * p.w * 16);
    // build scratch: the device partition's buffers (the host partition needs
    // only the statistics at their start), inside the rows' area when they fit
    const int64_t scratch = partition_scratch_bytes(N, p.w, p.leaf_size, l.leaf_budget);
    l.scratch = scratch <= rows_bytes ? l.rows : take(scratch);
    l.total = cur;
    return l;
}

int64_t ws_layout(const hs_index* idx, int32_t Q, int32_t k, QueryWs* ws, char* base, int64_t cand_fixed) {
    const IndexView& ix = idx->view;
    const int P = kPoolMin;
    const int64_t items = (int64_t)Q * ix.parts + 1;
    // candidate list: up to 1/8 of the collection per query on average,
    // between 64 Ki and 2 Gi entries (24 GB with the slices' 12 bytes each; the
    // 32-bit slice prefix stays below 2^32); a query whose candidates do not
    // fit is answered by the fused scan instead (no result changes)
    const int64_t cpq = cand_fixed > 0 ? 1 : idx->p.cand_per_query;
    const int64_t per_q = cpq > 0 ? cpq : std::max<int64_t>((ix.N + 7) / 8, 4096);
    const int64_t floor_c = cpq > 0 ? 1 : (1 << 16);
    const int64_t cand_total =
        cand_fixed > 0 ? std::min<int64_t>(cand_fixed, (int64_t)1 << 31)
                       : std::min<int64_t>(std::max<int64_t>((int64_t)Q * per_q, floor_c), (int64_t)1 << 31);
    // 3/4 in the filter wavefronts' private slices, 1/4 in a shared overflow slice
    // a partial low-precision copy: the bounding pass and the LB_SAX filter
    // each fill their own half of the slices
    const bool hybrid = idx->shadow.kind != 0 && idx->shadow.rows_n < ix.N;
    const int n_slices = idx->filter_waves * (hybrid ? 2 : 1);
    const int64_t slice_cap = (cand_total * 3 / 4 + n_slices - 1) / n_slices;
    const int64_t ovf_cap = std::max<int64_t>(cand_total / 4, cpq > 0 ? 1 : 4096);
    const int64_t cand = slice_cap * n_slices + ovf_cap;
    char* cur = base;
    QueryWs w{};
    carve(cur, (void**)&w.qrow, (int64_t)Q * ix.stride * 4);
    carve(cur, (void**)&w.qstat, (int64_t)Q * ix.w * 16);
    carve(cur, (void**)&w.qst32, (int64_t)Q * ix.w * 16);
    carve(cur, (void**)&w.lut, (int64_t)Q * ix.w * kCard * 4);
    carve(cur, (void**)&w.lbe, (int64_t)Q * ix.L * 4);
    carve(cur, (void**)&w.bkey, (int64_t)Q * 8);
    carve(cur, (void**)&w.pool_cnt, (int64_t)Q * 4);
    carve(cur, (void**)&w.flags, (int64_t)Q * 4);
    carve(cur, (void**)&w.kept, (int64_t)Q * 4);
    carve(cur, (void**)&w.pool, (int64_t)Q * P * 8);
    carve(cur, (void**)&w.stats, (int64_t)Q * kStatSlots * 8);
    carve(cur, (void**)&w.items, items * 8);
    carve(cur, (void**)&w.slice_pos, cand * 4);
    carve(cur, (void**)&w.slice_q, cand * 4);
    carve(cur, (void**)&w.slice_part, cand * 4);
    carve(cur, (void**)&w.slice_cnt, ((int64_t)n_slices + 1) * 4);
    carve(cur, (void**)&w.slice_start, ((int64_t)n_slices + 2) * 4);
    carve(cur, (void**)&w.counters, kNumCounters * 4);
    const int32_t Qpad = (Q + kBoundQueries - 1) / kBoundQueries * kBoundQueries;
    carve(cur, (void**)&w.qlow, (int64_t)Qpad * ix.stride * 2);
    carve(cur, (void**)&w.qnorm, (int64_t)Q * 16);
    carve(cur, (void**)&w.plist, (int64_t)Q * ix.parts * 4);
    carve(cur, (void**)&w.pcnt, (ix.parts + 1) * 4);
    carve(cur, (void**)&w.pnb, (ix.parts + 1) * 4);
    carve(cur, (void**)&w.pbo, (ix.parts + 2) * 4);
    carve(cur, (void**)&w.pscan, ((ix.parts + 1) / 1024 + 2) * 4);
    w.Qpad = Qpad;
    w.item_cap = items;
    w.slice_cap = slice_cap;
    w.ovf_cap = ovf_cap;
    w.n_slices = n_slices;
    w.P = P;
    if (ws) *ws = w;
    return (int64_t)(cur - base);
}

}  // namespace

extern "C" {

const char* hs_last_error(void) { return g_err.c_str(); }

hs_status hs_breakpoints(int32_t card_bits, float* out) {
    if (card_bits != 8) return fail(HS_EINVAL, "card_bits must be 8");
    if (!out) return fail(HS_EINVAL, "out is NULL");
    compute_breakpoints(out);
    return HS_OK;
}

hs_status hs_index_bytes(int64_t N, const hs_params* params, int64_t* bytes) {
    hs_status s = check_params(params);
    if (s) return s;
    if (!bytes) return fail(HS_EINVAL, "bytes is NULL");
    if (N < 1 || N >= (int64_t)1 << 32) return fail(HS_EINVAL, "N=%lld out of range [1, 2^32)", (long long)N);
    *bytes = index_layout(N, *params, nullptr).total;
    return HS_OK;
}

hs_status hs_build_begin(int64_t N, const hs_params* params, void* index_mem_dev, int64_t index_bytes, void* stream,
                         hs_builder** out) {
    if (!out) return fail(HS_EINVAL, "out is NULL");
    *out = nullptr;
    if (!index_mem_dev) return fail(HS_EINVAL, "index_mem_dev is NULL");
    int64_t need = 0;
    hs_status s = hs_index_bytes(N, params, &need);
    if (s) return s;
    if (index_bytes < need) return fail(HS_ENOMEM, "index_bytes=%lld < required %lld", (long long)index_bytes, (long long)need);
    const hs_params p = *params;
    int device = 0, cus = 0;
    HIP_TRY(hipGetDevice(&device));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));
    hs_builder* b = new (std::nothrow) hs_builder();
    hs_index* idx = new (std::nothrow) hs_index();
    if (!b || !idx) {
        delete b;
        delete idx;
        return fail(HS_ENOMEM, "host allocation failed");
    }
    b->idx = idx;
    b->st = (hipStream_t)stream;
    idx->p = p;
    idx->device = device;
    idx->cus = cus;
    // everything lives in the caller's index memory: the stored arrays, the
    // small tables (sized for at most lay.leaf_budget leaves) and, until the
    // rows arrive, the build's scratch (inside the rows' area when it fits)
    char* base = (char*)index_mem_dev;
    b->lay = index_layout(N, p, base);
    const IndexLayout& lay = b->lay;
    IndexView& ix = idx->view;
    ix.N = N;
    ix.n = p.n;
    ix.w = p.w;
    ix.stride = row_stride(p.n);
    ix.wstride = word_stride(p.w);
    ix.rows = (const float*)(base + lay.rows);
    ix.ids = (const uint32_t*)(base + lay.ids);
    ix.words = (const uint8_t*)(base + lay.words);
    ix.sig = (const uint8_t*)(base + lay.sig);
    ix.sig_h = 1.0f;
    idx->index_bytes = need;
    idx->beta_dev = (float*)(base + lay.beta);
    idx->leaf_start_dev = (int64_t*)(base + lay.leaf_start);
    idx->env_dev = (float4*)(base + lay.env);
    idx->part_start_dev = (int64_t*)(base + lay.part_start);
    idx->part_leaf_dev = (uint32_t*)(base + lay.part_leaf);
    idx->part_chunk_dev = (int64_t*)(base + lay.part_chunk);
    idx->chunk_start_dev = (int64_t*)(base + lay.chunk_start);
    idx->cenv_dev = (float4*)(base + lay.cenv);
    b->scratch = base + lay.scratch;
    b->bad = (uint32_t*)(base + lay.flag);
    b->st_dev = partition_stats_buffer(b->scratch, N, p.w, p.leaf_size, lay.leaf_budget);
    // until the rows arrive, the words' area holds each series' stored position
    b->pos = (uint32_t*)ix.words;
    // flag area: [0] NaN / Inf seen, [1] largest segment std (float bits)
    const hipError_t e = hipMemsetAsync(b->bad, 0, 2 * sizeof(uint32_t), b->st);
    if (e != hipSuccess) {
        delete idx;
        delete b;
        return fail(HS_EHIP, "hipMemsetAsync: %s", hipGetErrorString(e));
    }
    *out = b;
    return HS_OK;
}

hs_status hs_build_add_stats(hs_builder* b, const float* x_dev, int64_t row0, int64_t rows) {
    if (!b || !x_dev) return fail(HS_EINVAL, "NULL argument");
    if (b->stage != 0) return fail(HS_EINVAL, "statistics come before hs_build_partition");
    const IndexView& ix = b->idx->view;
    if (row0 != b->next_row || rows < 1 || row0 + rows > ix.N)
        return fail(HS_EINVAL, "rows [%lld, %lld): chunks must cover [0, N) in order (next row %lld)", (long long)row0,
                    (long long)(row0 + rows), (long long)b->next_row);
    HIP_TRY(launch_series_stats(x_dev, rows, ix.n, ix.w, b->st_dev + row0 * ix.w, b->bad, b->st));
    b->next_row = row0 + rows;
    return HS_OK;
}

hs_status hs_build_partition(hs_builder* b) {
    if (!b) return fail(HS_EINVAL, "NULL argument");
    hs_index* idx = b->idx;
    IndexView& ix = idx->view;
    const hs_params& p = idx->p;
    const IndexLayout& lay = b->lay;
    const int64_t N = ix.N;
    hipStream_t st = b->st;
    if (b->stage != 0 || b->next_row != N) return fail(HS_EINVAL, "the statistics of all N rows come first");
    // the deviation codes' width, from the largest segment std (the
    // statistics are overwritten by the rows later)
    HIP_TRY(launch_max_sigma(b->st_dev, N * p.w, b->bad + 1, st));
    uint32_t flags[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(flags, b->bad, sizeof flags, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (flags[0]) return fail(HS_EINVAL, "x contains NaN or Inf");
    ix.sig_h = sigma_step(bits_to_float_host(flags[1]));

    // leaf partition: on the device, or on the host (the reference the
    // device partition is tested against)
    std::vector<int64_t> leaf_start;
    if (p.build_flags & HS_BUILD_HOST_PARTITION) {
        Partition part;
        part.w = p.w;
        part.tau = p.leaf_size;
        std::vector<float2> st_host;
        std::vector<uint32_t> id_host;
        try {
            st_host.resize((size_t)N * p.w);
            id_host.resize((size_t)N);
            part.tmp_st.resize((size_t)N * p.w);
            part.tmp_id.resize((size_t)N);
        } catch (...) {
            return fail(HS_ENOMEM, "host allocation for the leaf partition failed");
        }
        HIP_TRY(hipMemcpyAsync(st_host.data(), b->st_dev, sizeof(float2) * N * p.w, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        for (int64_t i = 0; i < N; ++i) id_host[i] = (uint32_t)i;
        part.st = st_host.data();
        part.id = id_host.data();
        part.run(0, N, 0, false);
        std::sort(part.leaves.begin(), part.leaves.end());
        for (auto& lf : part.leaves) leaf_start.push_back(lf.first);
        if ((int64_t)leaf_start.size() > lay.leaf_budget)
            return fail(HS_ENOMEM, "the host partition made %lld leaves; the index memory holds tables for %lld",
                        (long long)leaf_start.size(), (long long)lay.leaf_budget);
        HIP_TRY(hipMemcpyAsync((void*)ix.ids, id_host.data(), sizeof(uint32_t) * N, hipMemcpyHostToDevice, st));
        HIP_TRY(hipStreamSynchronize(st));
    } else {
        hs_status s = partition_device(N, p.w, p.leaf_size, lay.leaf_budget, b->scratch, idx->cus, (uint32_t*)ix.ids,
                                       &leaf_start, st);
        if (s) return s;
    }
    const int64_t L = (int64_t)leaf_start.size();
    leaf_start.push_back(N);
    int64_t max_leaf = 0;
    for (int64_t i = 0; i < L; ++i) max_leaf = std::max(max_leaf, leaf_start[i + 1] - leaf_start[i]);
    ix.L = L;
    idx->max_leaf = max_leaf;
    // work items: every leaf cut into parts of at most kPartRows series;
    // chunks: every leaf cut into kChunkRows-series chunks (parts start on a
    // chunk boundary, so a part's chunks are consecutive)
    std::vector<int64_t> part_start, chunk_start;
    std::vector<uint32_t> part_leaf;
    std::vector<int64_t> part_chunk;
    for (int64_t i = 0; i < L; ++i) {
        for (int64_t r = leaf_start[i]; r < leaf_start[i + 1]; r += kChunkRows) {
            if ((r - leaf_start[i]) % kPartRows == 0) {
                part_start.push_back(r);
                part_leaf.push_back((uint32_t)i);
                part_chunk.push_back((int64_t)chunk_start.size());
            }
            chunk_start.push_back(r);
        }
    }
    const int64_t parts = (int64_t)part_leaf.size();
    const int64_t chunks = (int64_t)chunk_start.size();
    part_start.push_back(N);
    chunk_start.push_back(N);
    if (chunks > lay.chunk_cap || parts > lay.chunk_cap)
        return fail(HS_EHIP, "table sizes exceed their reservation (%lld chunks)", (long long)chunks);
    idx->part_start_host = part_start;
    ix.parts = parts;
    ix.chunks = chunks;
    idx->filter_waves = filter_waves(ix, idx->cus);

    float beta_host[kCard + 1];
    beta_host[0] = -INFINITY;
    compute_breakpoints(beta_host + 1);
    beta_host[kCard] = INFINITY;
    HIP_TRY(hipMemcpyAsync(idx->part_chunk_dev, part_chunk.data(), sizeof(int64_t) * parts, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(idx->chunk_start_dev, chunk_start.data(), sizeof(int64_t) * (chunks + 1),
                           hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(idx->leaf_start_dev, leaf_start.data(), sizeof(int64_t) * (L + 1), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(idx->part_start_dev, part_start.data(), sizeof(int64_t) * (parts + 1),
                           hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(idx->part_leaf_dev, part_leaf.data(), sizeof(uint32_t) * parts, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(idx->beta_dev, beta_host, sizeof(beta_host), hipMemcpyHostToDevice, st));
    ix.leaf_start = idx->leaf_start_dev;
    ix.env = idx->env_dev;
    ix.beta = idx->beta_dev;
    ix.part_start = idx->part_start_dev;
    ix.part_leaf = idx->part_leaf_dev;
    ix.part_chunk = idx->part_chunk_dev;
    ix.cenv = idx->cenv_dev;
    // each series' stored position, for the rows of the second pass (the
    // partition's scratch in the rows' area is no longer needed)
    HIP_TRY(launch_inverse_ids(ix.ids, N, b->pos, st));
    HIP_TRY(hipStreamSynchronize(st));
    b->stage = 1;
    b->next_row = 0;
    return HS_OK;
}

hs_status hs_build_add_rows(hs_builder* b, const float* x_dev, int64_t row0, int64_t rows) {
    if (!b || !x_dev) return fail(HS_EINVAL, "NULL argument");
    if (b->stage != 1) return fail(HS_EINVAL, "rows come after hs_build_partition");
    const IndexView& ix = b->idx->view;
    if (row0 != b->next_row || rows < 1 || row0 + rows > ix.N)
        return fail(HS_EINVAL, "rows [%lld, %lld): chunks must cover [0, N) in order (next row %lld)", (long long)row0,
                    (long long)(row0 + rows), (long long)b->next_row);
    HIP_TRY(launch_scatter_rows(x_dev, row0, rows, b->pos, ix.n, ix.stride, (float*)ix.rows, b->st));
    b->next_row = row0 + rows;
    return HS_OK;
}

hs_status hs_build_finish(hs_builder* b, hs_index** out) {
    if (!b || !out) return fail(HS_EINVAL, "NULL argument");
    *out = nullptr;
    hs_index* idx = b->idx;
    const IndexView& ix = idx->view;
    if (b->stage != 1 || b->next_row != ix.N) return fail(HS_EINVAL, "the rows of all N series come first");
    hipStream_t st = b->st;
    HIP_TRY(launch_words(ix, (uint8_t*)ix.words, (uint8_t*)ix.sig, st));
    HIP_TRY(launch_envelopes(ix, idx->leaf_start_dev, ix.L, idx->env_dev, st));
    HIP_TRY(launch_envelopes(ix, idx->chunk_start_dev, ix.chunks, idx->cenv_dev, st));
    HIP_TRY(hipStreamSynchronize(st));
    *out = idx;
    b->idx = nullptr;
    delete b;
    return HS_OK;
}

hs_status hs_build_abort(hs_builder* b) {
    if (!b) return HS_OK;
    if (b->st) (void)hipStreamSynchronize(b->st);
    delete b->idx;
    delete b;
    return HS_OK;
}

hs_status hs_build_summaries(const float* x_dev, int64_t N, const hs_params* params, void* index_mem_dev,
                             int64_t index_bytes, void* stream, hs_index** out) {
    if (!out) return fail(HS_EINVAL, "out is NULL");
    *out = nullptr;
    if (!x_dev || !index_mem_dev) return fail(HS_EINVAL, "x_dev or index_mem_dev is NULL");
    hs_builder* b = nullptr;
    hs_status s = hs_build_begin(N, params, index_mem_dev, index_bytes, stream, &b);
    if (s) return s;
    s = hs_build_add_stats(b, x_dev, 0, N);
    if (!s) s = hs_build_partition(b);
    if (!s) s = hs_build_add_rows(b, x_dev, 0, N);
    if (!s) s = hs_build_finish(b, out);
    if (s) {
        const std::string msg = g_err;
        hs_build_abort(b);
        g_err = msg;
    }
    return s;
}

hs_status hs_get_info(const hs_index* idx, hs_index_info* out) {
    if (!idx || !out) return fail(HS_EINVAL, "NULL argument");
    out->n_series = idx->view.N;
    out->n = idx->view.n;
    out->w = idx->view.w;
    out->row_stride = idx->view.stride;
    out->word_stride = idx->view.wstride;
    out->n_leaves = idx->view.L;
    out->max_leaf = idx->max_leaf;
    out->index_bytes = idx->index_bytes;
    out->n_chunks = idx->view.chunks;
    out->sigma_step = (double)idx->view.sig_h;
    return HS_OK;
}

hs_status hs_get_leaves(const hs_index* idx, int64_t* leaf_start, float* env) {
    if (!idx) return fail(HS_EINVAL, "idx is NULL");
    if (leaf_start)
        HIP_TRY(hipMemcpy(leaf_start, idx->leaf_start_dev, sizeof(int64_t) * (idx->view.L + 1), hipMemcpyDeviceToHost));
    if (env)
        HIP_TRY(hipMemcpy(env, idx->env_dev, sizeof(float4) * idx->view.L * idx->view.w, hipMemcpyDeviceToHost));
    return HS_OK;
}

hs_status hs_get_chunks(const hs_index* idx, int64_t* chunk_start, float* cenv) {
    if (!idx) return fail(HS_EINVAL, "idx is NULL");
    if (chunk_start)
        HIP_TRY(hipMemcpy(chunk_start, idx->chunk_start_dev, sizeof(int64_t) * (idx->view.chunks + 1),
                          hipMemcpyDeviceToHost));
    if (cenv)
        HIP_TRY(hipMemcpy(cenv, idx->cenv_dev, sizeof(float4) * idx->view.chunks * idx->view.w,
                          hipMemcpyDeviceToHost));
    return HS_OK;
}

hs_status hs_query_workspace_bytes(const hs_index* idx, int32_t Q, int32_t k, int64_t* bytes) {
    if (!idx || !bytes) return fail(HS_EINVAL, "NULL argument");
    if (Q < 0) return fail(HS_EINVAL, "Q=%d < 0", Q);
    if (k < 1 || k > HS_KMAX) return fail(HS_EINVAL, "k=%d out of range [1, %d]", k, HS_KMAX);
    *bytes = ws_layout(idx, Q, k, nullptr, nullptr);
    return HS_OK;
}

}  // extern "C"

namespace {

// Relative error bound of a compensated float32 distance over K stored points:
// one rounding of the final sum plus second-order terms of the residues.
double comp_err_rel(int K) { return std::ldexp(1.0, -23) + (4.0 * K + 64.0) * std::ldexp(1.0, -48); }

// Abandoning margin for K stored points (m = K / 64 chunks).  A running
// distance v, plain float32 partials added in any chunk order plus one
// addition of the cascade's bounds, passes through at most m + 10 roundings
// per term (2 for the difference squared, 4 in the lane's fma chain, 4 in the
// butterfly, m - 1 running additions, 1 for the bounds); with two to spare,
// v <= d (1 + g), g = (m + 12) u / (1 - (m + 12) u), u = 2^-24.  The
// compensated running form is tighter.  The result key c satisfies
// c >= d (1 - e_c), and fl(limit * marg) >= limit * marg (1 - u).  So
// v > fl(limit * marg) implies c > limit when
// marg >= (1 + g) / ((1 - u)(1 - e_c)); the float32 value is rounded up.
float abandon_margin(int K) {
    const double u = std::ldexp(1.0, -24);
    const double r = (double)(K / kChunk + 12) * u;
    const double g = r / (1.0 - r);
    const double mg = (1.0 + g) / ((1.0 - u) * (1.0 - comp_err_rel(K)));
    float mf = (float)mg;
    if ((double)mf < mg) mf = std::nextafter(mf, INFINITY);
    return mf;
}

}  // namespace

namespace hs {

// The refine's chunk order needs quarters of the word that cover whole
// quarters of chunks: n = stride = 256 2^e and w a multiple of 16.
static int32_t chunk_order_lg(const IndexView& ix) {
    if (ix.n != ix.stride || ix.w % 16 != 0 || ix.n % 256 != 0) return -1;
    const int cpq = ix.n / 256;
    if (cpq & (cpq - 1)) return -1;
    int lg = 0;
    while ((1 << lg) < cpq) ++lg;
    return lg;
}

hs_status knn_prepare(hs_index* idx, int32_t Q, int32_t k, void* ws_dev, int64_t ws_bytes, bool mixed,
                      KnnCall* c, int64_t cand_total) {
    if (!idx) return fail(HS_EINVAL, "idx is NULL");
    if (Q < 0) return fail(HS_EINVAL, "Q=%d < 0", Q);
    if (k < 1 || k > HS_KMAX) return fail(HS_EINVAL, "k=%d out of range [1, %d]", k, HS_KMAX);
    if ((int64_t)k > idx->view.N) return fail(HS_EINVAL, "k=%d > N=%lld", k, (long long)idx->view.N);
    if (mixed && idx->shadow.kind == 0) return fail(HS_EINVAL, "the index has no low-precision copy (hs_build_shadow)");
    if (Q >= (1 << 24)) return fail(HS_EINVAL, "Q=%d: at most 2^24 - 1 queries per call", Q);
    if ((int64_t)Q * idx->view.parts >= ((int64_t)1 << 31))
        return fail(HS_EINVAL, "Q=%d too large for this index (Q * parts must stay below 2^31); split the batch", Q);
    c->idx = idx;
    c->mixed = mixed;
    c->form = mixed ? kComp : kPlain;
    // both forms key their results by the compensated distance
    c->err_rel = comp_err_rel(idx->view.stride);
    if (Q == 0) return HS_OK;
    if (!ws_dev) return fail(HS_EINVAL, "NULL workspace");
    const int64_t need = ws_layout(idx, Q, k, nullptr, nullptr, cand_total);
    if (ws_bytes < need) return fail(HS_ENOMEM, "ws_bytes=%lld < required %lld", (long long)ws_bytes, (long long)need);
    ws_layout(idx, Q, k, &c->ws, (char*)ws_dev, cand_total);
    {
        std::lock_guard<std::mutex> g(g_prof_mu);
        if (g_union_bits) {
            const int64_t need_bits = union_bits(idx->view);
            if (g_union_bytes * 8 < need_bits)
                return fail(HS_ENOMEM, "batch-union array of %lld bytes < %lld needed for this index",
                            (long long)g_union_bytes, (long long)((need_bits + 31) / 32 * 4));
            c->ws.ubits = g_union_bits;
            c->ws.word_bit0 = idx->view.N * (int64_t)(idx->view.stride / kChunk);
            c->ws.env_bit0 = c->ws.word_bit0 + idx->view.N;
        }
    }
    const IndexView& ix = idx->view;
    c->sp = ScanParams{};
    c->sp.Q = Q;
    c->sp.k = k;
    c->sp.eapca_th = idx->p.eapca_th;
    c->sp.n_seed = (int)std::min<int64_t>(std::min<int64_t>(idx->p.l_max, ix.L), kMaxSeedLeaves);
    c->sp.seed_rows = idx->p.seed_rows;
    c->sp.order_lg = chunk_order_lg(ix);
    c->sp.marg = abandon_margin(ix.stride);
    c->sp.emit_part0 = 0;
    c->sp.slice0 = 0;
    c->sp.slices = c->ws.n_slices;
    return HS_OK;
}

// Steps 1-4 and the first merge, all stream-ordered launches (no host
// synchronisation, no memset), so the sequence can be captured in a graph.
// redo_host (pinned, may be NULL): receives counters[kCtrRedo], [kCtrNonFinite].
hs_status knn_enqueue(const KnnCall& c, const float* q_dev, int64_t* ids_dev, float* d2_dev, double* err_dev,
                      hs_query_stats* stats_out, hipStream_t st, uint32_t* redo_host, ScanTimer* timer) {
    const IndexView& ix = c.idx->view;
    const QueryWs& ws = c.ws;
    ScanParams sp = c.sp;
    auto timed = [&](int kind, auto&& launch) -> hipError_t {
        hipError_t e = timer ? timer->begin(st, kind) : hipSuccess;
        if (e != hipSuccess) return e;
        e = launch();
        if (e != hipSuccess) return e;
        return timer ? timer->end(st) : hipSuccess;
    };
    HIP_TRY(launch_query_prep(ix, q_dev, sp.Q, ws, st));
    if (c.mixed) HIP_TRY(launch_query_low(ix, c.idx->shadow.kind, sp.Q, ws, st));
    HIP_TRY(launch_lb_eapca(ix, sp.Q, ws, st));
    // step 1: approximate search seeds BSF_k
    HIP_TRY(launch_seed(ix, sp, ws, c.form, st));
    // step 2: candidate leaves; step 3: per-series filter (LB_SAX, or the
    // matrix-core bound of the precision form); step 4: refinement
    const ShadowView& sv = c.idx->shadow;
    const bool hybrid = c.mixed && sv.rows_n < ix.N;
    {
        // the precision form makes items only where its copy does not reach
        // (the bounding pass takes the parts of the copy from their lists)
        ScanParams se = sp;
        if (c.mixed) se.emit_part0 = sv.parts_n;
        HIP_TRY(launch_emit(ix, se, false, ws, st));
    }
    if (c.mixed) {
        ScanParams sb = sp;
        if (hybrid) {
            sb.slice0 = ws.n_slices / 2;
            sb.slices = ws.n_slices / 2;
        }
        HIP_TRY(timed(HS_PROF_BOUND, [&] { return launch_bound(ix, sv, sb, ws, c.idx->cus, st); }));
    }
    if (!c.mixed || hybrid) {
        ScanParams sf = sp;
        if (hybrid) sf.slices = ws.n_slices / 2;
        HIP_TRY(timed(HS_PROF_FILTER, [&] { return launch_filter(ix, sf, ws, c.idx->cus, st); }));
    }
    HIP_TRY(launch_slice_prefix(ws, st));
    HIP_TRY(timed(HS_PROF_REFINE, [&] { return launch_refine(ix, sp, ws, c.idx->cus, c.form, st); }));
    sp.final_pass = 1;
    HIP_TRY(launch_merge(ix, sp, false, ws, ids_dev, d2_dev, err_dev, c.err_rel, stats_out, st));
    if (redo_host)
        HIP_TRY(hipMemcpyAsync(redo_host, ws.counters + kCtrRedo, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    return HS_OK;
}

// Queries whose candidate list or result pool overflowed: rescan their
// candidate parts with the tightened BSF_k until nothing overflows (each merge
// keeps the best k so far, without repeats).  While no round has dropped
// candidates (only result pools overflowed), a round takes the main path:
// filter, candidate list and refine over the round's queries' items.  Once
// one has, every later round takes the fused scan, which needs no list.
// Synchronises.
hs_status knn_finish(const KnnCall& c, int64_t* ids_dev, float* d2_dev, double* err_dev, hs_query_stats* stats_out,
                     hipStream_t st, ScanTimer* timer) {
    const IndexView& ix = c.idx->view;
    const QueryWs& ws = c.ws;
    ScanParams sp = c.sp;
    sp.final_pass = 1;
    bool fused = false;
    for (int round = 0;; ++round) {
        uint32_t cnt[2] = {0, 0}, lost = 0;
        HIP_TRY(hipMemcpyAsync(cnt, ws.counters + kCtrRedo, sizeof cnt, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(&lost, ws.counters + kCtrLost, sizeof lost, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if (cnt[1])
            return fail(HS_EINVAL, "%u queries contain NaN or Inf%s", cnt[1],
                        c.mixed && c.idx->shadow.kind == kShadowF16 ? " or values beyond the fp16 range" : "");
        if (cnt[0] == 0) break;
        if (round >= 64) return fail(HS_EHIP, "result pool still overflowing after %d rounds", round);
        if (lost) fused = true;
        HIP_TRY(launch_emit(ix, sp, true, ws, st));
        hipError_t e = timer ? timer->begin(st, HS_PROF_FUSED) : hipSuccess;
        if (fused) {
            if (e == hipSuccess) e = launch_leaf_scan(ix, sp, ws, c.idx->cus, c.form, st);
        } else {
            // every slice takes part (the LB_SAX filter over all of the round's items)
            if (e == hipSuccess) e = launch_filter(ix, sp, ws, c.idx->cus, st);
            if (e == hipSuccess) e = launch_slice_prefix(ws, st);
            if (e == hipSuccess) e = launch_refine(ix, sp, ws, c.idx->cus, c.form, st);
        }
        if (e == hipSuccess && timer) e = timer->end(st);
        HIP_TRY(e);
        HIP_TRY(launch_merge(ix, sp, true, ws, ids_dev, d2_dev, err_dev, c.err_rel, stats_out, st));
    }
    if (timer) timer->collect();
    return HS_OK;
}

}  // namespace hs

namespace {

// The query driver shared by the plain and the precision form.
hs_status run_knn(hs_index* idx, const float* q_dev, int32_t Q, int32_t k, void* ws_dev, int64_t ws_bytes,
                  int64_t* ids_dev, float* d2_dev, double* err_dev, void* stats_dev, void* stream, bool mixed) {
    KnnCall c;
    hs_status s = knn_prepare(idx, Q, k, ws_dev, ws_bytes, mixed, &c);
    if (s || Q == 0) return s;
    if (!q_dev || !ids_dev || !d2_dev) return fail(HS_EINVAL, "NULL device pointer");
    hipStream_t st = (hipStream_t)stream;
    auto* stats_out = (hs_query_stats*)stats_dev;
    ScanTimer timer;
    s = knn_enqueue(c, q_dev, ids_dev, d2_dev, err_dev, stats_out, st, nullptr, &timer);
    if (s) return s;
    return knn_finish(c, ids_dev, d2_dev, err_dev, stats_out, st, &timer);
}

// The copy of the first R stored series is followed by kBoundRows zero rows
// (and zero norms), so the bounding pass may stage a whole tile past its last
// series.
int64_t shadow_layout(const IndexView& ix, int64_t R, uint16_t** rows, float4** norms, uint32_t** flag, char* base) {
    char* cur = base;
    void* a;
    carve(cur, &a, (R + kBoundRows) * ix.stride * 2);
    if (rows) *rows = (uint16_t*)a;
    carve(cur, &a, (R + kBoundRows) * 16);
    if (norms) *norms = (float4*)a;
    carve(cur, &a, 256);
    if (flag) *flag = (uint32_t*)a;
    return (int64_t)(cur - base);
}

// Series and parts a copy of (at most) shadow_rows series covers: whole parts
// from the first, all N for shadow_rows < 0 or >= N.
void shadow_extent(const hs_index* idx, int64_t shadow_rows, int64_t* rows, int64_t* parts) {
    const IndexView& ix = idx->view;
    if (shadow_rows < 0 || shadow_rows >= ix.N) {
        *rows = ix.N;
        *parts = ix.parts;
        return;
    }
    // parts cover [part_start[p], part_start[p + 1]) in order: the last whole one
    const std::vector<int64_t>& ps = idx->part_start_host;
    const int64_t p = (int64_t)(std::upper_bound(ps.begin(), ps.end(), shadow_rows) - ps.begin()) - 1;
    *parts = std::max<int64_t>(0, p);
    *rows = ps[(size_t)*parts];
}

}  // namespace

extern "C" {

hs_status hs_knn_exact(hs_index* idx, const float* q_dev, int32_t Q, int32_t k, void* ws_dev, int64_t ws_bytes,
                       int64_t* ids_dev, float* d2_dev, double* err_dev, void* stats_dev, void* stream) {
    return run_knn(idx, q_dev, Q, k, ws_dev, ws_bytes, ids_dev, d2_dev, err_dev, stats_dev, stream, false);
}

hs_status hs_knn_mixed(hs_index* idx, const float* q_dev, int32_t Q, int32_t k, void* ws_dev, int64_t ws_bytes,
                       int64_t* ids_dev, float* d2_dev, double* err_dev, void* stats_dev, void* stream) {
    return run_knn(idx, q_dev, Q, k, ws_dev, ws_bytes, ids_dev, d2_dev, err_dev, stats_dev, stream, true);
}

hs_status hs_shadow_bytes(const hs_index* idx, int32_t kind, int64_t shadow_rows, int64_t* bytes) {
    if (!idx || !bytes) return fail(HS_EINVAL, "NULL argument");
    if (kind != kShadowBf16 && kind != kShadowF16) return fail(HS_EINVAL, "unknown shadow kind %d", kind);
    int64_t R, P;
    shadow_extent(idx, shadow_rows, &R, &P);
    *bytes = shadow_layout(idx->view, R, nullptr, nullptr, nullptr, nullptr);
    return HS_OK;
}

hs_status hs_build_shadow(hs_index* idx, int32_t kind, int64_t shadow_rows, void* shadow_dev, int64_t shadow_bytes,
                          void* stream) {
    if (!idx || !shadow_dev) return fail(HS_EINVAL, "NULL argument");
    if (kind != kShadowBf16 && kind != kShadowF16) return fail(HS_EINVAL, "unknown shadow kind %d", kind);
    int64_t R, P;
    shadow_extent(idx, shadow_rows, &R, &P);
    const int64_t need = shadow_layout(idx->view, R, nullptr, nullptr, nullptr, nullptr);
    if (shadow_bytes < need)
        return fail(HS_ENOMEM, "shadow_bytes=%lld < required %lld", (long long)shadow_bytes, (long long)need);
    hipStream_t st = (hipStream_t)stream;
    uint16_t* rows;
    float4* norms;
    uint32_t* flag;
    shadow_layout(idx->view, R, &rows, &norms, &flag, (char*)shadow_dev);
    idx->shadow = ShadowView{};
    HIP_TRY(hipMemsetAsync(flag, 0, 4, st));
    HIP_TRY(hipMemsetAsync(rows + R * idx->view.stride, 0, (size_t)kBoundRows * idx->view.stride * 2, st));
    HIP_TRY(hipMemsetAsync(norms + R, 0, (size_t)kBoundRows * 16, st));
    HIP_TRY(launch_shadow(idx->view, kind, R, rows, norms, flag, st));
    uint32_t bad = 0;
    HIP_TRY(hipMemcpyAsync(&bad, flag, 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (bad) return fail(HS_EINVAL, "a series value lies beyond the fp16 range; use HS_SHADOW_BF16");
    idx->shadow.rows = rows;
    idx->shadow.norms = norms;
    idx->shadow.kind = kind;
    idx->shadow.rows_n = R;
    idx->shadow.parts_n = P;
    return HS_OK;
}

hs_status hs_profile_enable(int32_t on) {
    std::lock_guard<std::mutex> g(g_prof_mu);
    g_prof_on = on != 0;
    return HS_OK;
}

hs_status hs_union_bytes(const hs_index* idx, int64_t* bytes) {
    if (!idx || !bytes) return fail(HS_EINVAL, "NULL argument");
    *bytes = (union_bits(idx->view) + 31) / 32 * 4;
    return HS_OK;
}

hs_status hs_union_enable(void* bits_dev, int64_t bytes) {
    if (bits_dev && (bytes < 4 || bytes % 4)) return fail(HS_EINVAL, "bytes=%lld: a positive multiple of 4", (long long)bytes);
    std::lock_guard<std::mutex> g(g_prof_mu);
    g_union_bits = (uint32_t*)bits_dev;
    g_union_bytes = bits_dev ? bytes : 0;
    return HS_OK;
}

hs_status hs_union_count(const hs_index* idx, const void* bits_dev, uint64_t* counts_dev, void* stream) {
    if (!idx || !bits_dev || !counts_dev) return fail(HS_EINVAL, "NULL argument");
    HIP_TRY(launch_union_count(idx->view, (const uint32_t*)bits_dev, (unsigned long long*)counts_dev,
                               (hipStream_t)stream));
    return HS_OK;
}

hs_status hs_profile_read(int32_t kind, double* ms, int64_t* launches, int32_t reset) {
    if (kind < 0 || kind >= HS_PROF_KINDS) return fail(HS_EINVAL, "kind=%d out of range", kind);
    std::lock_guard<std::mutex> g(g_prof_mu);
    if (ms) *ms = g_prof_ms[kind];
    if (launches) *launches = g_prof_launches[kind];
    if (reset) {
        g_prof_ms[kind] = 0.0;
        g_prof_launches[kind] = 0;
    }
    return HS_OK;
}

hs_status hs_lds_probe(int32_t pattern, int32_t rounds, int32_t passes, uint32_t* sink_dev, void* stream,
                       double* lookups_per_s) {
    if (!sink_dev || !lookups_per_s) return fail(HS_EINVAL, "NULL argument");
    if ((pattern != 0 && pattern != 1) || rounds < 1 || rounds > (1 << 20) || passes < 1)
        return fail(HS_EINVAL, "pattern=%d (0 or 1), rounds=%d (1..2^20), passes=%d (>= 1)", pattern, rounds, passes);
    hipStream_t st = (hipStream_t)stream;
    int device = 0, cus = 0;
    HIP_TRY(hipGetDevice(&device));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = launch_lds_probe(pattern, rounds, sink_dev, cus, st);  // warm-up launch
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    for (int32_t i = 0; i < passes && e == hipSuccess; ++i) e = launch_lds_probe(pattern, rounds, sink_dev, cus, st);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) return fail(HS_EHIP, "LDS probe: %s", hipGetErrorString(e));
    if (!(t > 0.0f)) return fail(HS_EHIP, "LDS probe: no elapsed time");
    const double lookups = (double)cus * 4 * 256 * (double)rounds * 16 * passes;
    *lookups_per_s = lookups / ((double)t / 1e3);
    return HS_OK;
}

hs_status hs_read_probe(const void* buf_dev, int64_t bytes, int32_t passes, uint32_t* sink_dev, void* stream,
                        double* ms) {
    if (!buf_dev || !sink_dev || !ms) return fail(HS_EINVAL, "NULL argument");
    if (bytes < (1 << 20) || bytes % 16 || passes < 1)
        return fail(HS_EINVAL, "bytes=%lld (a multiple of 16, at least 1 MiB), passes=%d (>= 1)", (long long)bytes, passes);
    hipStream_t st = (hipStream_t)stream;
    int device = 0, cus = 0;
    HIP_TRY(hipGetDevice(&device));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = launch_read_probe(buf_dev, bytes, sink_dev, cus, st);  // warm-up pass
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    for (int32_t i = 0; i < passes && e == hipSuccess; ++i) e = launch_read_probe(buf_dev, bytes, sink_dev, cus, st);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) return fail(HS_EHIP, "read probe: %s", hipGetErrorString(e));
    *ms = (double)t;
    return HS_OK;
}

hs_status hs_index_free(hs_index* idx) {
    delete idx;  // the tables live in the caller's index memory
    return HS_OK;
}

}  // extern "C"
