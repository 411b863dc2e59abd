// Query-side kernels around the scan (Hercules Sec. 3.4, Exact-kNN):
//   init_counters  reset the per-call counters and candidate regions
//   query_prep     query PAA / segment stats (FP64) and the LB_SAX table
//   lb_eapca       LB_EAPCA of every (query, leaf)
//   seed           step 1, approximate search: in the l_max leaves with the
//                  smallest LB_EAPCA, refine the series with the smallest
//                  LB_SAX; their k-th distance is the first BSF_k
//   emit           step 2: (query, part) work items for the leaves whose
//                  LB_EAPCA does not exceed BSF_k
//   merge          per query: sort + dedupe the result pool, keep the top k,
//                  tighten BSF_k, write the final (d, id) lists
//   arm_redo       select the queries of the next fallback round
#include "hs_device.h"

namespace hs {
namespace {

__global__ void k_init_counters(QueryWs ws) {
    const int t = threadIdx.x;
    if (t < kNumCounters) ws.counters[t] = t == kCtrOvfEnd ? 0xffffffffu : 0u;
}

__global__ void __launch_bounds__(256) k_query_prep(IndexView ix, const float* __restrict__ qin, QueryWs ws) {
    __shared__ double s_paa[64];
    __shared__ int s_bad;
    const int q = blockIdx.x, t = threadIdx.x;
    const float* src = qin + (int64_t)q * ix.n;
    if (t == 0) s_bad = 0;
    __syncthreads();
    for (int j = t; j < ix.stride; j += blockDim.x) {
        float v = j < ix.n ? src[j] : 0.0f;
        if (!isfinite(v)) s_bad = 1;
        ws.qrow[(int64_t)q * ix.stride + j] = v;
    }
    const int32_t l = ix.n / ix.w;
    if (t < ix.w) {
        const float* p = src + t * l;
        double s = 0.0;
        for (int j = 0; j < l; ++j) s += (double)p[j];
        const double mu = s / l;
        double ss = 0.0;
        for (int j = 0; j < l; ++j) {
            double d = (double)p[j] - mu;
            ss += d * d;
        }
        const double sd = sqrt(ss / l);
        s_paa[t] = mu;
        ws.qstat[((int64_t)q * ix.w + t) * 2 + 0] = mu;
        ws.qstat[((int64_t)q * ix.w + t) * 2 + 1] = sd;
        ws.qst32[(int64_t)q * ix.w + t] =
            make_float4(__double2float_rd(mu), __double2float_ru(mu), __double2float_rd(sd), __double2float_ru(sd));
    }
    __syncthreads();
    // LB_SAX table: (n/w) * distance^2 from the query's PAA value to each
    // symbol's region, FP64, rounded down to float32
    const double scale = (double)ix.n / ix.w;
    for (int idx = t; idx < ix.w * kCard; idx += blockDim.x) {
        const int i = idx / kCard, s = idx % kCard;
        const double g = gap(s_paa[i], (double)ix.beta[s], (double)ix.beta[s + 1]);
        ws.lut[(int64_t)q * ix.w * kCard + idx] = __double2float_rd(scale * g * g);
    }
    if (t == 0) {
        ws.bkey[q] = kInfKey;
        ws.pool_cnt[q] = 0;
        ws.flags[q] = s_bad ? kFlagNonFinite : 0u;
        ws.kept[q] = 0;
        if (s_bad) atomicAdd(&ws.counters[kCtrNonFinite], 1u);
    }
    if (t < kStatSlots) ws.stats[(int64_t)q * kStatSlots + t] = 0;
}

// LB_EAPCA^2 = sum_i l_i [gap(mu_q, [mu_min, mu_max])^2 + gap(sd_q, [sd_min, sd_max])^2]
// in FP64, rounded down to float32.
__global__ void __launch_bounds__(256) k_lb_eapca(IndexView ix, QueryWs ws) {
    __shared__ double s_st[128];
    const int q = blockIdx.y;
    for (int j = threadIdx.x; j < 2 * ix.w; j += blockDim.x) s_st[j] = ws.qstat[(int64_t)q * ix.w * 2 + j];
    __syncthreads();
    const int64_t leaf = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (leaf >= ix.L) return;
    const double l = (double)(ix.n / ix.w);
    double acc = 0.0;
    for (int i = 0; i < ix.w; ++i) {
        const float4 e = ix.env[leaf * ix.w + i];
        const double gm = gap(s_st[2 * i], (double)e.x, (double)e.y);
        const double gs = gap(s_st[2 * i + 1], (double)e.z, (double)e.w);
        acc += l * (gm * gm + gs * gs);
    }
    ws.lbe[(int64_t)q * ix.L + leaf] = __double2float_rd(acc);
}

// Step 1 (approximate search), one block per query.  The paper refines every
// series of the L_max most promising leaves; here the same leaves are chosen
// (smallest LB_EAPCA) but only their series with the smallest LB_SAX are
// refined -- at least max(seed_rows, 2k) of them, cut at a histogram bin of
// LB_SAX values, at most kSeedList.  The selected series are gathered into a
// list, refined together (16 lanes per series; no abandoning, the block has no
// BSF_k yet), and the k best by (d, id), found by a bitonic sort of the list's
// keys, become the first pool entries and BSF_k.  Every distance here is a
// result key (compensated, natural chunk order).
// One workgroup per query: 512 threads (two fit a CU, so a batch of 512
// queries runs at once), or 1,024 when the batch has at most one query per
// CU, which halves each workgroup's passes over the words (single queries
// and batches of 60 about 2 % faster at 10M x 256).
constexpr int kSeedList = 2048;

template <int W16, int kSeedThreads>
__global__ void __launch_bounds__(kSeedThreads) k_seed(IndexView ix, ScanParams sp, QueryWs ws) {
    constexpr int kSeedWaves = kSeedThreads / 64;
    constexpr int kSeedBins = 2048 / kSeedThreads;  // histogram bins per thread
    constexpr int kPassRows = W16 == 1 ? 8 : (W16 == 2 ? 4 : 2);  // rows per thread per pass
    extern __shared__ float s_lut[];  // [16 W16][256], rows beyond w zero
    __shared__ uint32_t s_hist[2048];
    __shared__ unsigned long long s_keys[kSeedList];
    __shared__ uint32_t s_list[kSeedList];
    __shared__ uint32_t s_leaves[kMaxSeedLeaves];
    __shared__ unsigned long long s_tmp[kSeedWaves];
    __shared__ int s_w[kSeedWaves];
    __shared__ uint32_t s_binlim;
    __shared__ int s_cnt;
    const int q = blockIdx.x, t = threadIdx.x, sub = t & 15, grp = t >> 4;
    const int k = sp.k, lm = sp.n_seed;
    const int nchunks = ix.stride / kChunk;
    load_lut<W16>(s_lut, ws.lut + (int64_t)q * ix.w * kCard, ix.w, t, blockDim.x);
    for (int j = t; j < 2048; j += blockDim.x) s_hist[j] = 0;
    if (t == 0) {
        s_cnt = 0;
        s_binlim = 2047;
    }
    // the lm leaves with the smallest (LB_EAPCA, leaf id)
    unsigned long long last = 0;
    for (int r = 0; r < lm; ++r) {
        unsigned long long best = ~0ull;
        for (int64_t leaf = t; leaf < ix.L; leaf += blockDim.x) {
            const unsigned long long key = leaf_key(ws.lbe[(int64_t)q * ix.L + leaf], leaf);
            if ((r == 0 || key > last) && key < best) best = key;
        }
        best = block_min_u64(best, s_tmp);
        last = best;
        if (t == 0) s_leaves[r] = (uint32_t)(best & 0xffffffffu);
    }
    __syncthreads();
    // histogram of LB_SAX over the seed leaves (bins: float bits >> 20)
    int64_t rows = 0;
    for (int li = 0; li < lm; ++li) {
        const int64_t b = ix.leaf_start[s_leaves[li]], e = ix.leaf_start[s_leaves[li] + 1];
        rows += e - b;
        // kPassRows rows per thread per pass, their word loads in flight together
        for (int64_t tb = b; tb < e; tb += kPassRows * (int64_t)blockDim.x) {
            uint4 v[kPassRows][W16];
#pragma unroll
            for (int j = 0; j < kPassRows; ++j) {
                const int64_t r = min(tb + t + (int64_t)blockDim.x * j, e - 1);
                load_word<W16>(ix.words + r * ix.wstride, v[j]);
            }
#pragma unroll
            for (int j = 0; j < kPassRows; ++j) {
                if (tb + t + (int64_t)blockDim.x * j < e) {
                    const float lb = lb_sax_word<W16>(v[j], s_lut);
                    atomicAdd(&s_hist[min(__float_as_uint(lb) >> 20, 2047u)], 1u);
                }
            }
        }
    }
    __syncthreads();
    // the cut: the first bin at which the cumulative count reaches the target
    // (thread t owns bins kSeedBins t .. kSeedBins t + kSeedBins - 1)
    {
        const uint32_t want = (uint32_t)max(sp.seed_rows, 2 * k);
        int c8 = 0;
#pragma unroll
        for (int b = 0; b < kSeedBins; ++b) c8 += (int)s_hist[kSeedBins * t + b];
        int tot;
        uint32_t cum = (uint32_t)block_exclusive_scan<kSeedWaves>(c8, s_w, &tot);
        for (int b = 0; b < kSeedBins; ++b) {
            const uint32_t before = cum;
            cum += s_hist[kSeedBins * t + b];
            if (before < want && cum >= want) s_binlim = kSeedBins * t + b;  // one thread finds the crossing
        }
    }
    __syncthreads();
    const uint32_t lim = s_binlim;
    // gather the series whose LB_SAX bin does not exceed the cut (kPassRows per
    // thread per pass, one block scan per pass)
    for (int li = 0; li < lm; ++li) {
        const int64_t b = ix.leaf_start[s_leaves[li]], e = ix.leaf_start[s_leaves[li] + 1];
        for (int64_t tb = b; tb < e; tb += kPassRows * (int64_t)blockDim.x) {
            uint32_t pm = 0;
#pragma unroll
            for (int j = 0; j < kPassRows; ++j) {
                const int64_t r = tb + t + (int64_t)blockDim.x * j;
                if (r < e) {
                    uint4 v[W16];
                    load_word<W16>(ix.words + r * ix.wstride, v);
                    const float lb = lb_sax_word<W16>(v, s_lut);
                    if ((__float_as_uint(lb) >> 20) <= lim) pm |= 1u << j;
                }
            }
            int tot;
            const int off = block_exclusive_scan<kSeedWaves>(__popc(pm), s_w, &tot);
            const int base = s_cnt;
            int o = base + off;
#pragma unroll
            for (int j = 0; j < kPassRows; ++j) {
                if ((pm >> j) & 1u) {
                    if (o < kSeedList) s_list[o] = (uint32_t)(tb + t + (int64_t)blockDim.x * j);
                    ++o;
                }
            }
            __syncthreads();
            if (t == 0) s_cnt = min(base + tot, kSeedList);
            __syncthreads();
        }
    }
    const int M = s_cnt;
    // refine the list: a group takes kSeedRows rows at a time and loads their
    // chunks (kSeedChunks per row) together; each row adds its chunks in
    // chunk order, as everywhere
    constexpr int kSeedRows = 4, kSeedChunks = 4;
    const float* qr = ws.qrow + (int64_t)q * ix.stride + sub * 4;
    for (int i0 = grp * kSeedRows; i0 < M; i0 += (kSeedThreads / 16) * kSeedRows) {
        int64_t pos[kSeedRows];
#pragma unroll
        for (int r = 0; r < kSeedRows; ++r) pos[r] = s_list[min(i0 + r, M - 1)];
        Dist<kComp> d[kSeedRows];
        for (int c = 0; c < nchunks; c += kSeedChunks) {
            float4 qa[kSeedChunks], xa[kSeedRows][kSeedChunks];
#pragma unroll
            for (int b = 0; b < kSeedChunks; ++b)
                qa[b] = c + b < nchunks ? *reinterpret_cast<const float4*>(qr + (c + b) * kChunk)
                                        : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
            for (int r = 0; r < kSeedRows; ++r)
#pragma unroll
                for (int b = 0; b < kSeedChunks; ++b)
                    xa[r][b] = c + b < nchunks
                                   ? *reinterpret_cast<const float4*>(ix.rows + pos[r] * ix.stride + sub * 4 + (c + b) * kChunk)
                                   : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
            for (int r = 0; r < kSeedRows; ++r)
#pragma unroll
                for (int b = 0; b < kSeedChunks; ++b)
                    if (c + b < nchunks) d[r].add(qa[b], xa[r][b]);
        }
#pragma unroll
        for (int r = 0; r < kSeedRows; ++r)
            if (i0 + r < M && sub == 0)
                s_keys[i0 + r] = ((unsigned long long)__float_as_uint(d[r].value()) << 32) | ix.ids[pos[r]];
    }
    int Mp = 1;
    while (Mp < M) Mp <<= 1;
    for (int i = M + t; i < Mp; i += blockDim.x) s_keys[i] = ~0ull;
    __syncthreads();
    // bitonic sort of the keys, ascending
    for (int size = 2; size <= Mp; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = t; i < Mp; i += blockDim.x) {
                const int j2 = i ^ stride;
                if (j2 > i) {
                    const bool up = (i & size) == 0;
                    const unsigned long long a = s_keys[i], c = s_keys[j2];
                    if ((a > c) == up) {
                        s_keys[i] = c;
                        s_keys[j2] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    const int n = min(k, M);
    for (int j = t; j < n; j += blockDim.x) ws.pool[(int64_t)q * ws.P + j] = s_keys[j];
    if (t == 0) {
        ws.pool_cnt[q] = (uint32_t)n;
        if (n == k) ws.bkey[q] = s_keys[k - 1];
        unsigned long long* st = ws.stats + (int64_t)q * kStatSlots;
        st[1] += (unsigned long long)rows;
        st[2] += (unsigned long long)M;
        st[3] += (unsigned long long)M * nchunks;
    }
}

// Step 2: one block per query; the (query, part) items of every leaf whose
// LB_EAPCA does not exceed BSF_k, contiguous per query.  Also counts the
// candidate leaves and picks the access path (eapca_th).
__global__ void __launch_bounds__(256) k_emit(IndexView ix, ScanParams sp, int32_t redo_only, QueryWs ws) {
    __shared__ int s_w[4];
    __shared__ uint32_t s_base;
    const int q = blockIdx.x, t = threadIdx.x;
    const uint32_t f = ws.flags[q];
    if (redo_only && !(f & kFlagInRound)) return;
    const double thr = prune_limit(bits_to_float(bsf_bits(ws, q)));
    const float* lbe = ws.lbe + (int64_t)q * ix.L;
    if (!redo_only) {
        int kept = 0;
        for (int64_t leaf = t; leaf < ix.L; leaf += blockDim.x) kept += (double)lbe[leaf] <= thr;
        int tot;
        block_exclusive_scan(kept, s_w, &tot);
        if (t == 0) {
            ws.kept[q] = (uint32_t)tot;
            if (sp.eapca_th > 0.0f && (1.0 - (double)tot / (double)ix.L) < (double)sp.eapca_th)
                ws.flags[q] = f | kFlagSkipSax;
        }
    }
    // parts from emit_part0 on (a partial low-precision copy bounds the others)
    const int64_t p0 = redo_only ? 0 : sp.emit_part0;
    int cnt = 0;
    for (int64_t p = p0 + t; p < ix.parts; p += blockDim.x) cnt += (double)lbe[ix.part_leaf[p]] <= thr;
    int total;
    block_exclusive_scan(cnt, s_w, &total);
    if (t == 0) s_base = total ? atomicAdd(&ws.counters[kCtrItems], (uint32_t)total) : 0u;
    __syncthreads();
    uint32_t base = s_base;
    for (int64_t pb = p0; pb < ix.parts; pb += blockDim.x) {
        const int64_t p = pb + t;
        const bool c = p < ix.parts && (double)lbe[ix.part_leaf[p]] <= thr;
        int tot;
        const int off = block_exclusive_scan(c ? 1 : 0, s_w, &tot);
        if (c && (int64_t)(base + off) < ws.item_cap) ws.items[base + off] = ((uint64_t)q << 32) | (uint32_t)p;
        base += tot;
    }
}

__global__ void __launch_bounds__(1024) k_merge(IndexView ix, ScanParams sp, int32_t redo_only, QueryWs ws,
                                                int64_t* __restrict__ ids_out, float* __restrict__ d2_out,
                                                double* __restrict__ err_out, double err_rel,
                                                hs_query_stats* __restrict__ stats_out) {
    extern __shared__ unsigned long long s_keys[];  // [P]
    __shared__ int s_u;
    const int q = blockIdx.x, t = threadIdx.x;
    if (redo_only && !(ws.flags[q] & kFlagInRound)) return;
    const int k = sp.k;
    uint32_t cnt = ws.pool_cnt[q];
    if (cnt > (uint32_t)ws.P) cnt = ws.P;
    int M = 1;
    while (M < (int)cnt) M <<= 1;
    for (int j = t; j < M; j += blockDim.x) s_keys[j] = j < (int)cnt ? ws.pool[(int64_t)q * ws.P + j] : ~0ull;
    __syncthreads();
    // bitonic sort, ascending
    for (int size = 2; size <= M; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = t; i < M; i += blockDim.x) {
                const int j = i ^ stride;
                if (j > i) {
                    const bool up = (i & size) == 0;
                    const unsigned long long a = s_keys[i], c = s_keys[j];
                    if ((a > c) == up) {
                        s_keys[i] = c;
                        s_keys[j] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    if (t == 0) {
        // drop duplicates (a series re-admitted in a later round), keep the first k
        int u = 0;
        unsigned long long prev = ~0ull;
        for (int j = 0; j < (int)cnt && u < k; ++j) {
            const unsigned long long key = s_keys[j];
            if (u > 0 && key == prev) continue;
            s_keys[u++] = key;
            prev = key;
        }
        s_u = u;
        const uint32_t f = ws.flags[q];
        const bool again = (f & (kFlagOverflow | kFlagCandLost)) != 0;
        uint32_t nf = f & ~(kFlagOverflow | kFlagCandLost);
        if (again) {
            nf |= kFlagRedo;
            atomicAdd(&ws.counters[kCtrRedo], 1u);
            if (f & kFlagCandLost) atomicAdd(&ws.counters[kCtrLost], 1u);
        }
        ws.flags[q] = nf;
        ws.pool_cnt[q] = (uint32_t)u;
        if (u == k) atomicMin(&ws.bkey[q], s_keys[k - 1]);
        if (sp.final_pass) ws.stats[(int64_t)q * kStatSlots + 5] += 1;
    }
    __syncthreads();
    const int u = s_u;
    for (int j = t; j < u; j += blockDim.x) ws.pool[(int64_t)q * ws.P + j] = s_keys[j];
    if (sp.final_pass) {
        for (int j = t; j < k; j += blockDim.x) {
            if (j < u) {
                const float d = bits_to_float((uint32_t)(s_keys[j] >> 32));
                ids_out[(int64_t)q * k + j] = (int64_t)(s_keys[j] & 0xffffffffull);
                d2_out[(int64_t)q * k + j] = d;
                if (err_out) err_out[(int64_t)q * k + j] = err_rel * (double)d;
            } else {
                ids_out[(int64_t)q * k + j] = -1;
                d2_out[(int64_t)q * k + j] = INFINITY;
                if (err_out) err_out[(int64_t)q * k + j] = INFINITY;
            }
        }
        if (stats_out && t == 0) {
            const unsigned long long* st = ws.stats + (int64_t)q * kStatSlots;
            hs_query_stats o;
            o.leaves_kept = ws.kept[q];
            o.rows_filtered = st[1];
            o.rows_refined = st[2];
            o.chunks_read = st[3];
            o.path = (ws.flags[q] & kFlagSkipSax) ? 1 : 0;
            o.rounds = st[5];
            o.candidates = st[6];
            o.chunks_tested = st[7];
            o.rows_bounded = st[0];
            o.bound_pairs = st[4];
            o.rows_sigma = st[8];
            stats_out[q] = o;
        }
    }
}

// Batch-union diagnostics: the marked units of each region of the bit array
// (raw chunk pairs [0, word_bit0), words [word_bit0, env_bit0), envelopes
// [env_bit0, end)) added to counts[0..2].
__global__ void __launch_bounds__(256) k_union_count(const uint32_t* __restrict__ bits, int64_t nwords,
                                                      int64_t word_bit0, int64_t env_bit0, int64_t end_bit,
                                                      unsigned long long* counts) {
    __shared__ unsigned long long s_c[3][4];
    const int64_t b0[3] = {0, word_bit0, env_bit0}, b1[3] = {word_bit0, env_bit0, end_bit};
    unsigned long long c[3] = {0ull, 0ull, 0ull};
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nwords; i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t v = bits[i];
        if (!v) continue;
        const int64_t lo = i * 32, hi = lo + 32;
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            const int64_t a = max(lo, b0[r]), b = min(hi, b1[r]);
            if (a >= b) continue;
            const int sh = (int)(a - lo), len = (int)(b - a);
            const uint32_t m = (len == 32 ? 0xffffffffu : ((1u << len) - 1u)) << sh;
            c[r] += (unsigned long long)__popc(v & m);
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        unsigned long long x = c[r];
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
        if (lane == 0) s_c[r][wave] = x;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        const unsigned long long s = s_c[threadIdx.x][0] + s_c[threadIdx.x][1] + s_c[threadIdx.x][2] + s_c[threadIdx.x][3];
        if (s) atomicAdd(&counts[threadIdx.x], s);
    }
}

__global__ void k_reset_items(uint32_t* c) {
    if (threadIdx.x == 0) {
        c[kCtrItems] = 0;
        c[kCtrWork] = 0;
    }
}

__global__ void k_arm_redo(QueryWs ws, int32_t Q) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q == 0) {
        ws.counters[kCtrItems] = 0;
        ws.counters[kCtrWork] = 0;
        ws.counters[kCtrRedo] = 0;
        ws.counters[kCtrLost] = 0;
        // the candidate list's overflow slice, for a round that refills it
        ws.counters[kCtrOvf] = 0;
        ws.counters[kCtrOvfEnd] = 0xffffffffu;
    }
    if (q >= Q) return;
    uint32_t f = ws.flags[q];
    f = (f & kFlagRedo) ? ((f & ~kFlagRedo) | kFlagInRound) : (f & ~kFlagInRound);
    ws.flags[q] = f;
}

}  // namespace

hipError_t launch_query_prep(const IndexView& ix, const float* q, int32_t Q, const QueryWs& ws, hipStream_t st) {
    hipLaunchKernelGGL(k_init_counters, dim3(1), dim3(64), 0, st, ws);
    hipLaunchKernelGGL(k_query_prep, dim3(Q), dim3(256), 0, st, ix, q, ws);
    return hipGetLastError();
}

hipError_t launch_lb_eapca(const IndexView& ix, int32_t Q, const QueryWs& ws, hipStream_t st) {
    hipLaunchKernelGGL(k_lb_eapca, dim3((unsigned)((ix.L + 255) / 256), Q), dim3(256), 0, st, ix, ws);
    return hipGetLastError();
}

hipError_t launch_seed(const IndexView& ix, const ScanParams& sp, const QueryWs& ws, int form, hipStream_t st) {
    if (sp.n_seed <= 0) return hipSuccess;
    (void)form;  // the seed keys its results in the compensated form for both forms
    const size_t lds = sizeof(float) * (size_t)16 * w16_of(ix) * kCard;
    int device = 0, cus = 0;
    if (hipGetDevice(&device) == hipSuccess)
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    if (sp.Q <= cus) {
        HS_DISPATCH_W16_F(ix, k_seed, 1024, dim3(sp.Q), dim3(1024), lds, st, ix, sp, ws);
    } else {
        HS_DISPATCH_W16_F(ix, k_seed, 512, dim3(sp.Q), dim3(512), lds, st, ix, sp, ws);
    }
    return hipGetLastError();
}

hipError_t launch_emit(const IndexView& ix, const ScanParams& sp, bool redo_only, const QueryWs& ws,
                       hipStream_t st) {
    if (redo_only) {
        hipLaunchKernelGGL(k_arm_redo, dim3((sp.Q + 255) / 256), dim3(256), 0, st, ws, sp.Q);
    } else {
        hipLaunchKernelGGL(k_reset_items, dim3(1), dim3(64), 0, st, ws.counters);
    }
    hipLaunchKernelGGL(k_emit, dim3(sp.Q), dim3(kTile), 0, st, ix, sp, redo_only ? 1 : 0, ws);
    return hipGetLastError();
}

hipError_t launch_union_count(const IndexView& ix, const uint32_t* bits, unsigned long long* counts, hipStream_t st) {
    const int64_t end_bit = union_bits(ix);
    const int64_t word_bit0 = ix.N * (int64_t)(ix.stride / kChunk);
    const int64_t nwords = (end_bit + 31) / 32;
    hipLaunchKernelGGL(k_union_count, dim3(grid_for(nwords, 256, 4096)), dim3(256), 0, st, bits, nwords, word_bit0,
                       word_bit0 + ix.N, end_bit, counts);
    return hipGetLastError();
}

hipError_t launch_merge(const IndexView& ix, const ScanParams& sp, bool redo_only, const QueryWs& ws,
                        int64_t* ids_out, float* d2_out, double* err_out, double err_rel,
                        hs_query_stats* stats_out, hipStream_t st) {
    hipLaunchKernelGGL(k_merge, dim3(sp.Q), dim3(1024), sizeof(unsigned long long) * ws.P, st, ix, sp,
                       redo_only ? 1 : 0, ws, ids_out, d2_out, err_out, err_rel, stats_out);
    return hipGetLastError();
}

}  // namespace hs
