// HIP kernels for exact data-series k-NN search on gfx950 (CDNA4).
//
// Build side (Hercules Sec. 2 summaries, Sec. 3.1 tree):
//   series_stats  per (series, segment) mean and population std (FP64 math)
//   gather_rows   leaf-ordered, zero-padded copy of the series
//   words         iSAX symbol per (series, segment): FP64 PAA against the
//                 float32 Gaussian breakpoints
//   envelopes     per (leaf, segment) min/max of mean and std, rounded
//                 outward to float32 so they contain the FP64 statistics
//
// Query side (Hercules Sec. 3.3, Exact-kNN, steps 1-4):
//   query_prep    query PAA / segment stats (FP64) and the LB_SAX table
//   lb_eapca      LB_EAPCA of every (query, leaf)
//   seed          step 1, approximate search: in the l_max leaves with the
//                 smallest LB_EAPCA, refine the series with the smallest
//                 LB_SAX; their k-th distance is the first BSF_k
//   emit          step 2: (query, part) work items for the leaves whose
//                 LB_EAPCA does not exceed BSF_k
//   filter        step 3: LB_SAX of every series of every item; survivors are
//                 appended to a candidate list (wavefront scan compaction)
//   refine        step 4: exact float32 distance with early abandoning, each
//                 candidate re-checked against the current BSF_k; per-block
//                 top-k, BSF_k published with atomicMin, results to a pool
//   leaf_scan     steps 3+4 fused per item: the path for queries whose
//                 candidate list or result pool overflowed
//   merge         per query: sort + dedupe the pool, keep the top k, tighten
//                 BSF_k, write the final (d, id) lists
//
// Result keys are (float bits of d << 32 | original id): for d >= 0 the
// unsigned order of the key is the (d, id) lexicographic order.
//
// Distances: 16 lanes own one series; lane l holds points 4l..4l+3 of every
// 64-point chunk.  A chunk's partial is the lane's sequential fma chain over
// its 4 points, summed over the 16 lanes by a xor butterfly (commutative, so
// every lane holds the same value); d adds the chunk partials in chunk order.
// This order is the same in every kernel, so a (query, series) pair always
// gets the same float32 distance.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "hs_internal.h"

namespace hs {

namespace {

__device__ __forceinline__ double gap(double v, double lo, double hi) {
    return v < lo ? lo - v : (v > hi ? v - hi : 0.0);
}

__device__ __forceinline__ float bits_to_float(uint32_t b) { return __uint_as_float(b); }

__device__ __forceinline__ uint32_t load_relaxed(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ double prune_limit(float bsf) { return (double)bsf * (1.0 + kSlack); }

// ------------------------------------------------------------------ build

__global__ void k_series_stats(const float* __restrict__ x, int64_t N, int32_t n, int32_t w,
                               float2* __restrict__ out, uint32_t* bad) {
    const int32_t l = n / w;
    const int64_t total = N * (int64_t)w;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t row = t / w;
        const int32_t seg = (int32_t)(t - row * w);
        const float* p = x + row * n + (int64_t)seg * l;
        double s = 0.0;
        bool ok = true;
        for (int j = 0; j < l; ++j) {
            float v = p[j];
            ok &= isfinite(v);
            s += (double)v;
        }
        const double mu = s / l;
        double ss = 0.0;
        for (int j = 0; j < l; ++j) {
            double d = (double)p[j] - mu;
            ss += d * d;
        }
        if (!ok) atomicOr(bad, 1u);
        out[t] = make_float2((float)mu, (float)sqrt(ss / l));
    }
}

__global__ void k_gather_rows(const float* __restrict__ x, const uint32_t* __restrict__ perm, int64_t N,
                              int32_t n, int32_t stride, float* __restrict__ rows) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int64_t pos = blockIdx.x * (int64_t)(blockDim.x >> 6) + wave; pos < N;
         pos += (int64_t)gridDim.x * (blockDim.x >> 6)) {
        const float* src = x + (int64_t)perm[pos] * n;
        float* dst = rows + pos * stride;
        for (int j = lane; j < stride; j += 64) dst[j] = j < n ? src[j] : 0.0f;
    }
}

__global__ void k_words(IndexView ix, uint8_t* __restrict__ words) {
    __shared__ float s_beta[kCard + 1];
    for (int j = threadIdx.x; j <= kCard; j += blockDim.x) s_beta[j] = ix.beta[j];
    __syncthreads();
    const int32_t l = ix.n / ix.w;
    const int64_t total = ix.N * (int64_t)ix.w;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t pos = t / ix.w;
        const int32_t seg = (int32_t)(t - pos * ix.w);
        const float* p = ix.rows + pos * ix.stride + (int64_t)seg * l;
        double s = 0.0;
        for (int j = 0; j < l; ++j) s += (double)p[j];
        const double paa = s / l;
        // symbol = #{j in 1..255 : beta_j <= paa}: upper bound over beta[1..255]
        int lo = 1, hi = kCard;  // answer index in [1, 256]; symbol = index - 1
        while (lo < hi) {
            int mid = (lo + hi) >> 1;
            if ((double)s_beta[mid] <= paa) lo = mid + 1; else hi = mid;
        }
        words[pos * ix.wstride + seg] = (uint8_t)(lo - 1);
    }
}

__global__ void __launch_bounds__(256) k_envelopes(IndexView ix, float4* __restrict__ env) {
    __shared__ double s_red[256][4];
    const int64_t leaf = blockIdx.x;
    const int64_t b = ix.leaf_start[leaf], e = ix.leaf_start[leaf + 1];
    const int32_t w = ix.w, l = ix.n / w;
    const int G = 256 / w;  // threads per segment
    const int t = threadIdx.x;
    double mn = INFINITY, mx = -INFINITY, sn = INFINITY, sx = -INFINITY;
    if (t < G * w) {
        const int seg = t % w, grp = t / w;
        for (int64_t r = b + grp; r < e; r += G) {
            const float* p = ix.rows + r * ix.stride + (int64_t)seg * l;
            double s = 0.0;
            for (int j = 0; j < l; ++j) s += (double)p[j];
            const double mu = s / l;
            double ss = 0.0;
            for (int j = 0; j < l; ++j) {
                double d = (double)p[j] - mu;
                ss += d * d;
            }
            const double sd = sqrt(ss / l);
            mn = fmin(mn, mu);
            mx = fmax(mx, mu);
            sn = fmin(sn, sd);
            sx = fmax(sx, sd);
        }
    }
    s_red[t][0] = mn;
    s_red[t][1] = mx;
    s_red[t][2] = sn;
    s_red[t][3] = sx;
    __syncthreads();
    if (t < w) {
        for (int g = 1; g < G; ++g) {
            const int o = g * w + t;
            mn = fmin(mn, s_red[o][0]);
            mx = fmax(mx, s_red[o][1]);
            sn = fmin(sn, s_red[o][2]);
            sx = fmax(sx, s_red[o][3]);
        }
        // outward rounding: the float32 box contains every member's FP64 statistic
        env[leaf * w + t] = make_float4(__double2float_rd(mn), __double2float_ru(mx), __double2float_rd(sn),
                                        __double2float_ru(sx));
    }
}

// --------------------------------------------------------- shared pieces

// LB_SAX of one stored series: sum over segments of the query's table entry
// for the series' symbol (words are 16-byte aligned, W16 uint4 per word).
template <int W16>
__device__ __forceinline__ float lb_sax_word(const uint4 (&v)[W16], const float* s_lut, int w) {
    float acc = 0.0f;
#pragma unroll
    for (int u = 0; u < W16; ++u) {
        const uint32_t parts[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
#pragma unroll
        for (int p = 0; p < 4; ++p) {
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int i = u * 16 + p * 4 + b;
                if (i < w) acc += s_lut[i * kCard + ((parts[p] >> (8 * b)) & 0xffu)];
            }
        }
    }
    return acc;
}

template <int W16>
__device__ __forceinline__ void load_word(const uint8_t* __restrict__ wp, uint4 (&v)[W16]) {
#pragma unroll
    for (int u = 0; u < W16; ++u) v[u] = *reinterpret_cast<const uint4*>(wp + 16 * u);
}

__device__ __forceinline__ float chunk_partial(float4 q, float4 x) {
    const float t0 = q.x - x.x, t1 = q.y - x.y, t2 = q.z - x.z, t3 = q.w - x.w;
    float p = t0 * t0;
    p = fmaf(t1, t1, p);
    p = fmaf(t2, t2, p);
    p = fmaf(t3, t3, p);
    p += __shfl_xor(p, 1, 16);
    p += __shfl_xor(p, 2, 16);
    p += __shfl_xor(p, 4, 16);
    p += __shfl_xor(p, 8, 16);
    return p;
}

// Squared distance of one series, computed by the 16 lanes of a group (all 16
// active together).  xr / qr point at the lane's first point.  Chunks are
// loaded two at a time; after each pair the running sum is compared with
// thr and the series is abandoned once it exceeds it (the final sum can only
// be larger).  `chunks` counts the chunks read.
__device__ __forceinline__ float refine_row(const float* __restrict__ xr, const float* __restrict__ qr,
                                           int nchunks, float thr, bool& alive, unsigned& chunks) {
    float d = 0.0f;
    alive = true;
    for (int c = 0; c < nchunks; c += 2) {
        const bool two = c + 1 < nchunks;
        const float4 x0 = *reinterpret_cast<const float4*>(xr + c * kChunk);
        float4 x1 = make_float4(0.f, 0.f, 0.f, 0.f);
        if (two) x1 = *reinterpret_cast<const float4*>(xr + (c + 1) * kChunk);
        d += chunk_partial(*reinterpret_cast<const float4*>(qr + c * kChunk), x0);
        if (two) d += chunk_partial(*reinterpret_cast<const float4*>(qr + (c + 1) * kChunk), x1);
        chunks += two ? 2u : 1u;
        if (d > thr) {
            alive = false;
            break;
        }
    }
    return d;
}

// Insert key into the ascending list top[0..n) of capacity k (one thread).
__device__ __forceinline__ void topk_insert(unsigned long long* top, int& n, int k, unsigned long long key) {
    if (n == k && key >= top[k - 1]) return;
    int p = n < k ? n : k - 1;
    while (p > 0 && top[p - 1] > key) {
        top[p] = top[p - 1];
        --p;
    }
    top[p] = key;
    if (n < k) ++n;
}

// Publish a block's top-k for query q (one thread): tighten BSF_k with its
// k-th distance, then append the entries that do not exceed BSF_k to the pool.
__device__ void flush_topk(const QueryWs& ws, int q, int k, const unsigned long long* top, int n) {
    if (q < 0 || n == 0) return;
    float g = bits_to_float(load_relaxed(&ws.bsf[q]));
    if (n == k) {
        const uint32_t kb = (uint32_t)(top[k - 1] >> 32);
        if (bits_to_float(kb) < g) {
            atomicMin(&ws.bsf[q], kb);
            g = bits_to_float(kb);
        }
    }
    int cnt = 0;
    while (cnt < n && bits_to_float((uint32_t)(top[cnt] >> 32)) <= g) ++cnt;
    if (cnt == 0) return;
    const uint32_t base = atomicAdd(&ws.pool_cnt[q], (uint32_t)cnt);
    for (int j = 0; j < cnt; ++j)
        if (base + j < (uint32_t)ws.P) ws.pool[(int64_t)q * ws.P + base + j] = top[j];
    if (base + cnt > (uint32_t)ws.P) atomicOr(&ws.flags[q], kFlagOverflow);
}

// Exclusive prefix sum over the 256 threads of a block; returns the offset of
// this thread and writes the block total to *total.  s_w holds 4 ints.
__device__ __forceinline__ int block_exclusive_scan(int v, int* s_w, int* total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    if (lane == 63) s_w[wave] = inc;
    __syncthreads();
    int off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < kTile / 64; ++i) {
        const int c = s_w[i];
        if (i < wave) off += c;
        tot += c;
    }
    *total = tot;
    __syncthreads();
    return off + inc - v;
}

__device__ __forceinline__ uint64_t leaf_key(float lbe, int64_t leaf) {
    return ((uint64_t)__float_as_uint(lbe) << 32) | (uint64_t)(uint32_t)leaf;
}

__device__ unsigned long long block_min_u64(unsigned long long v, unsigned long long* s_tmp) {
    for (int o = 32; o > 0; o >>= 1) {
        unsigned long long other = __shfl_xor(v, o, 64);
        v = other < v ? other : v;
    }
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) s_tmp[wave] = v;
    __syncthreads();
    unsigned long long r = s_tmp[0];
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) r = s_tmp[i] < r ? s_tmp[i] : r;
    __syncthreads();
    return r;
}

// ------------------------------------------------------------------ query

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
        s_paa[t] = mu;
        ws.qstat[((int64_t)q * ix.w + t) * 2 + 0] = mu;
        ws.qstat[((int64_t)q * ix.w + t) * 2 + 1] = sqrt(ss / l);
    }
    __syncthreads();
    const double scale = (double)ix.n / ix.w;
    for (int idx = t; idx < ix.w * kCard; idx += blockDim.x) {
        const int i = idx / kCard, s = idx % kCard;
        const double g = gap(s_paa[i], (double)ix.beta[s], (double)ix.beta[s + 1]);
        ws.lut[(int64_t)q * ix.w * kCard + idx] = __double2float_rd(scale * g * g);
    }
    if (t == 0) {
        ws.bsf[q] = kInfBits;
        ws.pool_cnt[q] = 0;
        ws.flags[q] = s_bad ? kFlagNonFinite : 0u;
        ws.kept[q] = 0;
        if (s_bad) atomicAdd(&ws.counters[kCtrNonFinite], 1u);
    }
    if (t < 8) ws.stats[(int64_t)q * 8 + t] = 0;
}

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
// refined -- at least seed_rows of them, cut at a histogram bin of LB_SAX
// values.  The k best become the first pool entries and BSF_k.
template <int W16>
__global__ void __launch_bounds__(256) k_seed(IndexView ix, ScanParams sp, QueryWs ws) {
    extern __shared__ float s_lut[];  // [w][256]
    __shared__ unsigned long long s_top[HS_KMAX];
    __shared__ unsigned long long s_res[kTile];
    __shared__ uint32_t s_hits[kTile];
    __shared__ uint32_t s_hist[2048];
    __shared__ uint32_t s_leaves[kMaxSeedLeaves];
    __shared__ unsigned long long s_tmp[4];
    __shared__ int s_w[4];
    __shared__ int s_nres, s_topn;
    __shared__ float s_thr;
    __shared__ uint32_t s_binlim;
    __shared__ unsigned int s_ref, s_chunks;
    const int q = blockIdx.x, t = threadIdx.x, sub = t & 15, grp = t >> 4;
    const int k = sp.k, lm = sp.n_seed;
    const int nchunks = ix.stride / kChunk;
    for (int j = t; j < ix.w * kCard; j += blockDim.x) s_lut[j] = ws.lut[(int64_t)q * ix.w * kCard + j];
    for (int j = t; j < 2048; j += blockDim.x) s_hist[j] = 0;
    if (t == 0) {
        s_nres = 0;
        s_topn = 0;
        s_thr = INFINITY;
        s_ref = 0;
        s_chunks = 0;
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
        for (int64_t r = b + t; r < e; r += blockDim.x) {
            uint4 v[W16];
            load_word<W16>(ix.words + r * ix.wstride, v);
            const float lb = lb_sax_word<W16>(v, s_lut, ix.w);
            atomicAdd(&s_hist[min(__float_as_uint(lb) >> 20, 2047u)], 1u);
        }
    }
    __syncthreads();
    if (t == 0) {
        const uint32_t want = (uint32_t)max(sp.seed_rows, 2 * k);
        uint32_t cum = 0, lim = 2047;
        for (uint32_t b = 0; b < 2048; ++b) {
            cum += s_hist[b];
            if (cum >= want) {
                lim = b;
                break;
            }
        }
        s_binlim = lim;
    }
    __syncthreads();
    const uint32_t lim = s_binlim;
    unsigned my_chunks = 0, my_ref = 0;
    for (int li = 0; li < lm; ++li) {
        const int64_t b = ix.leaf_start[s_leaves[li]], e = ix.leaf_start[s_leaves[li] + 1];
        for (int64_t tb = b; tb < e; tb += kTile) {
            const int64_t r = tb + t;
            bool pass = false;
            if (r < e) {
                uint4 v[W16];
                load_word<W16>(ix.words + r * ix.wstride, v);
                const float lb = lb_sax_word<W16>(v, s_lut, ix.w);
                pass = (__float_as_uint(lb) >> 20) <= lim && (double)lb <= prune_limit(s_thr);
            }
            int nh;
            const int off = block_exclusive_scan(pass ? 1 : 0, s_w, &nh);
            if (pass) s_hits[off] = (uint32_t)(r - b);
            __syncthreads();
            const float thr = s_thr;
            for (int h = grp; h < nh; h += kTile / 16) {
                const int64_t pos = b + s_hits[h];
                bool alive;
                const float d = refine_row(ix.rows + pos * ix.stride + sub * 4,
                                           ws.qrow + (int64_t)q * ix.stride + sub * 4, nchunks, thr, alive,
                                           my_chunks);
                if (sub == 0) {
                    ++my_ref;
                    if (alive) s_res[atomicAdd(&s_nres, 1)] = ((unsigned long long)__float_as_uint(d) << 32) | ix.ids[pos];
                }
            }
            __syncthreads();
            if (t == 0) {
                int n = s_topn;
                for (int i = 0; i < s_nres; ++i) topk_insert(s_top, n, k, s_res[i]);
                s_topn = n;
                s_nres = 0;
                if (n == k) s_thr = bits_to_float((uint32_t)(s_top[k - 1] >> 32));
            }
            __syncthreads();
        }
    }
    if (sub == 0) {
        atomicAdd(&s_ref, my_ref);
        atomicAdd(&s_chunks, my_chunks);
    }
    __syncthreads();
    const int n = s_topn;
    for (int j = t; j < n; j += blockDim.x) ws.pool[(int64_t)q * ws.P + j] = s_top[j];
    if (t == 0) {
        ws.pool_cnt[q] = (uint32_t)n;
        if (n == k) ws.bsf[q] = (uint32_t)(s_top[k - 1] >> 32);
        unsigned long long* st = ws.stats + (int64_t)q * 8;
        st[1] += (unsigned long long)rows;
        st[2] += s_ref;
        st[3] += s_chunks;
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
    const double thr = prune_limit(bits_to_float(ws.bsf[q]));
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
    int cnt = 0;
    for (int64_t p = t; p < ix.parts; p += blockDim.x) cnt += (double)lbe[ix.part_leaf[p]] <= thr;
    int total;
    block_exclusive_scan(cnt, s_w, &total);
    if (t == 0) s_base = total ? atomicAdd(&ws.counters[kCtrItems], (uint32_t)total) : 0u;
    __syncthreads();
    uint32_t base = s_base;
    for (int64_t p0 = 0; p0 < ix.parts; p0 += blockDim.x) {
        const int64_t p = p0 + t;
        const bool c = p < ix.parts && (double)lbe[ix.part_leaf[p]] <= thr;
        int tot;
        const int off = block_exclusive_scan(c ? 1 : 0, s_w, &tot);
        if (c && (int64_t)(base + off) < ws.item_cap) ws.items[base + off] = ((uint64_t)q << 32) | (uint32_t)p;
        base += tot;
    }
}

// Step 3: persistent blocks take units of kUnit consecutive items (items of
// one query are contiguous, so the LB_SAX table is reloaded only when the
// query changes).  Each thread evaluates up to kPartRows / 256 series; the
// survivors of an item are appended with one atomicAdd.
constexpr int kUnit = 4;
constexpr int kRowsPerThread = kPartRows / kTile;

template <int W16>
__global__ void __launch_bounds__(256) k_filter(IndexView ix, ScanParams sp, QueryWs ws) {
    extern __shared__ float s_lut[];  // [w][256]
    __shared__ uint32_t s_unit, s_base;
    __shared__ int s_w[4];
    const int t = threadIdx.x;
    const uint32_t n_items = ws.counters[kCtrItems];
    int cur_q = -1;
    while (true) {
        if (t == 0) s_unit = atomicAdd(&ws.counters[kCtrWork], (uint32_t)kUnit);
        __syncthreads();
        const uint32_t u0 = s_unit;
        __syncthreads();
        if (u0 >= n_items) break;
        for (int it = 0; it < kUnit; ++it) {
            const uint32_t idx = u0 + it;
            if (idx >= n_items || (int64_t)idx >= ws.item_cap) break;
            const uint64_t item = ws.items[idx];
            const int q = (int)(item >> 32);
            const int64_t p = (int64_t)(uint32_t)item;
            if (q != cur_q) {
                for (int j = t; j < ix.w * kCard; j += blockDim.x) s_lut[j] = ws.lut[(int64_t)q * ix.w * kCard + j];
                cur_q = q;
                __syncthreads();
            }
            const bool skip = (ws.flags[q] & kFlagSkipSax) != 0;
            const double thr = prune_limit(bits_to_float(ws.bsf[q]));
            if ((double)ws.lbe[(int64_t)q * ix.L + ix.part_leaf[p]] > thr) continue;
            const int64_t pb = ix.part_start[p], pe = ix.part_start[p + 1];
            uint4 v[kRowsPerThread][W16];
#pragma unroll
            for (int j = 0; j < kRowsPerThread; ++j) {
                const int64_t r = pb + t + j * kTile;
                if (!skip && r < pe) load_word<W16>(ix.words + r * ix.wstride, v[j]);
            }
            float lbv[kRowsPerThread];
            uint32_t mask = 0;
#pragma unroll
            for (int j = 0; j < kRowsPerThread; ++j) {
                const int64_t r = pb + t + j * kTile;
                lbv[j] = 0.0f;
                if (r < pe) {
                    if (!skip) lbv[j] = lb_sax_word<W16>(v[j], s_lut, ix.w);
                    if ((double)lbv[j] <= thr) mask |= 1u << j;
                }
            }
            int total;
            const int off = block_exclusive_scan(__popc(mask), s_w, &total);
            if (t == 0) {
                uint32_t base = 0xffffffffu;
                if (total > 0) {
                    // once the list is full no more ranges are reserved, so the
                    // 32-bit counter overshoots the capacity by at most one
                    // range per resident block
                    if ((int64_t)load_relaxed(&ws.counters[kCtrCand]) >= ws.cand_cap) {
                        atomicOr(&ws.flags[q], kFlagCandLost);
                    } else {
                        const uint32_t b = atomicAdd(&ws.counters[kCtrCand], (uint32_t)total);
                        if ((int64_t)b + total <= ws.cand_cap) {
                            base = b;
                        } else {
                            // this range is never written; the refine kernel stops below it
                            atomicMin(&ws.counters[kCtrCandEnd], b);
                            atomicOr(&ws.flags[q], kFlagCandLost);
                        }
                    }
                }
                s_base = base;
                if (!skip) atomicAdd(&ws.stats[(int64_t)q * 8 + 1], (unsigned long long)(pe - pb));
            }
            __syncthreads();
            const uint32_t base = s_base;
            if (base != 0xffffffffu) {
                int o = off;
#pragma unroll
                for (int j = 0; j < kRowsPerThread; ++j) {
                    if (mask & (1u << j)) {
                        const int64_t slot = (int64_t)base + o;
                        ws.cand_pos[slot] = (uint32_t)(pb + t + j * kTile);
                        ws.cand_q[slot] = (uint32_t)q;
                        ws.cand_lb[slot] = lbv[j];
                        ++o;
                    }
                }
            }
            __syncthreads();
        }
    }
}

// Step 4: persistent blocks take kGrab consecutive candidates; each 16-lane
// group refines kGrab / 16 of them.  A candidate whose LB_SAX exceeds the
// query's current BSF_k is skipped without reading its values.  Admitted
// results go to a block-local top-k of the current query, flushed to the pool
// when the query changes and at the end.
constexpr int kGrab = 64;

__global__ void __launch_bounds__(256) k_refine(IndexView ix, ScanParams sp, QueryWs ws) {
    __shared__ unsigned long long s_top[HS_KMAX];
    __shared__ unsigned long long s_res[kGrab];
    __shared__ int s_resq[kGrab];
    __shared__ int s_nres, s_topn, s_curq;
    __shared__ uint32_t s_grab;
    const int t = threadIdx.x, lane = t & 63, sub = t & 15, grp = t >> 4;
    const int k = sp.k;
    const int nchunks = ix.stride / kChunk;
    // every entry below min(counter, first range that did not fit) was written
    const int64_t ncand =
        min(min((int64_t)ws.counters[kCtrCand], (int64_t)ws.counters[kCtrCandEnd]), ws.cand_cap);
    if (t == 0) {
        s_nres = 0;
        s_topn = 0;
        s_curq = -1;
    }
    int st_q = -1;
    unsigned st_ref = 0, st_chunks = 0;
    while (true) {
        if (t == 0) s_grab = atomicAdd(&ws.counters[kCtrRefine], (uint32_t)kGrab);
        __syncthreads();
        const int64_t base = s_grab;
        if (base >= ncand) break;
#pragma unroll 1
        for (int j = 0; j < kGrab / 16; ++j) {
            const int64_t c = base + grp * (kGrab / 16) + j;
            if (c >= ncand) break;
            const int q = (int)ws.cand_q[c];
            const uint32_t pos = ws.cand_pos[c];
            const float lb = ws.cand_lb[c];
            // one BSF_k value for the whole group: the 16 lanes leave the chunk loop together
            float thr = bits_to_float(load_relaxed(&ws.bsf[q]));
            thr = __shfl(thr, lane & ~15, 64);
            if ((double)lb > prune_limit(thr)) continue;
            if (q != st_q) {
                if (sub == 0 && st_q >= 0) {
                    atomicAdd(&ws.stats[(int64_t)st_q * 8 + 2], (unsigned long long)st_ref);
                    atomicAdd(&ws.stats[(int64_t)st_q * 8 + 3], (unsigned long long)st_chunks);
                }
                st_q = q;
                st_ref = 0;
                st_chunks = 0;
            }
            bool alive;
            const float d = refine_row(ix.rows + (int64_t)pos * ix.stride + sub * 4,
                                       ws.qrow + (int64_t)q * ix.stride + sub * 4, nchunks, thr, alive, st_chunks);
            if (sub == 0) {
                ++st_ref;
                if (alive) {
                    const int slot = atomicAdd(&s_nres, 1);
                    s_res[slot] = ((unsigned long long)__float_as_uint(d) << 32) | ix.ids[pos];
                    s_resq[slot] = q;
                }
            }
        }
        __syncthreads();
        if (t == 0) {
            int n = s_topn, cq = s_curq;
            for (int i = 0; i < s_nres; ++i) {
                if (s_resq[i] != cq) {
                    flush_topk(ws, cq, k, s_top, n);
                    cq = s_resq[i];
                    n = 0;
                }
                topk_insert(s_top, n, k, s_res[i]);
            }
            s_topn = n;
            s_curq = cq;
            s_nres = 0;
        }
        __syncthreads();
    }
    if (sub == 0 && st_q >= 0) {
        // chunks were counted by every lane of the group; lane 0's count is the group's
        atomicAdd(&ws.stats[(int64_t)st_q * 8 + 2], (unsigned long long)st_ref);
        atomicAdd(&ws.stats[(int64_t)st_q * 8 + 3], (unsigned long long)st_chunks);
    }
    if (t == 0) flush_topk(ws, s_curq, k, s_top, s_topn);
}

// Steps 3+4 fused per (query, part) item: the path taken by queries whose
// candidate list or result pool overflowed.  Needs no candidate buffer.
struct ScanShared {
    unsigned long long top[HS_KMAX];
    unsigned long long res[kTile];
    uint32_t hits[kTile];
    int w[4];
    int nres, topn;
    float thr;  // block-uniform pruning threshold (a valid upper bound of BSF_k)
    uint32_t item_idx;
    unsigned int st_filt, st_ref, st_chunks;
};

template <int W16>
__global__ void __launch_bounds__(256) k_leaf_scan(IndexView ix, ScanParams sp, QueryWs ws) {
    extern __shared__ float s_dyn[];
    __shared__ ScanShared sh;
    float* s_q = s_dyn;                    // [stride]
    float* s_lut = s_dyn + ix.stride;      // [w][256]
    const int t = threadIdx.x;
    const int grp = t >> 4, sub = t & 15;
    const uint32_t n_items = ws.counters[kCtrItems];
    const int nchunks = ix.stride / kChunk;
    const int k = sp.k;

    while (true) {
        if (t == 0) sh.item_idx = atomicAdd(&ws.counters[kCtrWork], 1u);
        __syncthreads();
        const uint32_t idx = sh.item_idx;
        if (idx >= n_items || (int64_t)idx >= ws.item_cap) break;
        const uint64_t item = ws.items[idx];
        const int q = (int)(item >> 32);
        const int64_t part = (int64_t)(uint32_t)item;

        for (int j = t; j < ix.stride; j += blockDim.x) s_q[j] = ws.qrow[(int64_t)q * ix.stride + j];
        for (int j = t; j < ix.w * kCard; j += blockDim.x) s_lut[j] = ws.lut[(int64_t)q * ix.w * kCard + j];
        if (t == 0) {
            sh.topn = 0;
            sh.nres = 0;
            sh.st_filt = 0;
            sh.st_ref = 0;
            sh.st_chunks = 0;
            sh.thr = bits_to_float(load_relaxed(&ws.bsf[q]));
        }
        const bool skip_sax = (ws.flags[q] & kFlagSkipSax) != 0;
        const int64_t b = ix.part_start[part], e = ix.part_start[part + 1];
        unsigned int my_filt = 0, my_ref = 0, my_chunks = 0;
        __syncthreads();
        float thr = sh.thr;

        for (int64_t tb = b; tb < e; tb += kTile) {
            const int64_t r = tb + t;
            bool pass = false;
            if (r < e) {
                if (skip_sax) {
                    pass = true;
                } else {
                    uint4 v[W16];
                    load_word<W16>(ix.words + r * ix.wstride, v);
                    const float lb = lb_sax_word<W16>(v, s_lut, ix.w);
                    ++my_filt;
                    pass = (double)lb <= prune_limit(thr);
                }
            }
            int nh;
            const int off = block_exclusive_scan(pass ? 1 : 0, sh.w, &nh);
            if (pass) sh.hits[off] = (uint32_t)(r - b);
            __syncthreads();
            for (int h = grp; h < nh; h += kTile / 16) {
                const int64_t pos = b + sh.hits[h];
                bool alive;
                const float d = refine_row(ix.rows + pos * ix.stride + sub * 4, s_q + sub * 4, nchunks, thr, alive,
                                           my_chunks);
                if (sub == 0) {
                    ++my_ref;
                    if (alive) sh.res[atomicAdd(&sh.nres, 1)] = ((unsigned long long)__float_as_uint(d) << 32) | ix.ids[pos];
                }
            }
            __syncthreads();
            if (t == 0) {
                int n = sh.topn;
                for (int i = 0; i < sh.nres; ++i) topk_insert(sh.top, n, k, sh.res[i]);
                sh.topn = n;
                sh.nres = 0;
                const float g = bits_to_float(load_relaxed(&ws.bsf[q]));
                const float lk = n == k ? bits_to_float((uint32_t)(sh.top[k - 1] >> 32)) : INFINITY;
                sh.thr = fminf(g, lk);
            }
            __syncthreads();
            thr = sh.thr;
        }

        atomicAdd(&sh.st_filt, my_filt);
        if (sub == 0) {
            atomicAdd(&sh.st_ref, my_ref);
            atomicAdd(&sh.st_chunks, my_chunks);
        }
        __syncthreads();
        if (t == 0) {
            flush_topk(ws, q, k, sh.top, sh.topn);
            unsigned long long* st = ws.stats + (int64_t)q * 8;
            atomicAdd(&st[1], (unsigned long long)sh.st_filt);
            atomicAdd(&st[2], (unsigned long long)sh.st_ref);
            atomicAdd(&st[3], (unsigned long long)sh.st_chunks);
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ merge

__global__ void __launch_bounds__(1024) k_merge(IndexView ix, ScanParams sp, int32_t redo_only, QueryWs ws,
                                                int64_t* __restrict__ ids_out, float* __restrict__ d2_out,
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
        }
        ws.flags[q] = nf;
        ws.pool_cnt[q] = (uint32_t)u;
        if (u == k) atomicMin(&ws.bsf[q], (uint32_t)(s_keys[k - 1] >> 32));
        if (sp.final_pass) ws.stats[(int64_t)q * 8 + 5] += 1;
    }
    __syncthreads();
    const int u = s_u;
    for (int j = t; j < u; j += blockDim.x) ws.pool[(int64_t)q * ws.P + j] = s_keys[j];
    if (sp.final_pass) {
        for (int j = t; j < k; j += blockDim.x) {
            if (j < u) {
                ids_out[(int64_t)q * k + j] = (int64_t)(s_keys[j] & 0xffffffffull);
                d2_out[(int64_t)q * k + j] = bits_to_float((uint32_t)(s_keys[j] >> 32));
            } else {
                ids_out[(int64_t)q * k + j] = -1;
                d2_out[(int64_t)q * k + j] = INFINITY;
            }
        }
        if (stats_out && t == 0) {
            const unsigned long long* st = ws.stats + (int64_t)q * 8;
            hs_query_stats o;
            o.leaves_kept = ws.kept[q];
            o.rows_filtered = st[1];
            o.rows_refined = st[2];
            o.chunks_read = st[3];
            o.path = (ws.flags[q] & kFlagSkipSax) ? 1 : 0;
            o.rounds = st[5];
            o.reserved[0] = 0;
            o.reserved[1] = 0;
            stats_out[q] = o;
        }
    }
}

__global__ void k_set_counters(uint32_t* c, int first, int count) {
    const int i = first + (int)threadIdx.x;
    if ((int)threadIdx.x < count) c[i] = i == kCtrCandEnd ? 0xffffffffu : 0u;
}

__global__ void k_arm_redo(QueryWs ws, int32_t Q) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q == 0) {
        for (int i = 0; i < kNumCounters; ++i)
            if (i != kCtrNonFinite) ws.counters[i] = i == kCtrCandEnd ? 0xffffffffu : 0u;
    }
    if (q >= Q) return;
    uint32_t f = ws.flags[q];
    f = (f & kFlagRedo) ? ((f & ~kFlagRedo) | kFlagInRound) : (f & ~kFlagInRound);
    ws.flags[q] = f;
}

int grid_for(int64_t work, int block, int cap = 65536) {
    int64_t g = (work + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

int w16_of(const IndexView& ix) { return (ix.wstride + 15) / 16; }

int blocks_per_cu(size_t lds_bytes) {
    int per_cu = (int)((160 * 1024) / (lds_bytes + 1024));
    if (per_cu > 8) per_cu = 8;
    if (per_cu < 1) per_cu = 1;
    return per_cu;
}

}  // namespace

// ---------------------------------------------------------------- launchers

#define HS_DISPATCH_W16(ix, KERNEL, ...)                                              \
    switch (w16_of(ix)) {                                                            \
        case 1: hipLaunchKernelGGL(KERNEL<1>, __VA_ARGS__); break;                   \
        case 2: hipLaunchKernelGGL(KERNEL<2>, __VA_ARGS__); break;                   \
        case 3: hipLaunchKernelGGL(KERNEL<3>, __VA_ARGS__); break;                   \
        default: hipLaunchKernelGGL(KERNEL<4>, __VA_ARGS__); break;                  \
    }

hipError_t launch_series_stats(const float* x, int64_t N, int32_t n, int32_t w, float2* st_out, uint32_t* bad,
                               hipStream_t st) {
    hipLaunchKernelGGL(k_series_stats, dim3(grid_for(N * w, 256)), dim3(256), 0, st, x, N, n, w, st_out, bad);
    return hipGetLastError();
}

hipError_t launch_gather_rows(const float* x, const uint32_t* perm, int64_t N, int32_t n, int32_t stride,
                              float* rows, hipStream_t st) {
    hipLaunchKernelGGL(k_gather_rows, dim3(grid_for(N, 4)), dim3(256), 0, st, x, perm, N, n, stride, rows);
    return hipGetLastError();
}

hipError_t launch_words(const IndexView& ix, uint8_t* words, hipStream_t st) {
    hipLaunchKernelGGL(k_words, dim3(grid_for(ix.N * ix.w, 256)), dim3(256), 0, st, ix, words);
    return hipGetLastError();
}

hipError_t launch_envelopes(const IndexView& ix, float4* env, hipStream_t st) {
    hipLaunchKernelGGL(k_envelopes, dim3((unsigned)ix.L), dim3(256), 0, st, ix, env);
    return hipGetLastError();
}

hipError_t launch_query_prep(const IndexView& ix, const float* q, int32_t Q, const QueryWs& ws, hipStream_t st) {
    hipLaunchKernelGGL(k_set_counters, dim3(1), dim3(64), 0, st, ws.counters, 0, kNumCounters);
    hipLaunchKernelGGL(k_query_prep, dim3(Q), dim3(256), 0, st, ix, q, ws);
    return hipGetLastError();
}

hipError_t launch_lb_eapca(const IndexView& ix, int32_t Q, const QueryWs& ws, hipStream_t st) {
    hipLaunchKernelGGL(k_lb_eapca, dim3((unsigned)((ix.L + 255) / 256), Q), dim3(256), 0, st, ix, ws);
    return hipGetLastError();
}

hipError_t launch_seed(const IndexView& ix, const ScanParams& sp, const QueryWs& ws, hipStream_t st) {
    if (sp.n_seed <= 0) return hipSuccess;
    const size_t lds = sizeof(float) * (size_t)ix.w * kCard;
    HS_DISPATCH_W16(ix, k_seed, dim3(sp.Q), dim3(kTile), lds, st, ix, sp, ws);
    return hipGetLastError();
}

hipError_t launch_emit(const IndexView& ix, const ScanParams& sp, bool redo_only, const QueryWs& ws,
                       hipStream_t st) {
    if (redo_only) {
        hipLaunchKernelGGL(k_arm_redo, dim3((sp.Q + 255) / 256), dim3(256), 0, st, ws, sp.Q);
    } else {
        hipLaunchKernelGGL(k_set_counters, dim3(1), dim3(64), 0, st, ws.counters, kCtrItems, 2);
    }
    hipLaunchKernelGGL(k_emit, dim3(sp.Q), dim3(kTile), 0, st, ix, sp, redo_only ? 1 : 0, ws);
    return hipGetLastError();
}

hipError_t launch_filter(const IndexView& ix, const ScanParams& sp, const QueryWs& ws, int device_cus,
                         hipStream_t st) {
    const size_t lds = sizeof(float) * (size_t)ix.w * kCard;
    HS_DISPATCH_W16(ix, k_filter, dim3(device_cus * blocks_per_cu(lds + 64)), dim3(kTile), lds, st, ix, sp, ws);
    return hipGetLastError();
}

hipError_t launch_refine(const IndexView& ix, const ScanParams& sp, const QueryWs& ws, int device_cus,
                         hipStream_t st) {
    hipLaunchKernelGGL(k_refine, dim3(device_cus * 8), dim3(kTile), 0, st, ix, sp, ws);
    return hipGetLastError();
}

hipError_t launch_leaf_scan(const IndexView& ix, const ScanParams& sp, const QueryWs& ws, int device_cus,
                            hipStream_t st) {
    const size_t lds = sizeof(float) * ((size_t)ix.stride + (size_t)ix.w * kCard);
    HS_DISPATCH_W16(ix, k_leaf_scan, dim3(device_cus * blocks_per_cu(lds + sizeof(ScanShared))), dim3(kTile), lds,
                    st, ix, sp, ws);
    return hipGetLastError();
}

hipError_t launch_merge(const IndexView& ix, const ScanParams& sp, bool redo_only, const QueryWs& ws,
                        int64_t* ids_out, float* d2_out, hs_query_stats* stats_out, hipStream_t st) {
    hipLaunchKernelGGL(k_merge, dim3(sp.Q), dim3(1024), sizeof(unsigned long long) * ws.P, st, ix, sp,
                       redo_only ? 1 : 0, ws, ids_out, d2_out, stats_out);
    return hipGetLastError();
}

}  // namespace hs
