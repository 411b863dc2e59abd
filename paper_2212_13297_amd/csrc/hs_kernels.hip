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
// Query side (Hercules Sec. 3.3, Exact-kNN):
//   query_prep    query PAA / segment stats (FP64) and the LB_SAX table
//   lb_eapca      LB_EAPCA of every (query, leaf)
//   seed_select   the l_max leaves with the smallest LB_EAPCA (approximate
//                 search, step 1)
//   emit_main     candidate leaves: LB_EAPCA <= BSF_k (step 2)
//   leaf_scan     persistent workgroups over (query, leaf) items: LB_SAX per
//                 series with wavefront ballot compaction (step 3), then exact
//                 float32 refinement with early abandoning and a per-item
//                 top-k, publishing BSF_k with atomicMin (step 4)
//   merge         per query: sort + dedupe the candidate pool, keep the top k,
//                 tighten BSF_k, write the final (d, id) lists
//
// Result keys are (float bits of d << 32 | original id): for d >= 0 the
// unsigned order of the key is the (d, id) lexicographic order.
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

constexpr int kFlagOverflow = 1;
constexpr int kFlagNonFinite = 4;
constexpr int kFlagRedo = 8;      // needs another refinement round
constexpr int kFlagInRound = 16;  // takes part in the current redo round

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
        ws.flags[q] = s_bad ? kFlagNonFinite : 0;
        ws.kept[q] = 0;
        ws.seed_key[q] = 0;
        if (s_bad) atomicAdd(&ws.counters[3], 1u);
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

__device__ __forceinline__ uint64_t leaf_key(float lbe, int64_t leaf) {
    return ((uint64_t)__float_as_uint(lbe) << 32) | (uint64_t)(uint32_t)leaf;
}

template <typename T>
__device__ T block_min_u64(T v, T* s_tmp) {
    // 256-thread block minimum of unsigned 64-bit values
    for (int o = 32; o > 0; o >>= 1) {
        T other = __shfl_xor(v, o, 64);
        v = other < v ? other : v;
    }
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) s_tmp[wave] = v;
    __syncthreads();
    T r = s_tmp[0];
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) r = s_tmp[i] < r ? s_tmp[i] : r;
    __syncthreads();
    return r;
}

__global__ void __launch_bounds__(256) k_seed_select(IndexView ix, int32_t l_max, QueryWs ws) {
    __shared__ unsigned long long s_tmp[4];
    const int q = blockIdx.x;
    const int lm = (int)(l_max < ix.L ? l_max : ix.L);
    unsigned long long last = 0;
    for (int r = 0; r < lm; ++r) {
        unsigned long long best = ~0ull;
        for (int64_t leaf = threadIdx.x; leaf < ix.L; leaf += blockDim.x) {
            unsigned long long key = leaf_key(ws.lbe[(int64_t)q * ix.L + leaf], leaf);
            if ((r == 0 || key > last) && key < best) best = key;
        }
        best = block_min_u64(best, s_tmp);
        last = best;
        if (threadIdx.x == 0) ws.items[(int64_t)q * lm + r] = ((uint64_t)q << 32) | (uint32_t)(best & 0xffffffffu);
    }
    // a leaf is a seed leaf iff its key < seed_key (seed_key = last + 1, 0 = none)
    if (threadIdx.x == 0) ws.seed_key[q] = lm > 0 ? last + 1 : 0;
}

__global__ void k_set_counters(uint32_t* c, uint32_t c0, uint32_t c1) {
    if (threadIdx.x == 0) {
        c[0] = c0;
        c[1] = c1;
    }
}

__global__ void k_arm_redo(QueryWs ws, int32_t Q) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q == 0) {
        ws.counters[0] = 0;
        ws.counters[1] = 0;
        ws.counters[2] = 0;
    }
    if (q >= Q) return;
    uint32_t f = ws.flags[q];
    f = (f & kFlagRedo) ? ((f & ~kFlagRedo) | kFlagInRound) : (f & ~kFlagInRound);
    ws.flags[q] = f;
}

__global__ void __launch_bounds__(256) k_emit_main(IndexView ix, int32_t redo_only, QueryWs ws) {
    const int q = blockIdx.y;
    if (redo_only && !(ws.flags[q] & kFlagInRound)) return;
    const int64_t leaf = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const double thr = (double)bits_to_float(ws.bsf[q]) * (1.0 + kSlack);
    bool cand = false;
    if (leaf < ix.L) {
        const float lb = ws.lbe[(int64_t)q * ix.L + leaf];
        const bool seed = !redo_only && leaf_key(lb, leaf) < ws.seed_key[q];
        cand = !seed && (double)lb <= thr;
    }
    const uint64_t mask = __ballot(cand);
    const int lane = threadIdx.x & 63;
    const int cnt = __popcll(mask);
    uint32_t base = 0;
    if (lane == 0 && cnt) {
        base = atomicAdd(&ws.counters[0], (uint32_t)cnt);
        if (!redo_only) atomicAdd(&ws.kept[q], (uint32_t)cnt);
    }
    base = __shfl(base, 0, 64);
    if (cand) {
        const int rank = __popcll(mask & ((1ull << lane) - 1ull));
        const int64_t slot = (int64_t)base + rank;
        if (slot < ws.item_cap) ws.items[slot] = ((uint64_t)q << 32) | (uint32_t)leaf;
    }
}

// ------------------------------------------------------------- leaf scan

struct ScanShared {
    unsigned long long top[HS_KMAX];
    unsigned long long res[kTile];
    uint32_t hits[kTile];
    int wcnt[kTile / 64];
    int nhits, nres, topn;
    float thr;  // block-uniform pruning threshold (a valid upper bound of BSF_k)
    uint32_t item_idx;
    unsigned int st_filt, st_ref, st_chunks;
};

// LB_SAX of one stored series: sum over segments of the query's table entry
// for the series' symbol.
__device__ __forceinline__ float lb_sax_row(const uint8_t* __restrict__ wp, const float* s_lut, int w) {
    float acc = 0.0f;
    for (int base = 0; base < w; base += 16) {
        const uint4 v = *reinterpret_cast<const uint4*>(wp + base);
        const uint32_t parts[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int p = 0; p < 4; ++p) {
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int i = base + p * 4 + b;
                if (i < w) acc += s_lut[i * kCard + ((parts[p] >> (8 * b)) & 0xffu)];
            }
        }
    }
    return acc;
}

__global__ void __launch_bounds__(256) k_leaf_scan(IndexView ix, ScanParams sp, QueryWs ws) {
    extern __shared__ float s_dyn[];
    __shared__ ScanShared sh;
    float* s_q = s_dyn;                    // [stride]
    float* s_lut = s_dyn + ix.stride;      // [w][256]
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int grp = t >> 4, sub = t & 15;
    const uint32_t n_items = ws.counters[0];
    const int nchunks = ix.stride / kChunk;
    const int k = sp.k;

    while (true) {
        if (t == 0) sh.item_idx = atomicAdd(&ws.counters[1], 1u);
        __syncthreads();
        const uint32_t idx = sh.item_idx;
        if (idx >= n_items || (int64_t)idx >= ws.item_cap) break;
        const uint64_t item = ws.items[idx];
        const int q = (int)(item >> 32);
        const int64_t leaf = (int64_t)(uint32_t)item;

        for (int j = t; j < ix.stride; j += blockDim.x) s_q[j] = ws.qrow[(int64_t)q * ix.stride + j];
        for (int j = t; j < ix.w * kCard; j += blockDim.x) s_lut[j] = ws.lut[(int64_t)q * ix.w * kCard + j];
        if (t == 0) {
            sh.topn = 0;
            sh.nres = 0;
            sh.st_filt = 0;
            sh.st_ref = 0;
            sh.st_chunks = 0;
        }
        const bool skip_sax =
            sp.eapca_th > 0.0f && (1.0 - (double)ws.kept[q] / (double)ix.L) < (double)sp.eapca_th;
        const int64_t b = ix.leaf_start[leaf], e = ix.leaf_start[leaf + 1];
        if (t == 0) sh.thr = bits_to_float(load_relaxed(&ws.bsf[q]));
        unsigned int my_filt = 0, my_ref = 0, my_chunks = 0;
        __syncthreads();
        // every thread of the block must see the same threshold: the 16 lanes
        // refining one series leave the chunk loop together
        float thr = sh.thr;

        for (int64_t tb = b; tb < e; tb += kTile) {
            const int64_t r = tb + t;
            bool pass = false;
            if (r < e) {
                if (skip_sax) {
                    pass = true;
                } else {
                    const float lb = lb_sax_row(ix.words + r * ix.wstride, s_lut, ix.w);
                    ++my_filt;
                    pass = (double)lb <= (double)thr * (1.0 + kSlack);
                }
            }
            // block-wide stream compaction of the surviving series
            const uint64_t mask = __ballot(pass);
            if (lane == 0) sh.wcnt[wave] = __popcll(mask);
            __syncthreads();
            int off = 0;
            for (int i = 0; i < wave; ++i) off += sh.wcnt[i];
            const int nh = sh.wcnt[0] + sh.wcnt[1] + sh.wcnt[2] + sh.wcnt[3];
            if (pass) sh.hits[off + __popcll(mask & ((1ull << lane) - 1ull))] = (uint32_t)(r - b);
            __syncthreads();

            // exact refinement: 16 lanes per series, 64-point chunks, early abandoning
            for (int h = grp; h < nh; h += kTile / 16) {
                const int64_t pos = b + sh.hits[h];
                const float* xr = ix.rows + pos * ix.stride + sub * 4;
                const float* qr = s_q + sub * 4;
                float d = 0.0f;
                bool alive = true;
                float4 xv = *reinterpret_cast<const float4*>(xr);
                for (int c = 0; c < nchunks; ++c) {
                    float4 xn = xv;
                    if (c + 1 < nchunks) xn = *reinterpret_cast<const float4*>(xr + (c + 1) * kChunk);
                    const float4 qv = *reinterpret_cast<const float4*>(qr + c * kChunk);
                    const float t0 = qv.x - xv.x, t1 = qv.y - xv.y, t2 = qv.z - xv.z, t3 = qv.w - xv.w;
                    float p = t0 * t0;
                    p = fmaf(t1, t1, p);
                    p = fmaf(t2, t2, p);
                    p = fmaf(t3, t3, p);
                    p += __shfl_xor(p, 1, 16);
                    p += __shfl_xor(p, 2, 16);
                    p += __shfl_xor(p, 4, 16);
                    p += __shfl_xor(p, 8, 16);
                    d += p;
                    ++my_chunks;
                    xv = xn;
                    if (d > thr) {
                        alive = false;
                        break;
                    }
                }
                if (sub == 0) ++my_ref;
                if (alive && sub == 0) {
                    const int slot = atomicAdd(&sh.nres, 1);
                    sh.res[slot] = ((unsigned long long)__float_as_uint(d) << 32) | ix.ids[pos];
                }
            }
            __syncthreads();
            if (t == 0) {
                // merge this tile's admitted results into the item's sorted top-k
                int n = sh.topn;
                for (int i = 0; i < sh.nres; ++i) {
                    const unsigned long long key = sh.res[i];
                    if (n == k && key >= sh.top[k - 1]) continue;
                    int p = n < k ? n : k - 1;
                    while (p > 0 && sh.top[p - 1] > key) {
                        sh.top[p] = sh.top[p - 1];
                        --p;
                    }
                    sh.top[p] = key;
                    if (n < k) ++n;
                }
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
        if (sub == 0) atomicAdd(&sh.st_ref, my_ref);
        if (sub == 0) atomicAdd(&sh.st_chunks, my_chunks);
        __syncthreads();
        if (t == 0) {
            float g = bits_to_float(load_relaxed(&ws.bsf[q]));
            const int n = sh.topn;
            if (n == k) {
                const uint32_t kb = (uint32_t)(sh.top[k - 1] >> 32);
                if (bits_to_float(kb) < g) {
                    atomicMin(&ws.bsf[q], kb);
                    g = bits_to_float(kb);
                }
            }
            int cnt = 0;
            while (cnt < n && bits_to_float((uint32_t)(sh.top[cnt] >> 32)) <= g) ++cnt;
            if (cnt > 0) {
                const uint32_t base = atomicAdd(&ws.pool_cnt[q], (uint32_t)cnt);
                for (int j = 0; j < cnt; ++j)
                    if (base + j < (uint32_t)ws.P) ws.pool[(int64_t)q * ws.P + base + j] = sh.top[j];
                if (base + cnt > (uint32_t)ws.P) atomicOr(&ws.flags[q], (uint32_t)kFlagOverflow);
            }
            unsigned long long* st = ws.stats + (int64_t)q * 8;
            atomicAdd(&st[1], (unsigned long long)sh.st_filt);
            atomicAdd(&st[2], (unsigned long long)sh.st_ref);
            atomicAdd(&st[3], (unsigned long long)sh.st_chunks);
            if (skip_sax) st[4] = 1;
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
        const bool over = (f & kFlagOverflow) != 0;
        uint32_t nf = f & ~(uint32_t)kFlagOverflow;
        if (over) {
            nf |= kFlagRedo;
            atomicAdd(&ws.counters[2], 1u);
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
            o.leaves_kept = (uint64_t)ws.kept[q] + (uint64_t)sp.n_seed;
            o.rows_filtered = st[1];
            o.rows_refined = st[2];
            o.chunks_read = st[3];
            o.path = st[4];
            o.rounds = st[5];
            o.reserved[0] = 0;
            o.reserved[1] = 0;
            stats_out[q] = o;
        }
    }
}

int grid_for(int64_t work, int block, int cap = 65536) {
    int64_t g = (work + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

}  // namespace

// ---------------------------------------------------------------- launchers

hipError_t launch_series_stats(const float* x, int64_t N, int32_t n, int32_t w, float2* st_out, uint32_t* bad,
                               hipStream_t st) {
    hipLaunchKernelGGL(k_series_stats, dim3(grid_for(N * w, 256)), dim3(256), 0, st, x, N, n, w, st_out, bad);
    return hipGetLastError();
}

hipError_t launch_gather_rows(const float* x, const uint32_t* perm, int64_t N, int32_t n, int32_t stride,
                              float* rows, uint32_t* /*ids*/, hipStream_t st) {
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
    hipLaunchKernelGGL(k_set_counters, dim3(1), dim3(64), 0, st, ws.counters, 0u, 0u);
    hipLaunchKernelGGL(k_set_counters, dim3(1), dim3(64), 0, st, ws.counters + 2, 0u, 0u);
    hipLaunchKernelGGL(k_query_prep, dim3(Q), dim3(256), 0, st, ix, q, ws);
    return hipGetLastError();
}

hipError_t launch_lb_eapca(const IndexView& ix, int32_t Q, const QueryWs& ws, hipStream_t st) {
    hipLaunchKernelGGL(k_lb_eapca, dim3((unsigned)((ix.L + 255) / 256), Q), dim3(256), 0, st, ix, ws);
    return hipGetLastError();
}

hipError_t launch_seed_select(const IndexView& ix, int32_t Q, int32_t l_max, const QueryWs& ws, hipStream_t st) {
    const int lm = (int)(l_max < ix.L ? l_max : ix.L);
    if (lm > 0) hipLaunchKernelGGL(k_seed_select, dim3(Q), dim3(256), 0, st, ix, lm, ws);
    hipLaunchKernelGGL(k_set_counters, dim3(1), dim3(64), 0, st, ws.counters, (uint32_t)(Q * lm), 0u);
    return hipGetLastError();
}

hipError_t launch_emit_main(const IndexView& ix, int32_t Q, bool redo_only, const QueryWs& ws, hipStream_t st) {
    if (redo_only) {
        hipLaunchKernelGGL(k_arm_redo, dim3((Q + 255) / 256), dim3(256), 0, st, ws, Q);
    } else {
        hipLaunchKernelGGL(k_set_counters, dim3(1), dim3(64), 0, st, ws.counters, 0u, 0u);
    }
    hipLaunchKernelGGL(k_emit_main, dim3((unsigned)((ix.L + 255) / 256), Q), dim3(256), 0, st, ix,
                       redo_only ? 1 : 0, ws);
    return hipGetLastError();
}

size_t scan_lds_bytes(const IndexView& ix) { return sizeof(float) * ((size_t)ix.stride + (size_t)ix.w * kCard); }

hipError_t launch_leaf_scan(const IndexView& ix, const ScanParams& sp, const QueryWs& ws, int device_cus,
                            hipStream_t st) {
    const size_t lds = scan_lds_bytes(ix);
    int per_cu = (int)((160 * 1024) / (lds + sizeof(ScanShared) + 1024));
    if (per_cu > 8) per_cu = 8;
    if (per_cu < 1) per_cu = 1;
    hipLaunchKernelGGL(k_leaf_scan, dim3(device_cus * per_cu), dim3(kTile), lds, st, ix, sp, ws);
    return hipGetLastError();
}

hipError_t launch_merge(const IndexView& ix, const ScanParams& sp, bool redo_only, const QueryWs& ws,
                        int64_t* ids_out, float* d2_out, hs_query_stats* stats_out, hipStream_t st) {
    hipLaunchKernelGGL(k_merge, dim3(sp.Q), dim3(1024), sizeof(unsigned long long) * ws.P, st, ix, sp,
                       redo_only ? 1 : 0, ws, ids_out, d2_out, stats_out);
    return hipGetLastError();
}

hipError_t launch_reset_counters(const QueryWs& ws, hipStream_t st) {
    hipLaunchKernelGGL(k_set_counters, dim3(1), dim3(64), 0, st, ws.counters, 0u, 0u);
    return hipGetLastError();
}

}  // namespace hs
