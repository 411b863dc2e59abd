// The scan kernels (Hercules Sec. 3.3, steps 3 and 4):
//   filter     LB_SAX of every series of every (query, part) item; the
//              survivors are appended to a candidate list (block-wide scan
//              compaction, one reservation per item)
//   refine     exact float32 distance with early abandoning for every
//              candidate, re-checked against the current BSF_k first;
//              block-local top-k, BSF_k published with atomicMin, results
//              appended to the per-query pool
//   leaf_scan  filter + refine fused per item, without a candidate list: the
//              path of queries whose candidate list or pool overflowed
//
// Work is split into contiguous static ranges per workgroup (items are
// ordered by query, so a workgroup reloads the LB_SAX table rarely), and the
// candidate list into kRegions regions with a counter each: no address is the
// target of atomics from every workgroup.
#include "hs_device.h"

namespace hs {
namespace {

constexpr int kRowsPerThread = kPartRows / kTile;

__device__ __forceinline__ int64_t item_count(const QueryWs& ws) {
    return min((int64_t)ws.counters[kCtrItems], ws.item_cap);
}

// ------------------------------------------------------------------ filter

// Each wavefront owns, at step j of an item, the 64 consecutive series
// pb + 256 j + 64 wave + lane: exactly one chunk.  The chunk's LB_EAPCA
// (float32 over outward-rounded intervals, a wave-wide sum, so the decision
// is wave-uniform) is tested first; the iSAX words of a pruned chunk are
// never read.
template <int W16>
__global__ void __launch_bounds__(256) k_filter(IndexView ix, ScanParams sp, QueryWs ws) {
    extern __shared__ float s_lut[];  // [w][256]
    __shared__ float4 s_qst[64];      // query segment mean / std intervals
    __shared__ long long s_base;
    __shared__ int s_w[4];
    __shared__ unsigned int s_eval, s_tests;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int region = blockIdx.x % kRegions;
    const float lseg = (float)(ix.n / ix.w);
    int64_t i0, i1;
    block_range(item_count(ws), i0, i1);
    int cur_q = -1;
    unsigned long long acc_filt = 0, acc_cand = 0, acc_tests = 0;  // thread 0: counters of cur_q
    if (t == 0) {
        s_eval = 0;
        s_tests = 0;
    }
    for (int64_t idx = i0; idx < i1; ++idx) {
        const uint64_t item = ws.items[idx];
        const int q = (int)(item >> 32);
        const int64_t p = (int64_t)(uint32_t)item;
        if (q != cur_q) {
            if (t == 0 && cur_q >= 0) {
                atomicAdd(&ws.stats[(int64_t)cur_q * 8 + 1], acc_filt);
                atomicAdd(&ws.stats[(int64_t)cur_q * 8 + 6], acc_cand);
                atomicAdd(&ws.stats[(int64_t)cur_q * 8 + 7], acc_tests);
            }
            acc_filt = acc_cand = acc_tests = 0;
            for (int j = t; j < ix.w * kCard; j += blockDim.x) s_lut[j] = ws.lut[(int64_t)q * ix.w * kCard + j];
            if (t < ix.w) s_qst[t] = ws.qst32[(int64_t)q * ix.w + t];
            cur_q = q;
            __syncthreads();
        }
        const bool skip = (ws.flags[q] & kFlagSkipSax) != 0;
        const double thr = prune_limit(bits_to_float(ws.bsf[q]));
        const int64_t pb = ix.part_start[p], pe = ix.part_start[p + 1];
        uint32_t live = skip ? 0xffu : 0u;
        unsigned my_eval = 0, my_tests = 0;
        if (!skip) {
            const int64_t c0 = ix.part_chunk[p];
#pragma unroll
            for (int j = 0; j < kRowsPerThread; ++j) {
                const int64_t r0 = pb + j * kTile + wave * kChunkRows;
                if (r0 < pe) {
                    float term = 0.0f;
                    if (lane < ix.w) {
                        const float4 e = ix.cenv[(c0 + j * (kTile / kChunkRows) + wave) * ix.w + lane];
                        const float4 s = s_qst[lane];
                        const float gm = fmaxf(0.0f, fmaxf(e.x - s.y, s.x - e.y));
                        const float gs = fmaxf(0.0f, fmaxf(e.z - s.w, s.z - e.w));
                        term = lseg * (gm * gm + gs * gs);
                    }
#pragma unroll
                    for (int o = 32; o > 0; o >>= 1) term += __shfl_xor(term, o, 64);
                    ++my_tests;
                    if ((double)term <= thr) {
                        live |= 1u << j;
                        my_eval += (unsigned)min((int64_t)kChunkRows, pe - r0);
                    }
                }
            }
            if (lane == 0) {
                atomicAdd(&s_eval, my_eval);
                atomicAdd(&s_tests, my_tests);
            }
        }
        uint4 v[kRowsPerThread][W16];
#pragma unroll
        for (int j = 0; j < kRowsPerThread; ++j) {
            const int64_t r = pb + t + j * kTile;
            if (!skip && ((live >> j) & 1u) && r < pe) load_word<W16>(ix.words + r * ix.wstride, v[j]);
        }
        float lbv[kRowsPerThread];
        uint32_t mask = 0;
#pragma unroll
        for (int j = 0; j < kRowsPerThread; ++j) {
            const int64_t r = pb + t + j * kTile;
            lbv[j] = 0.0f;
            if (((live >> j) & 1u) && r < pe) {
                if (!skip) lbv[j] = lb_sax_word<W16>(v[j], s_lut, ix.w);
                if ((double)lbv[j] <= thr) mask |= 1u << j;
            }
        }
        int total;
        const int off = block_exclusive_scan(__popc(mask), s_w, &total);
        if (t == 0) {
            long long base = -1;
            if (total > 0) {
                // once a region is full no more ranges are reserved in it, so
                // its 32-bit counter overshoots the capacity by at most one
                // range per workgroup mapped to it
                uint32_t* cnt = &ws.cand_cnt[region];
                if ((int64_t)load_relaxed(cnt) >= ws.cand_cap) {
                    atomicOr(&ws.flags[q], kFlagCandLost);
                } else {
                    const uint32_t b = atomicAdd(cnt, (uint32_t)total);
                    if ((int64_t)b + total <= ws.cand_cap) {
                        base = (long long)region * ws.cand_cap + b;
                        acc_cand += (unsigned long long)total;
                    } else {
                        // this range is never written; the refine kernel stops below it
                        atomicMin(&ws.cand_end[region], b);
                        atomicOr(&ws.flags[q], kFlagCandLost);
                    }
                }
            }
            s_base = base;
            // s_eval / s_tests were complete at the scan's barriers
            acc_filt += s_eval;
            acc_tests += s_tests;
            s_eval = 0;
            s_tests = 0;
        }
        __syncthreads();
        const long long base = s_base;
        if (base >= 0) {
            int o = off;
#pragma unroll
            for (int j = 0; j < kRowsPerThread; ++j) {
                if (mask & (1u << j)) {
                    const int64_t slot = base + o;
                    ws.cand_pos[slot] = (uint32_t)(pb + t + j * kTile);
                    ws.cand_q[slot] = (uint32_t)q;
                    ws.cand_lb[slot] = lbv[j];
                    ++o;
                }
            }
        }
        __syncthreads();
    }
    if (t == 0 && cur_q >= 0) {
        atomicAdd(&ws.stats[(int64_t)cur_q * 8 + 1], acc_filt);
        atomicAdd(&ws.stats[(int64_t)cur_q * 8 + 6], acc_cand);
        atomicAdd(&ws.stats[(int64_t)cur_q * 8 + 7], acc_tests);
    }
}

// ------------------------------------------------------------------ refine

constexpr int kGrab = 64;  // candidates per workgroup step: 16 groups x 4

__global__ void __launch_bounds__(256) k_refine(IndexView ix, ScanParams sp, QueryWs ws) {
    __shared__ unsigned long long s_top[HS_KMAX];
    __shared__ unsigned long long s_res[kGrab];
    __shared__ int s_resq[kGrab];
    __shared__ int s_cq[kGrab];        // query of each candidate of the step (-1: none)
    __shared__ uint32_t s_cch[kGrab];  // chunks read for it (0: not refined)
    __shared__ long long s_start[kRegions + 1];
    __shared__ int s_nres, s_topn, s_curq;
    __shared__ float s_lk;  // k-th distance of the block's top-k of s_curq (inf until full)
    const int t = threadIdx.x, lane = t & 63, sub = t & 15, grp = t >> 4;
    const int k = sp.k;
    const int nchunks = ix.stride / kChunk;
    if (t == 0) {
        // every entry of a region below min(counter, first range that did not fit) was written
        long long acc = 0;
        for (int r = 0; r < kRegions; ++r) {
            s_start[r] = acc;
            acc += min(min((long long)ws.cand_cnt[r], (long long)ws.cand_end[r]), (long long)ws.cand_cap);
        }
        s_start[kRegions] = acc;
        s_nres = 0;
        s_topn = 0;
        s_curq = -1;
        s_lk = INFINITY;
    }
    __syncthreads();
    const long long T = s_start[kRegions];
    const long long nsteps = (T + kGrab - 1) / kGrab;
    for (long long g = blockIdx.x; g < nsteps; g += gridDim.x) {
        // lanes 0..3 of a group fetch the group's 4 candidates and their BSF_k
        int mq = -1;
        uint32_t mpos = 0;
        float mlb = 0.0f, mthr = 0.0f;
        if (sub < 4) {
            const long long c = g * kGrab + grp * 4 + sub;
            if (c < T) {
                int lo = 0, hi = kRegions;
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (s_start[mid] <= c) lo = mid; else hi = mid;
                }
                const int64_t slot = (int64_t)lo * ws.cand_cap + (c - s_start[lo]);
                mq = (int)ws.cand_q[slot];
                mpos = ws.cand_pos[slot];
                mlb = ws.cand_lb[slot];
                mthr = bits_to_float(load_relaxed(&ws.bsf[mq]));
            }
        }
        for (int j = 0; j < 4; ++j) {
            // group-uniform values: the 16 lanes leave the chunk loop together
            const int src = (lane & ~15) + j;
            const int q = __shfl(mq, src, 64);
            const uint32_t pos = __shfl(mpos, src, 64);
            const float lb = __shfl(mlb, src, 64);
            float thr = __shfl(mthr, src, 64);
            unsigned chunks = 0;
            if (q >= 0) {
                if (q == s_curq) thr = fminf(thr, s_lk);
                if ((double)lb <= prune_limit(thr)) {
                    bool alive;
                    const float d = refine_row(ix.rows + (int64_t)pos * ix.stride + sub * 4,
                                               ws.qrow + (int64_t)q * ix.stride + sub * 4, nchunks, thr, alive,
                                               chunks);
                    if (sub == 0 && alive) {
                        const int slot = atomicAdd(&s_nres, 1);
                        s_res[slot] = ((unsigned long long)__float_as_uint(d) << 32) | ix.ids[pos];
                        s_resq[slot] = q;
                    }
                }
            }
            if (sub == 0) {
                s_cq[grp * 4 + j] = q;
                s_cch[grp * 4 + j] = chunks;
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
            s_nres = 0;
            s_topn = n;
            s_curq = cq;
            s_lk = INFINITY;
            if (cq >= 0 && n == k) {
                const uint32_t kb = (uint32_t)(s_top[k - 1] >> 32);
                s_lk = bits_to_float(kb);
                if (s_lk < bits_to_float(load_relaxed(&ws.bsf[cq]))) atomicMin(&ws.bsf[cq], kb);
            }
            // counters, one update per run of equal queries
            int rq = -1;
            unsigned long long nref = 0, nch = 0;
            for (int i = 0; i <= kGrab; ++i) {
                const int ci = i < kGrab ? s_cq[i] : -2;
                if (ci != rq) {
                    if (rq >= 0 && nref) {
                        atomicAdd(&ws.stats[(int64_t)rq * 8 + 2], nref);
                        atomicAdd(&ws.stats[(int64_t)rq * 8 + 3], nch);
                    }
                    rq = ci;
                    nref = nch = 0;
                }
                if (i < kGrab && ci >= 0 && s_cch[i]) {
                    ++nref;
                    nch += s_cch[i];
                }
            }
        }
        __syncthreads();
    }
    if (t == 0) flush_topk(ws, s_curq, k, s_top, s_topn);
}

// ------------------------------------------------------- fused fallback

struct ScanShared {
    unsigned long long top[HS_KMAX];
    unsigned long long res[kTile];
    uint32_t hits[kTile];
    int w[4];
    int nres, topn;
    float thr;  // block-uniform pruning threshold (a valid upper bound of BSF_k)
    unsigned int st_filt, st_ref, st_chunks;
};

template <int W16>
__global__ void __launch_bounds__(256) k_leaf_scan(IndexView ix, ScanParams sp, QueryWs ws) {
    extern __shared__ float s_dyn[];
    __shared__ ScanShared sh;
    float* s_q = s_dyn;                // [stride]
    float* s_lut = s_dyn + ix.stride;  // [w][256]
    const int t = threadIdx.x;
    const int grp = t >> 4, sub = t & 15;
    const int nchunks = ix.stride / kChunk;
    const int k = sp.k;
    int64_t i0, i1;
    block_range(item_count(ws), i0, i1);
    int cur_q = -1;

    for (int64_t idx = i0; idx < i1; ++idx) {
        const uint64_t item = ws.items[idx];
        const int q = (int)(item >> 32);
        const int64_t part = (int64_t)(uint32_t)item;
        if (q != cur_q) {
            for (int j = t; j < ix.stride; j += blockDim.x) s_q[j] = ws.qrow[(int64_t)q * ix.stride + j];
            for (int j = t; j < ix.w * kCard; j += blockDim.x) s_lut[j] = ws.lut[(int64_t)q * ix.w * kCard + j];
            cur_q = q;
        }
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
                    if (alive)
                        sh.res[atomicAdd(&sh.nres, 1)] = ((unsigned long long)__float_as_uint(d) << 32) | ix.ids[pos];
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

}  // namespace

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

}  // namespace hs
