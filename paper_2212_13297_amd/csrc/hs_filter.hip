// The two-stage scan (Hercules Sec. 3.3, steps 3 and 4):
//   filter  LB_SAX of the series of every (query, part) item; survivors are
//           appended to a candidate list
//   refine  exact float32 distance with early abandoning for every candidate,
//           re-checked against the current BSF_k first; block-local top-k,
//           BSF_k published with atomicMin, results appended to the pool
//
// Both kernels are written so that wavefronts never wait for each other on
// the hot path: workgroup barriers happen only when the filter switches to
// another query's LB_SAX table and around the refine kernel's per-step
// top-k merge.  Work is split into contiguous static ranges per workgroup
// and the candidate list into kRegions regions with a counter each, so no
// address is the target of atomics from every workgroup.
#include "hs_device.h"

namespace hs {
namespace {

constexpr int kSlots = kPartRows / (kChunkRows * (kTile / 64));  // chunks per wave per item (8)

__device__ __forceinline__ int64_t item_count(const QueryWs& ws) {
    return min((int64_t)ws.counters[kCtrItems], ws.item_cap);
}

// ------------------------------------------------------------------ filter
//
// Wave `wave` owns chunks wave + 4 s (s = 0..7) of the item's part: lane l
// handles series pb + 64 (wave + 4 s) + l.  First the chunks' LB_EAPCA
// (float32 over outward-rounded intervals, summed over L = pow2 >= w lanes;
// the butterfly leaves every lane of a group the same value) decides which
// chunks are read at all; then the words of the live chunks are loaded
// together and each lane evaluates LB_SAX of its series; the wave's
// survivors are appended with one reservation.
template <int W16>
__global__ void __launch_bounds__(256) k_filter(IndexView ix, ScanParams sp, QueryWs ws) {
    extern __shared__ float s_lut[];  // [w][256]
    __shared__ float4 s_qst[64];      // query segment mean / std intervals
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int region = (blockIdx.x * (kTile / 64) + wave) % kRegions;
    const float lseg = (float)(ix.n / ix.w);
    int L = 1;
    while (L < ix.w) L <<= 1;
    const int cpp = 64 / L;  // chunk envelopes tested per pass
    const uint64_t lt_mask = (1ull << lane) - 1ull;
    int64_t i0, i1;
    block_range(item_count(ws), i0, i1);
    int cur_q = -1;
    unsigned long long a_filt = 0, a_cand = 0, a_tests = 0;  // this wave's counters of cur_q
    for (int64_t idx = i0; idx < i1; ++idx) {
        const uint64_t item = ws.items[idx];
        const int q = (int)(item >> 32);
        const int64_t p = (int64_t)(uint32_t)item;
        if (q != cur_q) {
            if (lane == 0 && cur_q >= 0) {
                atomicAdd(&ws.stats[(int64_t)cur_q * 8 + 1], a_filt);
                atomicAdd(&ws.stats[(int64_t)cur_q * 8 + 6], a_cand);
                atomicAdd(&ws.stats[(int64_t)cur_q * 8 + 7], a_tests);
            }
            a_filt = a_cand = a_tests = 0;
            __syncthreads();  // no wave still reads the previous table
            for (int j = t; j < ix.w * kCard; j += blockDim.x) s_lut[j] = ws.lut[(int64_t)q * ix.w * kCard + j];
            if (t < ix.w) s_qst[t] = ws.qst32[(int64_t)q * ix.w + t];
            cur_q = q;
            __syncthreads();
        }
        const bool skip = (ws.flags[q] & kFlagSkipSax) != 0;
        const double thr = prune_limit(bits_to_float(ws.bsf[q]));
        const int64_t pb = ix.part_start[p], pe = ix.part_start[p + 1];
        const int64_t c0 = ix.part_chunk[p];
        const int nch = (int)((pe - pb + kChunkRows - 1) / kChunkRows);

        // 1. chunk envelopes
        uint32_t live = 0;
        if (skip) {
            live = 0xffu;
        } else {
            for (int sb = 0; sb < kSlots; sb += cpp) {
                const int s = sb + lane / L, seg = lane % L;
                const int ch = wave + (kTile / 64) * s;
                const bool valid = s < kSlots && ch < nch;
                float term = 0.0f;
                if (valid && seg < ix.w) {
                    const float4 e = ix.cenv[(c0 + ch) * ix.w + seg];
                    const float4 qs = s_qst[seg];
                    const float gm = fmaxf(0.0f, fmaxf(e.x - qs.y, qs.x - e.y));
                    const float gs = fmaxf(0.0f, fmaxf(e.z - qs.w, qs.z - e.w));
                    term = lseg * (gm * gm + gs * gs);
                }
                for (int o = L >> 1; o > 0; o >>= 1) term += __shfl_xor(term, o, 64);
                const uint64_t tested = __ballot(valid && seg == 0);
                const uint64_t ok = __ballot(valid && seg == 0 && (double)term <= thr);
                a_tests += (unsigned long long)__popcll(tested);
                for (int i = 0; i < cpp && sb + i < kSlots; ++i)
                    if ((ok >> (i * L)) & 1ull) live |= 1u << (sb + i);
            }
        }

        // 2. words of the live chunks, all loads in flight together
        uint4 v[kSlots][W16];
#pragma unroll
        for (int s = 0; s < kSlots; ++s) {
            const int64_t r = pb + (int64_t)(wave + (kTile / 64) * s) * kChunkRows + lane;
            if (!skip && ((live >> s) & 1u) && r < pe) load_word<W16>(ix.words + r * ix.wstride, v[s]);
        }

        // 3. LB_SAX and the wave's survivors
        float lbv[kSlots];
        uint32_t mask = 0;
        unsigned evaluated = 0;
#pragma unroll
        for (int s = 0; s < kSlots; ++s) {
            const int64_t r0 = pb + (int64_t)(wave + (kTile / 64) * s) * kChunkRows;
            const int64_t r = r0 + lane;
            lbv[s] = 0.0f;
            if ((live >> s) & 1u) {
                if (r0 < pe) evaluated += (unsigned)min((int64_t)kChunkRows, pe - r0);
                if (r < pe) {
                    if (!skip) lbv[s] = lb_sax_word<W16>(v[s], s_lut, ix.w);
                    if ((double)lbv[s] <= thr) mask |= 1u << s;
                }
            }
        }
        uint64_t bal[kSlots];
        int total = 0;
#pragma unroll
        for (int s = 0; s < kSlots; ++s) {
            bal[s] = __ballot((mask >> s) & 1u);
            total += __popcll(bal[s]);
        }
        if (!skip) a_filt += evaluated;
        if (total > 0) {
            long long base = -1;
            if (lane == 0) {
                // once a region is full no more ranges are reserved in it, so
                // its 32-bit counter overshoots the capacity by at most one
                // range per wavefront mapped to it
                uint32_t* cnt = &ws.cand_cnt[region];
                if ((int64_t)load_relaxed(cnt) >= ws.cand_cap) {
                    atomicOr(&ws.flags[q], kFlagCandLost);
                } else {
                    const uint32_t b = atomicAdd(cnt, (uint32_t)total);
                    if ((int64_t)b + total <= ws.cand_cap) {
                        base = (long long)region * ws.cand_cap + b;
                    } else {
                        // this range is never written; the refine kernel stops below it
                        atomicMin(&ws.cand_end[region], b);
                        atomicOr(&ws.flags[q], kFlagCandLost);
                    }
                }
            }
            base = __shfl(base, 0, 64);
            if (base >= 0) {
                a_cand += (unsigned long long)total;
                long long off = base;
#pragma unroll
                for (int s = 0; s < kSlots; ++s) {
                    if ((mask >> s) & 1u) {
                        const long long slot = off + __popcll(bal[s] & lt_mask);
                        ws.cand_pos[slot] = (uint32_t)(pb + (int64_t)(wave + (kTile / 64) * s) * kChunkRows + lane);
                        ws.cand_q[slot] = (uint32_t)q;
                        ws.cand_lb[slot] = lbv[s];
                    }
                    off += __popcll(bal[s]);
                }
            }
        }
    }
    if (lane == 0 && cur_q >= 0) {
        atomicAdd(&ws.stats[(int64_t)cur_q * 8 + 1], a_filt);
        atomicAdd(&ws.stats[(int64_t)cur_q * 8 + 6], a_cand);
        atomicAdd(&ws.stats[(int64_t)cur_q * 8 + 7], a_tests);
    }
}

// ------------------------------------------------------------------ refine
//
// A workgroup step takes kGrab consecutive candidates; each 16-lane group
// refines 4 of them together: the first two chunks of all 4 series are
// loaded at once, the sums checked against BSF_k, and the next two chunks
// loaded for the series still alive.  Admitted results go to a block-local
// top-k of the current query, flushed to the pool when the query changes and
// at the end; its k-th distance is published to BSF_k at once.

constexpr int kPerGroup = 4;
constexpr int kGrab = (kTile / 16) * kPerGroup;  // 64

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
    const int gbase = lane & ~15;
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
        // lanes 0..3 of a group fetch the group's candidates and their BSF_k
        int mq = -1;
        uint32_t mpos = 0;
        float mlb = 0.0f, mthr = 0.0f;
        if (sub < kPerGroup) {
            const long long c = g * kGrab + grp * kPerGroup + sub;
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
                if (mq == s_curq) mthr = fminf(mthr, s_lk);
            }
        }
        // group-uniform copies: the 16 lanes of a group take every branch together
        int q[kPerGroup];
        uint32_t pos[kPerGroup];
        float thr[kPerGroup], d[kPerGroup];
        bool alive[kPerGroup], refined[kPerGroup];
        unsigned chunks[kPerGroup];
#pragma unroll
        for (int j = 0; j < kPerGroup; ++j) {
            q[j] = __shfl(mq, gbase + j, 64);
            pos[j] = __shfl(mpos, gbase + j, 64);
            const float lb = __shfl(mlb, gbase + j, 64);
            thr[j] = __shfl(mthr, gbase + j, 64);
            refined[j] = q[j] >= 0 && (double)lb <= prune_limit(thr[j]);
            alive[j] = refined[j];
            d[j] = 0.0f;
            chunks[j] = 0;
        }
        for (int c = 0; c < nchunks; c += 2) {
            const bool two = c + 1 < nchunks;
            float4 xa[kPerGroup], xb[kPerGroup];
#pragma unroll
            for (int j = 0; j < kPerGroup; ++j) {
                if (alive[j]) {
                    const float* xr = ix.rows + (int64_t)pos[j] * ix.stride + sub * 4 + c * kChunk;
                    xa[j] = *reinterpret_cast<const float4*>(xr);
                    xb[j] = two ? *reinterpret_cast<const float4*>(xr + kChunk) : make_float4(0.f, 0.f, 0.f, 0.f);
                }
            }
#pragma unroll
            for (int j = 0; j < kPerGroup; ++j) {
                if (alive[j]) {
                    const float* qr = ws.qrow + (int64_t)q[j] * ix.stride + sub * 4 + c * kChunk;
                    d[j] += chunk_partial(*reinterpret_cast<const float4*>(qr), xa[j]);
                    if (two) d[j] += chunk_partial(*reinterpret_cast<const float4*>(qr + kChunk), xb[j]);
                    chunks[j] += two ? 2u : 1u;
                    if (d[j] > thr[j]) alive[j] = false;
                }
            }
        }
        if (sub == 0) {
#pragma unroll
            for (int j = 0; j < kPerGroup; ++j) {
                if (refined[j] && alive[j]) {
                    const int slot = atomicAdd(&s_nres, 1);
                    s_res[slot] = ((unsigned long long)__float_as_uint(d[j]) << 32) | ix.ids[pos[j]];
                    s_resq[slot] = q[j];
                }
                s_cq[grp * kPerGroup + j] = q[j];
                s_cch[grp * kPerGroup + j] = refined[j] ? chunks[j] : 0u;
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

}  // namespace

hipError_t launch_filter(const IndexView& ix, const ScanParams& sp, const QueryWs& ws, int device_cus,
                         hipStream_t st) {
    const size_t lds = sizeof(float) * (size_t)ix.w * kCard;
    HS_LAUNCH_RESIDENT(ix, k_filter, lds, device_cus, st, ix, sp, ws);
    return hipGetLastError();
}

hipError_t launch_refine(const IndexView& ix, const ScanParams& sp, const QueryWs& ws, int device_cus,
                         hipStream_t st) {
    hipLaunchKernelGGL(k_refine, dim3(resident_grid(k_refine, kTile, 0, device_cus)), dim3(kTile), 0, st, ix, sp,
                       ws);
    return hipGetLastError();
}

}  // namespace hs
