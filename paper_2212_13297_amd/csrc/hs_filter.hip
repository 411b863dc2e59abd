// The LB_SAX filter (Hercules Sec. 3.3, step 3): the series of every
// (query, part) item whose bounds do not exceed BSF_k are appended to a
// candidate list for the refine kernel.
//
// Wavefronts never wait for each other on the hot path: workgroup barriers
// happen only when a workgroup switches to another query's LB_SAX table.
// Work is split into contiguous static ranges per workgroup, and the
// candidate list into kRegions regions with a counter each.
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
            // a query's candidates go to region q mod kRegions: long runs of one
            // query for the refine kernel, and few wavefronts per counter
            const int region = q % kRegions;
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

}  // namespace

hipError_t launch_filter(const IndexView& ix, const ScanParams& sp, const QueryWs& ws, int device_cus,
                         hipStream_t st) {
    const size_t lds = sizeof(float) * (size_t)ix.w * kCard;
    HS_LAUNCH_RESIDENT(ix, k_filter, lds, device_cus, st, ix, sp, ws);
    return hipGetLastError();
}

}  // namespace hs
