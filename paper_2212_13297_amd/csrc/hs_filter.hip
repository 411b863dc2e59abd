// The LB_SAX filter (Hercules Sec. 3.4, step 3): the series of every
// (query, part) item whose bounds do not exceed BSF_k become candidates for
// the refine kernel.
//
// Every wavefront appends to a private slice of the candidate buffer with a
// counter in a register (no atomics), and wavefronts never wait for each
// other except when their workgroup switches to another query's LB_SAX table
// (items are ordered by query and each workgroup takes a contiguous range).
// After the filter, slice_prefix computes where each slice starts in the
// candidate list, the slices' concatenation, which the refine kernel reads
// in place.
#include "hs_device.h"

namespace hs {
namespace {

constexpr int kWaves = kTile / 64;                 // wavefronts per workgroup
constexpr int kSlots = 8;                          // chunks per wavefront per round
constexpr int kRoundSpan = kSlots * kWaves;        // chunks per round (2048 series)

__device__ __forceinline__ int64_t item_count(const QueryWs& ws) {
    return min((int64_t)ws.counters[kCtrItems], ws.item_cap);
}

// Envelope passes per round: a pass tests 64 / L chunks (L = pow2 >= w lanes each).
template <int W16>
constexpr int max_passes() {
    return W16 == 1 ? 2 : (W16 == 2 ? 4 : 8);
}

// Load the chunk envelopes a wave tests in round rb (one float4 per lane and pass).
template <int W16>
__device__ __forceinline__ void load_cenv(const IndexView& ix, int64_t c0, int nch, int rb, int wave, int lane,
                                          int L, int cpp, float4 (&ce)[max_passes<W16>()]) {
#pragma unroll
    for (int i = 0; i < max_passes<W16>(); ++i) {
        const int s = i * cpp + lane / L, seg = lane % L;
        const int ch = rb + wave + kWaves * s;
        ce[i] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (i * cpp < kSlots && s < kSlots && ch < nch && seg < ix.w) ce[i] = ix.cenv[(c0 + ch) * ix.w + seg];
    }
}

// A part is processed in rounds of kRoundSpan chunks; in a round, wave
// `wave` owns chunks rb + wave + 4 s (s = 0..7): lane l handles the series
// 64 chunk + l.  First the chunks' LB_EAPCA (float32 over outward-rounded
// intervals, summed over L = pow2 >= w lanes; the butterfly leaves every lane
// of a group the same value) decides which chunks are read at all; then the
// words of the live chunks are loaded together and each lane evaluates
// LB_SAX of its series.
template <int W16>
__global__ void __launch_bounds__(256) k_filter(IndexView ix, ScanParams sp, QueryWs ws) {
    extern __shared__ float s_lut[];  // [16 W16][256], rows beyond w zero
    __shared__ float4 s_qst[64];      // query segment mean / std intervals
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const float lseg = (float)(ix.n / ix.w);
    int L = 1;
    while (L < ix.w) L <<= 1;
    const int cpp = 64 / L;  // chunk envelopes tested per pass
    const uint64_t lt_mask = (1ull << lane) - 1ull;
    const int64_t slice = (int64_t)blockIdx.x * kWaves + wave;
    uint32_t* spos = ws.slice_pos + slice * ws.slice_cap;
    uint32_t* sq = ws.slice_q + slice * ws.slice_cap;
    float* slb = ws.slice_lb + slice * ws.slice_cap;
    uint32_t cnt = 0;  // entries in this wave's slice (uniform)
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
            load_lut<W16>(s_lut, ws.lut + (int64_t)q * ix.w * kCard, ix.w, t, blockDim.x);
            if (t < ix.w) s_qst[t] = ws.qst32[(int64_t)q * ix.w + t];
            cur_q = q;
            __syncthreads();
        }
        const bool skip = (ws.flags[q] & kFlagSkipSax) != 0;
        const double thr = prune_limit(bits_to_float(ws.bsf[q]));
        const int64_t pb = ix.part_start[p], pe = ix.part_start[p + 1];
        const int64_t c0 = ix.part_chunk[p];
        const int nch = (int)((pe - pb + kChunkRows - 1) / kChunkRows);
        bool lost = false;
        float4 ce[max_passes<W16>()];
        if (!skip) load_cenv<W16>(ix, c0, nch, 0, wave, lane, L, cpp, ce);
        for (int rb = 0; rb < nch; rb += kRoundSpan) {
            // 1. chunk envelopes (loaded during the previous round)
            uint32_t live = 0;
            if (skip) {
                live = 0xffu;
            } else {
#pragma unroll
                for (int i = 0; i < max_passes<W16>(); ++i) {
                    const int sb = i * cpp;
                    if (sb >= kSlots) break;
                    const int s = sb + lane / L, seg = lane % L;
                    const int ch = rb + wave + kWaves * s;
                    const bool valid = s < kSlots && ch < nch;
                    float term = 0.0f;
                    if (valid && seg < ix.w) {
                        const float4 e = ce[i];
                        const float4 qs = s_qst[seg];
                        const float gm = fmaxf(0.0f, fmaxf(e.x - qs.y, qs.x - e.y));
                        const float gs = fmaxf(0.0f, fmaxf(e.z - qs.w, qs.z - e.w));
                        term = lseg * (gm * gm + gs * gs);
                    }
                    for (int o = L >> 1; o > 0; o >>= 1) term += __shfl_xor(term, o, 64);
                    const uint64_t tested = __ballot(valid && seg == 0);
                    const uint64_t ok = __ballot(valid && seg == 0 && (double)term <= thr);
                    a_tests += (unsigned long long)__popcll(tested);
                    for (int j = 0; j < cpp && sb + j < kSlots; ++j)
                        if ((ok >> (j * L)) & 1ull) live |= 1u << (sb + j);
                }
            }

            // 2. words of the live chunks, all loads in flight together, and
            //    the next round's envelopes behind them
            uint4 v[kSlots][W16];
#pragma unroll
            for (int s = 0; s < kSlots; ++s) {
                const int64_t r = pb + (int64_t)(rb + wave + kWaves * s) * kChunkRows + lane;
                if (!skip && ((live >> s) & 1u) && r < pe) load_word<W16>(ix.words + r * ix.wstride, v[s]);
            }
            if (!skip && rb + kRoundSpan < nch) load_cenv<W16>(ix, c0, nch, rb + kRoundSpan, wave, lane, L, cpp, ce);

            // 3. LB_SAX and the wave's survivors
            float lbv[kSlots];
            uint32_t mask = 0;
            unsigned evaluated = 0;
#pragma unroll
            for (int s = 0; s < kSlots; ++s) {
                const int64_t r0 = pb + (int64_t)(rb + wave + kWaves * s) * kChunkRows;
                const int64_t r = r0 + lane;
                lbv[s] = 0.0f;
                if ((live >> s) & 1u) {
                    if (r0 < pe) evaluated += (unsigned)min((int64_t)kChunkRows, pe - r0);
                    if (r < pe) {
                        if (!skip) lbv[s] = lb_sax_word<W16>(v[s], s_lut);
                        if ((double)lbv[s] <= thr) mask |= 1u << s;
                    }
                }
            }
            if (!skip) a_filt += evaluated;
            uint32_t total = 0;
#pragma unroll
            for (int s = 0; s < kSlots; ++s) total += (uint32_t)__popcll(__ballot((mask >> s) & 1u));
            if (total == 0) continue;
            uint32_t* dpos = spos;
            uint32_t* dq = sq;
            float* dlb = slb;
            uint32_t off = cnt;
            const bool own = (int64_t)cnt + total <= ws.slice_cap;
            if (!own) {
                // the private slice is full: reserve a range of the shared
                // overflow slice; once that is full too, the query takes the
                // fallback path.  Reservations stop at capacity, so the 32-bit
                // counter overshoots it by at most one range per wavefront.
                long long b = -1;
                if (lane == 0) {
                    uint32_t* oc = &ws.counters[kCtrOvf];
                    if ((int64_t)load_relaxed(oc) < ws.ovf_cap) {
                        const uint32_t r = atomicAdd(oc, total);
                        if ((int64_t)r + total <= ws.ovf_cap) b = r;
                        else atomicMin(&ws.counters[kCtrOvfEnd], r);  // never written: the list stops below it
                    }
                }
                b = __shfl(b, 0, 64);
                if (b < 0) {
                    lost = true;
                    continue;
                }
                const int64_t ob = (int64_t)ws.n_slices * ws.slice_cap;
                dpos = ws.slice_pos + ob;
                dq = ws.slice_q + ob;
                dlb = ws.slice_lb + ob;
                off = (uint32_t)b;
            }
#pragma unroll
            for (int s = 0; s < kSlots; ++s) {
                const uint64_t bal = __ballot((mask >> s) & 1u);
                if ((mask >> s) & 1u) {
                    const uint32_t slot = off + (uint32_t)__popcll(bal & lt_mask);
                    dpos[slot] = (uint32_t)(pb + (int64_t)(rb + wave + kWaves * s) * kChunkRows + lane);
                    dq[slot] = (uint32_t)q;
                    dlb[slot] = lbv[s];
                }
                off += (uint32_t)__popcll(bal);
            }
            if (own) cnt += total;
            a_cand += total;
        }
        if (lost && lane == 0) atomicOr(&ws.flags[q], kFlagCandLost);
    }
    if (lane == 0) {
        ws.slice_cnt[slice] = cnt;
        if (cur_q >= 0) {
            atomicAdd(&ws.stats[(int64_t)cur_q * 8 + 1], a_filt);
            atomicAdd(&ws.stats[(int64_t)cur_q * 8 + 6], a_cand);
            atomicAdd(&ws.stats[(int64_t)cur_q * 8 + 7], a_tests);
        }
    }
}

// Exclusive prefix of the slice counts (one workgroup); the total goes to
// counters[kCtrCand].
__global__ void __launch_bounds__(1024) k_slice_prefix(QueryWs ws) {
    __shared__ uint32_t s_part[1024];
    const int t = threadIdx.x, n = ws.n_slices + 1;  // the private slices and the overflow slice
    if (t == 0) {
        // every overflow entry below min(counter, first range that did not fit) was written
        const int64_t c = min(min((int64_t)ws.counters[kCtrOvf], (int64_t)ws.counters[kCtrOvfEnd]), ws.ovf_cap);
        ws.slice_cnt[ws.n_slices] = (uint32_t)c;
    }
    __syncthreads();
    const int per = (n + 1023) / 1024;
    const int a = min(n, t * per), b = min(n, a + per);
    uint32_t sum = 0;
    for (int i = a; i < b; ++i) sum += ws.slice_cnt[i];
    s_part[t] = sum;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {  // inclusive Hillis-Steele scan
        const uint32_t v = t >= o ? s_part[t - o] : 0u;
        __syncthreads();
        s_part[t] += v;
        __syncthreads();
    }
    uint32_t run = s_part[t] - sum;
    for (int i = a; i < b; ++i) {
        ws.slice_start[i] = run;
        run += ws.slice_cnt[i];
    }
    if (t == 1023) {
        ws.slice_start[n] = s_part[1023];
        ws.counters[kCtrCand] = s_part[1023];
    }
}

template <int W16>
int filter_blocks(const IndexView& ix, int cus) {
    return resident_grid(k_filter<W16>, kTile, sizeof(float) * (size_t)lut_floats<W16>(), cus);
}

}  // namespace

int filter_waves(const IndexView& ix, int device_cus) {
    int blocks = 1;
    switch (w16_of(ix)) {
        case 1: blocks = filter_blocks<1>(ix, device_cus); break;
        case 2: blocks = filter_blocks<2>(ix, device_cus); break;
        case 3: blocks = filter_blocks<3>(ix, device_cus); break;
        default: blocks = filter_blocks<4>(ix, device_cus); break;
    }
    return blocks * kWaves;
}

hipError_t launch_filter(const IndexView& ix, const ScanParams& sp, const QueryWs& ws, int device_cus,
                         hipStream_t st) {
    const size_t lds = sizeof(float) * (size_t)16 * w16_of(ix) * kCard;
    const dim3 grid(ws.n_slices / kWaves);  // one slice per wavefront
    HS_DISPATCH_W16(ix, k_filter, grid, dim3(kTile), lds, st, ix, sp, ws);
    return hipGetLastError();
}

hipError_t launch_slice_prefix(const QueryWs& ws, hipStream_t st) {
    hipLaunchKernelGGL(k_slice_prefix, dim3(1), dim3(1024), 0, st, ws);
    return hipGetLastError();
}

}  // namespace hs
