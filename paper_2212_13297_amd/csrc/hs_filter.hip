// The LB_SAX filter (Hercules Sec. 3.4, step 3): the series of every
// (query, part) item whose bounds do not exceed BSF_k become candidates for
// the refine kernel.
//
// Every wavefront appends to a private slice of the candidate buffer with a
// counter in a register (no atomics).  Items are ordered by query; workgroups
// take units of consecutive items from a counter and stage them in LDS a
// window at a time (a window holds items of one query); the workgroup's
// wavefronts wait for each other only between windows.  After the filter,
// slice_prefix computes where each slice starts in the candidate list, the
// slices' concatenation, which the refine kernel reads in place.
#include "hs_device.h"

namespace hs {
namespace {

constexpr int kWaves = kTile / 64;  // wavefronts per workgroup
constexpr int kUnit = 8;            // most items per unit of work (and per window)
// Chunks whose words one wavefront loads together, and the kernel's
// occupancy target.  The deviation stage's queue (12 bytes per entry, 64
// (chunks + 1) entries per wavefront) shares the LDS with the LB_SAX table:
// one 16-byte word per series takes 4 chunks at 4 wavefronts per SIMD (about
// 120 registers, 37 KB per workgroup); two words 3 chunks at 3 (50 KB); three
// words 3 chunks at 2 (66 KB); four words fit one workgroup per CU (82 KB).
template <int W16>
constexpr int batch_chunks() {
    return W16 == 1 ? 4 : 3;
}
template <int W16>
constexpr int filter_occupancy() {
    return W16 == 1 ? 4 : (W16 == 2 ? 3 : (W16 == 3 ? 2 : 1));
}
constexpr int kQueue = 128;         // live-chunk queue per wavefront (power of two)

__device__ __forceinline__ int64_t item_count(const QueryWs& ws) {
    return min((int64_t)ws.counters[kCtrItems], ws.item_cap);
}

// Per-wavefront output and counters.
struct FilterOut {
    uint32_t* spos;
    uint32_t* sq;
    uint32_t* spart;
    uint32_t cnt;  // entries in this wavefront's slice (uniform)
    unsigned long long filt, cand, tests, sig;
    bool lost;
};

// Appends the lanes' candidates of NSL rows each (pos[s], pk[s] where bit s of
// mask is set) to the wavefront's private slice, or to a reserved range of
// the shared overflow slice once the private one is full.
template <int NSL>
__device__ __forceinline__ void emit_candidates(const QueryWs& ws, FilterOut& o, int lane, int q, uint32_t mask,
                                                const uint32_t (&pos)[NSL], const uint32_t (&pk)[NSL]) {
    const uint64_t lt_mask = (1ull << lane) - 1ull;
    uint32_t total = 0;
#pragma unroll
    for (int s = 0; s < NSL; ++s) total += (uint32_t)__popcll(__ballot((mask >> s) & 1u));
    if (total == 0) return;
    uint32_t* dpos = o.spos;
    uint32_t* dq = o.sq;
    uint32_t* dpart = o.spart;
    uint32_t off = o.cnt;
    const bool own = (int64_t)o.cnt + total <= ws.slice_cap;
    if (!own) {
        // the private slice is full: reserve a range of the shared overflow
        // slice; once that is full too, the query takes the fallback path.
        // Reservations stop at capacity, so the 32-bit counter overshoots it
        // by at most one range per wavefront.
        long long b = -1;
        if (lane == 0) {
            uint32_t* oc = &ws.counters[kCtrOvf];
            if ((int64_t)load_relaxed(oc) < ws.ovf_cap) {
                const uint32_t rr = atomicAdd(oc, total);
                if ((int64_t)rr + total <= ws.ovf_cap) b = rr;
                else atomicMin(&ws.counters[kCtrOvfEnd], rr);  // never written: the list stops below it
            }
        }
        b = __shfl(b, 0, 64);
        if (b < 0) {
            o.lost = true;
            return;
        }
        const int64_t ob = (int64_t)ws.n_slices * ws.slice_cap;
        dpos = ws.slice_pos + ob;
        dq = ws.slice_q + ob;
        dpart = ws.slice_part + ob;
        off = (uint32_t)b;
    }
#pragma unroll
    for (int s = 0; s < NSL; ++s) {
        const uint64_t bal = __ballot((mask >> s) & 1u);
        if ((mask >> s) & 1u) {
            const uint32_t slot = off + (uint32_t)__popcll(bal & lt_mask);
            dpos[slot] = pos[s];
            dq[slot] = (uint32_t)q;
            dpart[slot] = pk[s];
        }
        off += (uint32_t)__popcll(bal);
    }
    if (own) o.cnt += total;
    o.cand += total;
}

// The deviation stage for the first m (<= 64) of the wavefront's queued
// LB_SAX survivors (position; LB_SAX by quarters times the queue's power-of-2
// scale, as fp16 pairs rounded toward zero, so at most the float32 quarters
// once unscaled): lane l loads series sq_pos[l]'s
// deviation codes and adds the deviation term (segment length x the squared
// distance from the query's std interval [lo, hi] to the code's interval
// [c h, (c + 1) h]) to each quarter, and keeps the series when the sum of the
// four does not exceed thr; a kept series carries them packed.
// s_sig[i] = (-hi, lo - h rounded down) of segment i, zeros past w: the gap
// max(0, c h - hi, (lo - h) - c h) takes one rounding on each side (c h is
// exact) and is at most the exact gap before it.
template <int W16>
__device__ __forceinline__ void sigma_stage(const IndexView& ix, const QueryWs& ws, const uint32_t* sq_pos,
                                            const uint32_t* sq_h01, const uint32_t* sq_h23, float unscale, int m,
                                            int q, float thr, const float2* s_sig, int lane, FilterOut& o) {
    constexpr int kQ = 4 * W16;
    const bool valid = lane < m;
    const int e = valid ? lane : 0;
    const uint32_t pos = sq_pos[e], h01 = sq_h01[e], h23 = sq_h23[e];
    o.sig += (unsigned long long)m;
    uint4 c[W16];
    load_word<W16>(ix.sig + (int64_t)pos * ix.wstride, c);
    const float h = ix.sig_h, lseg = (float)(ix.n / ix.w);
    float a[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int u = 0; u < W16; ++u) {
        const uint32_t parts[4] = {c[u].x, c[u].y, c[u].z, c[u].w};
#pragma unroll
        for (int p = 0; p < 4; ++p) {
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int i = u * 16 + p * 4 + b;
                const float code = (float)((parts[p] >> (8 * b)) & 0xffu);
                const float2 qs = s_sig[i];
                const float gap = fmaxf(0.0f, fmaxf(fmaf(code, h, qs.x), fmaf(-code, h, qs.y)));
                a[i / kQ] = fmaf(gap, gap, a[i / kQ]);
            }
        }
    }
    const float q16[4] = {(float)__builtin_bit_cast(_Float16, (uint16_t)(h01 & 0xffffu)) * unscale,
                          (float)__builtin_bit_cast(_Float16, (uint16_t)(h01 >> 16)) * unscale,
                          (float)__builtin_bit_cast(_Float16, (uint16_t)(h23 & 0xffffu)) * unscale,
                          (float)__builtin_bit_cast(_Float16, (uint16_t)(h23 >> 16)) * unscale};
#pragma unroll
    for (int p = 0; p < 4; ++p) a[p] = fmaf(a[p], lseg, q16[p]);
    const float lb = (a[0] + a[1]) + (a[2] + a[3]);
    const uint32_t posv[1] = {pos}, pkv[1] = {pack_quarters(a[0], a[1], a[2], a[3])};
    emit_candidates<1>(ws, o, lane, q, (valid && lb <= thr) ? 1u : 0u, posv, pkv);
}

// The wavefront's queue of LB_SAX survivors waiting for the deviation stage.
// The quarters are stored times scale = 2^-e, e >= 0 the smallest putting
// the threshold below 2^14, so that quarters up to four times the threshold
// keep fp16's relative precision; a larger quarter is stored as the largest
// finite fp16, still above the threshold once unscaled (a series holding one
// is pruned either way).  Scaling by a power of 2 is exact.
struct SigQueue {
    uint32_t* pos;
    uint32_t* h01;  // quarters 0 and 1 (scaled) as fp16, rounded toward zero
    uint32_t* h23;  // quarters 2 and 3
    uint32_t cnt;   // entries (uniform)
    float scale, unscale;  // 2^-e and 2^e
};

// Runs the deviation stage on the queued survivors 64 at a time; with
// flush, also on the last fewer than 64.  The rest move to the queue's front.
template <int W16>
__device__ __forceinline__ void drain_sigma(const IndexView& ix, const QueryWs& ws, SigQueue& sq, bool flush, int q,
                                            float thr, const float2* s_sig, int lane, FilterOut& o) {
    uint32_t done = 0;
    while (sq.cnt - done >= 64) {
        sigma_stage<W16>(ix, ws, sq.pos + done, sq.h01 + done, sq.h23 + done, sq.unscale, 64, q, thr, s_sig, lane,
                         o);
        done += 64;
    }
    const uint32_t rem = sq.cnt - done;
    if (flush && rem) {
        sigma_stage<W16>(ix, ws, sq.pos + done, sq.h01 + done, sq.h23 + done, sq.unscale, (int)rem, q, thr, s_sig,
                         lane, o);
        sq.cnt = 0;
        return;
    }
    if (done) {
        // rem < 64 <= done: the source and destination ranges do not overlap
        const bool mv = (uint32_t)lane < rem;
        const uint32_t a = mv ? sq.pos[done + lane] : 0u, b = mv ? sq.h01[done + lane] : 0u,
                       c = mv ? sq.h23[done + lane] : 0u;
        __builtin_amdgcn_wave_barrier();
        if (mv) {
            sq.pos[lane] = a;
            sq.h01[lane] = b;
            sq.h23[lane] = c;
        }
        __builtin_amdgcn_wave_barrier();
    }
    sq.cnt = rem;
}

// LB_SAX of up to batch_chunks<W16>() queued chunks (rows [r0, r1) each, r1 - r0 <= 64).
// Lane l takes series r0 + l of every chunk; the word loads of all chunks
// are issued before the first table lookup, and rows past a chunk (or slots
// past the batch) load zeros from no memory.  The survivors (position and
// quarters) join the wavefront's deviation queue sq (fewer than 64
// entries on entry, so it holds at most 63 + 64 kBatch), which is drained 64
// at a time.
// skip: the skip-sequential path, where every series is a candidate with
// bound 0 and no word is read.  U: batch-union diagnostics (marks the series
// whose words are read).
template <int W16, bool U>
__device__ __forceinline__ void filter_batch(const IndexView& ix, const QueryWs& ws, const uint2* queue,
                                             uint32_t head, int nb, int q, float thr, bool skip,
                                             const float* s_lut, const float2* s_sig, SigQueue& sq, int lane,
                                             FilterOut& o) {
    const uint32_t wb = (uint32_t)ix.wstride;
    constexpr int kBatch = batch_chunks<W16>();
    uint32_t r0[kBatch], r1[kBatch];
    uint4 v[kBatch][W16];
#pragma unroll
    for (int s = 0; s < kBatch; ++s) {
        const uint2 e = queue[(head + s) & (kQueue - 1)];
        r0[s] = __builtin_amdgcn_readfirstlane(e.x);
        r1[s] = s < nb ? __builtin_amdgcn_readfirstlane(e.y) : r0[s];
        const __amdgpu_buffer_rsrc_t rs =
            buffer_rsrc(ix.words + (int64_t)r0[s] * wb, skip ? 0u : (r1[s] - r0[s]) * wb);
#pragma unroll
        for (int u = 0; u < W16; ++u) v[s][u] = buffer_load16(rs, (uint32_t)lane * wb + 16u * u);
    }
    if (skip) {
        uint32_t mask = 0;
        uint32_t pos[kBatch], pk[kBatch];
#pragma unroll
        for (int s = 0; s < kBatch; ++s) {
            pos[s] = r0[s] + (uint32_t)lane;
            pk[s] = 0u;
            if (s < nb) {
                o.filt += r1[s] - r0[s];
                if ((uint32_t)lane < r1[s] - r0[s]) mask |= 1u << s;
            }
        }
        emit_candidates<kBatch>(ws, o, lane, q, mask, pos, pk);
        return;
    }
    const uint64_t lt_mask = (1ull << lane) - 1ull;
#pragma unroll
    for (int s = 0; s < kBatch; ++s) {
        if (s < nb) {
            float a[4];
            lb_sax_quarters<W16>(v[s], s_lut, a);
            const float lb = (a[0] + a[1]) + (a[2] + a[3]);
            o.filt += r1[s] - r0[s];
            if (U && (uint32_t)lane < r1[s] - r0[s]) {
                const int64_t bit = ws.word_bit0 + (int64_t)(r0[s] + (uint32_t)lane);
                atomicOr(&ws.ubits[bit >> 5], 1u << (bit & 31));
            }
            const bool keep = (uint32_t)lane < r1[s] - r0[s] && lb <= thr;
            const uint64_t bal = __ballot(keep);
            if (keep) {
                const uint32_t at = sq.cnt + (uint32_t)__popcll(bal & lt_mask);
                sq.pos[at] = r0[s] + (uint32_t)lane;
                sq.h01[at] = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(a[0] * sq.scale, a[1] * sq.scale));
                sq.h23[at] = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(a[2] * sq.scale, a[3] * sq.scale));
            }
            sq.cnt += (uint32_t)__popcll(bal);
        }
    }
    __builtin_amdgcn_wave_barrier();
    drain_sigma<W16>(ix, ws, sq, false, q, thr, s_sig, lane, o);
}

// Every wavefront takes part in every item of the window (a unit of up to
// kUnit items of one query); of item j's chunks it owns wave, wave + 4,
// wave + 8, ...  Its owned chunks of all the window's items are numbered in
// item order and tested 64 at a time, one lane per chunk: LB_EAPCA in float32
// over the chunk's outward-rounded segment intervals, summed segment by
// segment in the lane.  Chunks that pass join the wavefront's queue in LDS,
// and every batch_chunks<W16>() queued chunks go through filter_batch, so the
// LB_SAX work comes in full batches whatever fraction of chunks pass.
// U: batch-union diagnostics (marks the envelopes tested and the words read).
template <int W16, bool U>
__global__ void __launch_bounds__(256, filter_occupancy<W16>()) k_filter(IndexView ix, ScanParams sp, QueryWs ws) {
    constexpr int kBatch = batch_chunks<W16>();
    // the table first, at a fixed LDS address, so its row offsets fold into
    // the lookups' immediate offsets
    __shared__ float s_lut[lut_floats<W16>()];  // [16 W16][256], rows beyond w zero
    __shared__ uint2 s_queue[kWaves][kQueue];   // (r0, r1) of live chunks
    // LB_SAX survivors waiting for the deviation stage
    constexpr int kSigCap = 64 * (batch_chunks<W16>() + 1);
    __shared__ uint32_t s_sq_pos[kWaves][kSigCap], s_sq_h01[kWaves][kSigCap], s_sq_h23[kWaves][kSigCap];
    __shared__ uint32_t s_pb[kUnit], s_pe[kUnit], s_c0[kUnit];
    __shared__ uint32_t s_pre[kWaves][kUnit + 1];  // owned chunks before each item, per wavefront
    __shared__ float4 s_qst[64];                // query segment mean / std intervals
    __shared__ float2 s_sig[64];                // the deviation stage's terms of the std intervals
    __shared__ int s_end;
    __shared__ long long s_unit;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const float lseg = (float)(ix.n / ix.w);
    const uint64_t lt_mask = (1ull << lane) - 1ull;
    uint2* queue = s_queue[wave];
    uint32_t* pre = s_pre[wave];
    SigQueue sq{s_sq_pos[wave], s_sq_h01[wave], s_sq_h23[wave], 0u, 1.0f, 1.0f};

    const int64_t slice = (int64_t)sp.slice0 + (int64_t)blockIdx.x * kWaves + wave;
    FilterOut o{ws.slice_pos + slice * ws.slice_cap, ws.slice_q + slice * ws.slice_cap,
                ws.slice_part + slice * ws.slice_cap, 0u, 0ull, 0ull, 0ull, 0ull, false};
    // Items are dealt out in units of up to kUnit (fewer for a short item
    // list, so that a small batch still spreads over the GPU): a workgroup's
    // first unit by its index, each next one from a counter once it has
    // filtered the last, so workgroups whose items keep many candidates take
    // fewer units.
    const int64_t total = item_count(ws);
    const int64_t unit = max((int64_t)1, min((int64_t)kUnit, total / ((int64_t)gridDim.x * 4)));
    int64_t idx = (int64_t)blockIdx.x * unit, uend = min(total, idx + unit);
    int cur_q = -1;
    while (idx < uend) {
        const int n = (int)min((int64_t)kUnit, uend - idx);
        const int q = (int)(ws.items[idx] >> 32);
        __syncthreads();  // no wave still reads the previous window or table
        if (t == 0) s_end = n;
        __syncthreads();
        for (int j = t; j < n; j += blockDim.x) {
            const uint64_t it = ws.items[idx + j];
            const int64_t p = (int64_t)(uint32_t)it;
            if ((int)(it >> 32) != q) atomicMin(&s_end, j);
            s_pb[j] = (uint32_t)ix.part_start[p];
            s_pe[j] = (uint32_t)ix.part_start[p + 1];
            s_c0[j] = (uint32_t)ix.part_chunk[p];
        }
        if (q != cur_q) {
            load_lut<W16>(s_lut, ws.lut + (int64_t)q * ix.w * kCard, ix.w, t, blockDim.x);
            // zeros past w: the padding segments add nothing to the deviation term
            if (t < 64) {
                const float4 qs = t < ix.w ? ws.qst32[(int64_t)q * ix.w + t] : make_float4(0.f, 0.f, 0.f, 0.f);
                s_qst[t] = qs;
                s_sig[t] = t < ix.w ? make_float2(-qs.w, __double2float_rd((double)qs.z - (double)ix.sig_h)) : make_float2(0.f, 0.f);
            }
            cur_q = q;
        }
        __syncthreads();
        const int m = s_end;  // the window's items of query q
        const bool skip = (ws.flags[q] & kFlagSkipSax) != 0;
        // largest float32 not above the prune limit: for a float32 bound b,
        // b <= thr exactly when (double) b <= limit
        const float thr = __double2float_rd(prune_limit(bits_to_float(bsf_bits(ws, q))));
        {
            const int e = thr < INFINITY && thr >= 16384.0f ? ilogbf(thr) - 13 : 0;  // thr 2^-e < 2^14
            sq.scale = ldexpf(1.0f, -e);
            sq.unscale = ldexpf(1.0f, e);
        }
        o.filt = o.cand = o.tests = o.sig = 0;
        o.lost = false;
        uint32_t head = 0, tail = 0;  // queue positions (uniform)

        // skip-sequential path: every chunk of every item is queued untested,
        // and every series becomes a candidate
        for (int j = 0; skip && j < m; ++j) {
            const uint32_t pb = s_pb[j], pe = s_pe[j];
            const int nch = (int)((pe - pb + kChunkRows - 1) / kChunkRows);
            const int owned = nch > wave ? (nch - wave + kWaves - 1) / kWaves : 0;
            for (int s0 = 0; s0 < owned; s0 += 64) {
                const int s = s0 + lane;
                if (s < owned) {
                    const uint32_t a = pb + (uint32_t)((wave + kWaves * s) * kChunkRows);
                    queue[(tail + (uint32_t)s - (uint32_t)s0) & (kQueue - 1)] = make_uint2(a, min(pe, a + kChunkRows));
                }
                const uint32_t add = (uint32_t)min(64, owned - s0);
                // drain as the queue fills (at most kBatch - 1 + 64 < kQueue entries)
                tail += add;
                __builtin_amdgcn_wave_barrier();
                while (tail - head >= kBatch) {
                    filter_batch<W16, U>(ix, ws, queue, head, kBatch, q, thr, true, s_lut, s_sig, sq, lane, o);
                    head += kBatch;
                }
            }
        }
        if (!skip) {
            // the wavefront's owned chunks per item (lanes 0..m-1) and their
            // running total: owned chunk g lies in the last item j with pre[j] <= g
            uint32_t own = 0;
            if (lane < m) {
                const uint32_t nch = (s_pe[lane] - s_pb[lane] + kChunkRows - 1) / kChunkRows;
                own = nch > (uint32_t)wave ? (nch - (uint32_t)wave + kWaves - 1) / kWaves : 0u;
            }
            uint32_t inc = own;
#pragma unroll
            for (int d = 1; d < kUnit; d <<= 1) {
                const uint32_t y = __shfl_up(inc, d, 64);
                if (lane >= d) inc += y;
            }
            if (lane < m) pre[lane + 1] = inc;
            if (lane == 0) pre[0] = 0u;
            const uint32_t total_owned = (uint32_t)__shfl(inc, m - 1, 64);
            __builtin_amdgcn_wave_barrier();
            for (uint32_t g0 = 0; g0 < total_owned; g0 += 64) {
                const uint32_t g = g0 + (uint32_t)lane;
                const bool valid = g < total_owned;
                int j = 0;
#pragma unroll
                for (int step = kUnit / 2; step; step >>= 1)
                    if (j + step < m && pre[j + step] <= g) j += step;
                const uint32_t cn = (uint32_t)wave + kWaves * (g - pre[j]);  // chunk number in item j
                const uint32_t pb = s_pb[j], pe = s_pe[j];
                const int64_t chunk = (int64_t)s_c0[j] + cn;
                float acc = 0.0f;
                if (valid) {
                    const float4* e = ix.cenv + chunk * ix.w;
                    int i = 0;
                    for (; i + 4 <= ix.w; i += 4) {
                        float4 ce[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) ce[u] = e[i + u];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const float4 qs = s_qst[i + u];
                            const float gm = fmaxf(0.0f, fmaxf(ce[u].x - qs.y, qs.x - ce[u].y));
                            const float gs = fmaxf(0.0f, fmaxf(ce[u].z - qs.w, qs.z - ce[u].w));
                            acc = fmaf(gm, gm, acc);
                            acc = fmaf(gs, gs, acc);
                        }
                    }
                    for (; i < ix.w; ++i) {
                        const float4 ce = e[i], qs = s_qst[i];
                        const float gm = fmaxf(0.0f, fmaxf(ce.x - qs.y, qs.x - ce.y));
                        const float gs = fmaxf(0.0f, fmaxf(ce.z - qs.w, qs.z - ce.w));
                        acc = fmaf(gm, gm, acc);
                        acc = fmaf(gs, gs, acc);
                    }
                }
                const bool live = valid && lseg * acc <= thr;
                o.tests += (unsigned long long)__popcll(__ballot(valid));
                if (U && valid) {
                    const int64_t bit = ws.env_bit0 + chunk;
                    atomicOr(&ws.ubits[bit >> 5], 1u << (bit & 31));
                }
                const uint64_t lm = __ballot(live);
                if (live) {
                    const uint32_t a = pb + cn * kChunkRows;
                    queue[(tail + (uint32_t)__popcll(lm & lt_mask)) & (kQueue - 1)] = make_uint2(a, min(pe, a + kChunkRows));
                }
                tail += (uint32_t)__popcll(lm);
                __builtin_amdgcn_wave_barrier();
                while (tail - head >= kBatch) {
                    filter_batch<W16, U>(ix, ws, queue, head, kBatch, q, thr, false, s_lut, s_sig, sq, lane, o);
                    head += kBatch;
                }
            }
        }
        if (tail != head)
            filter_batch<W16, U>(ix, ws, queue, head, (int)(tail - head), q, thr, skip, s_lut, s_sig, sq, lane, o);
        // the window's last survivors, before the next window's query and table
        drain_sigma<W16>(ix, ws, sq, true, q, thr, s_sig, lane, o);
        idx += m;
        if (lane == 0) {
            atomicAdd(&ws.stats[(int64_t)q * kStatSlots + 1], skip ? 0ull : o.filt);
            atomicAdd(&ws.stats[(int64_t)q * kStatSlots + 6], o.cand);
            atomicAdd(&ws.stats[(int64_t)q * kStatSlots + 7], o.tests);
            atomicAdd(&ws.stats[(int64_t)q * kStatSlots + 8], o.sig);
            if (o.lost) atomicOr(&ws.flags[q], kFlagCandLost);
        }
        if (idx >= uend) {
            __syncthreads();  // every wave has read s_unit and the window
            if (t == 0) s_unit = (long long)gridDim.x + (long long)atomicAdd(&ws.counters[kCtrWork], 1u);
            __syncthreads();
            idx = s_unit * unit;
            uend = min(total, idx + unit);
        }
    }
    if (lane == 0) ws.slice_cnt[slice] = o.cnt;
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
        ws.counters[kCtrRefine] = 0u;  // the refine's segment counter
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
int filter_blocks(int cus) {
    return resident_grid(k_filter<W16, false>, kTile, 0, cus);
}

}  // namespace

int filter_waves(const IndexView& ix, int device_cus) {
    int blocks = 1;
    switch (w16_of(ix)) {
        case 1: blocks = filter_blocks<1>(device_cus); break;
        case 2: blocks = filter_blocks<2>(device_cus); break;
        case 3: blocks = filter_blocks<3>(device_cus); break;
        default: blocks = filter_blocks<4>(device_cus); break;
    }
    return blocks * kWaves;
}

hipError_t launch_filter(const IndexView& ix, const ScanParams& sp, const QueryWs& ws, int /*device_cus*/,
                         hipStream_t st) {
    const dim3 grid(sp.slices / kWaves);  // one slice per wavefront
    if (ws.ubits) {
        switch (w16_of(ix)) {
            case 1: k_filter<1, true><<<grid, dim3(kTile), 0, st>>>(ix, sp, ws); break;
            case 2: k_filter<2, true><<<grid, dim3(kTile), 0, st>>>(ix, sp, ws); break;
            case 3: k_filter<3, true><<<grid, dim3(kTile), 0, st>>>(ix, sp, ws); break;
            default: k_filter<4, true><<<grid, dim3(kTile), 0, st>>>(ix, sp, ws); break;
        }
    } else {
        switch (w16_of(ix)) {
            case 1: k_filter<1, false><<<grid, dim3(kTile), 0, st>>>(ix, sp, ws); break;
            case 2: k_filter<2, false><<<grid, dim3(kTile), 0, st>>>(ix, sp, ws); break;
            case 3: k_filter<3, false><<<grid, dim3(kTile), 0, st>>>(ix, sp, ws); break;
            default: k_filter<4, false><<<grid, dim3(kTile), 0, st>>>(ix, sp, ws); break;
        }
    }
    return hipGetLastError();
}

hipError_t launch_slice_prefix(const QueryWs& ws, hipStream_t st) {
    hipLaunchKernelGGL(k_slice_prefix, dim3(1), dim3(1024), 0, st, ws);
    return hipGetLastError();
}

}  // namespace hs
