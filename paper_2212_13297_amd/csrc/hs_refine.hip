// Refinement of the candidate list (Hercules Sec. 3.4, step 4): the exact
// float32 squared distance with early abandoning for every candidate, first
// re-checked against the current BSF_k; per-wavefront top-k, BSF_k published
// with atomicMin, results appended to the per-query pool.
//
// Wavefronts take runs of consecutive candidates (a run holds long stretches
// of one query) and never wait for one another.  Their 4-lane groups refine
// one series each, one 64-point chunk per round, in the order of the series'
// quarter bounds (the filter's lower bound -- LB_SAX plus the deviation term
// -- split by quarters of the word), abandoning a series as soon as its
// running distance, plus the bounds of its unread quarters, exceeds the
// limit, and taking the next candidate in its place.
//
// What bounds the kernel is the latency of its scattered chunk reads: the
// memory system serves about the batch's distinct chunks (re-reads of a
// chunk by other queries mostly hit the caches), and a wavefront waits for
// its round's chunks before it can hand out the next candidates.  So
// resident wavefronts count more than candidates in flight per wavefront:
// one slot per group at four wavefronts per SIMD is faster than two slots at
// three or four slots at two.
#include "hs_device.h"

namespace hs {
namespace {

constexpr int kRefineLanes = 4;  // lanes per series
constexpr int kRefineSlots = 1;  // candidates in flight per group
constexpr int kSeg = 512;        // candidates per segment of a long list (a multiple of 64, >= 128)
constexpr uint32_t kNaturalPerm = 0xE4u;  // quarters 0, 1, 2, 3

struct Meta {
    int q;
    uint32_t pos;
    uint32_t part;  // the filter's lower bound by quarters, four bytes
};

// The candidate list is the concatenation of the filter's slices (the private
// slices, then the overflow slice); slice_start holds their exclusive prefix.
// Slice of list entry c: the last s with slice_start[s] <= c, searched from the
// lane's previous slice (entries are visited in increasing order, so the hint
// is almost always right and otherwise a short binary search finds it).
__device__ __forceinline__ int slice_of(const QueryWs& ws, long long c, int hint) {
    if ((long long)ws.slice_start[hint + 1] > c) return hint;
    int lo = hint + 1, hi = ws.n_slices;  // answer in [lo, hi]
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if ((long long)ws.slice_start[mid] <= c) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Candidate c of the list, read by every lane of a wavefront for consecutive
// c.  The lane keeps its slice's first entry and end in registers: only a
// step across a slice end loads the prefix again (a lane's c only grows).  A
// lane without a candidate reads entry T - 1 and marks it invalid, so the
// loads do not depend on c.
struct SliceCursor {
    int s = 0;
    long long begin = 0, end = 0;
};

__device__ __forceinline__ Meta load_meta(const QueryWs& ws, long long c, bool valid, long long T,
                                          SliceCursor& cur) {
    const long long cc = valid ? c : T - 1;
    if (cc >= cur.end) {
        cur.s = slice_of(ws, cc, cur.s);
        cur.begin = ws.slice_start[cur.s];
        cur.end = ws.slice_start[cur.s + 1];
    }
    const long long e = (long long)cur.s * ws.slice_cap + (cc - cur.begin);
    Meta m;
    m.q = (int)ws.slice_q[e];
    m.pos = ws.slice_pos[e];
    m.part = ws.slice_part[e];
    if (!valid) m.q = -1;
    return m;
}

typedef _Float16 half2_t __attribute__((ext_vector_type(2)));

// The order in which a series' quarters are read: the largest partial bound
// first, equal bounds in natural order.  Quarter j of the order sits in bits
// 2j and 2j + 1.  The bytes of the packed bounds order as their values; the
// sort keys carry 3 - p in their low two bits.  rem: the bounds of the
// quarters still unread after the first one and after the first two, each
// divided by (1 + slack), as two fp16 rounded toward zero.
__device__ __forceinline__ uint32_t chunk_perm(uint32_t part, uint32_t& rem) {
    uint32_t k[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) k[p] = (((part >> (8 * p)) & 0xffu) << 2) | (uint32_t)(3 - p);
    auto ce = [](uint32_t& x, uint32_t& y) {
        const uint32_t hi = max(x, y), lo = min(x, y);
        x = hi;
        y = lo;
    };
    ce(k[0], k[1]);
    ce(k[2], k[3]);
    ce(k[0], k[2]);
    ce(k[1], k[3]);
    ce(k[1], k[2]);
    uint32_t perm = 0u;
#pragma unroll
    for (int j = 0; j < 4; ++j) perm |= (3u - (k[j] & 3u)) << (2 * j);
    const double v2 = quarter_value(k[2] >> 2), v3 = quarter_value(k[3] >> 2);
    const double r2 = v2 + v3, r1 = (double)quarter_value(k[1] >> 2) + r2;  // exact
    rem = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(__double2float_rd(r1 / (1.0 + kSlack)),
                                                                   __double2float_rd(r2 / (1.0 + kSlack))));
    return perm;
}

// Ring entry (q | perm << 24, pos, lbs, bsf): lbs = the lower bound / (1 +
// slack) rounded down, from the exact float64 sum of the four packed partials
// (each at most the float32 one), so lbs > limit implies a bound above
// limit (1 + slack);
// bsf, a BSF_k of the entry's query read before it is handed out (+inf until
// then).  An entry without a candidate has x = 0xffffffff.  rem: chunk_perm's
// (0 in natural order).
__device__ __forceinline__ uint4 ring_entry(const Meta& m, bool ord, uint32_t& rem) {
    double lb = 0.0;
#pragma unroll
    for (int p = 0; p < 4; ++p) lb += (double)quarter_value((m.part >> (8 * p)) & 0xffu);
    rem = 0u;
    const uint32_t perm = ord ? chunk_perm(m.part, rem) : kNaturalPerm;
    return make_uint4(m.q < 0 ? 0xffffffffu : ((uint32_t)m.q | perm << 24), m.pos,
                      __float_as_uint(__double2float_rd(lb / (1.0 + kSlack))), 0x7f800000u);
}

// The partial of one 64-point chunk for a group of LG lanes (4 or 8): lane j
// holds points 4 (j + LG i) .. + 3 for i < 16 / LG (so each load of a group
// reads 4 LG contiguous floats).  The lane squares its differences into four
// accumulators (a chain of 16 / LG each), adds them pairwise, and log2(LG)
// DPP steps sum the group.  A term passes through at most as many roundings
// as in the 16-lane partial (at LG = 4: 4 in the chain, 2 pairwise, 2 in
// the butterfly; at LG = 8: 2, 2 and 3), so the abandoning margin holds
// unchanged.
template <int LG>
__device__ __forceinline__ float group_partial(const float4 (&q)[16 / LG], const float4 (&x)[16 / LG]) {
    float4 a;
    {
        const float t0 = q[0].x - x[0].x, t1 = q[0].y - x[0].y, t2 = q[0].z - x[0].z, t3 = q[0].w - x[0].w;
        a = make_float4(t0 * t0, t1 * t1, t2 * t2, t3 * t3);
    }
#pragma unroll
    for (int i = 1; i < 16 / LG; ++i) {
        const float t0 = q[i].x - x[i].x, t1 = q[i].y - x[i].y, t2 = q[i].z - x[i].z, t3 = q[i].w - x[i].w;
        a.x = fmaf(t0, t0, a.x);
        a.y = fmaf(t1, t1, a.y);
        a.z = fmaf(t2, t2, a.z);
        a.w = fmaf(t3, t3, a.w);
    }
    float p = (a.x + a.y) + (a.z + a.w);
    p += row_xor<1>(p);
    p += row_xor<2>(p);
    if (LG >= 8) p += row_xor<4>(p);
    return p;
}

// One bit per LG-lane group: its first lane.
constexpr uint64_t group_heads(int lg) {
    uint64_t m = 0ull;
    for (int i = 0; i < 64; i += lg) m |= 1ull << i;
    return m;
}

// LG: lanes per series (4 or 8).  NS: candidates in flight per group.
//
// A wavefront refines a stream of candidates: one contiguous range of a short
// list, or segments of kSeg of a long one, its first by its index and each
// next one from a counter when its ring reaches it (so wavefronts that meet
// costly candidates take fewer segments).  Each of its 64 / LG groups of LG
// lanes keeps NS slots; a round loads one 64-point chunk of every slot's series
// (and the query's chunk), adds the chunk's partial to the slot's running
// distance, and retires the slots whose distance exceeds their limit
// (abandoned) or whose series is complete.  Retired slots take the next
// candidates of the stream at once, so every round reads NS useful chunks
// per group however early candidates are abandoned.  With few lanes per
// series the per-candidate bookkeeping (hand-out, order, cascade, limits) is
// spread over LG lanes instead of 16, and a round covers 64 / LG NS series.
//
// The running distance is plain float32 in any chunk order.  A series that
// completes within its limit is read again for its result key, the
// compensated distance in natural chunk order (key_distance, by one 16-lane
// row of the wavefront; up to four such series per pass), the value every
// kernel keys the pair with.
//
// The candidates' metadata pass through a ring of 128 entries in LDS per
// wavefront (the next 64 are loaded while the current ones are handed out),
// each with a BSF_k of its own query, read once its metadata has arrived.  A
// slot's limit is the smaller of that BSF_k and, for the query of the
// wavefront's top-k, its own k-th distance; an older BSF_k is only a looser
// limit.
// Counters accumulate per group in registers; only rounds that complete a
// series within its limit, or retire a candidate of another query, go
// through lane 0, which alone keeps the wavefront's top-k in LDS and
// publishes its improvements with atomicMin.
// Q1: one chunk per quarter in the chunk order (n = 256): the chunk index is a
// field of the order word and the cascade's bounds shift out as it is read.
// U: batch-union diagnostics (marks every (series, chunk) pair read).
template <int LG, int NS, bool Q1, bool U>
__global__ void __launch_bounds__(256, 4) k_refine(IndexView ix, ScanParams sp, QueryWs ws) {
    static_assert(LG == 4 || LG == 8, "4 or 8 lanes per series");
    constexpr int kRing = 128;
    constexpr int kGroups = 64 / LG;                      // groups per wavefront
    constexpr int kNV = 16 / LG;                          // float4 loads per lane per chunk
    constexpr uint64_t kHeads = group_heads(LG);          // the first lane of every group
    static_assert(kGroups * NS <= 64, "a hand-out must stay within the ring's loaded half");
    __shared__ unsigned long long s_top[kTile / 64][HS_KMAX];
    // ring_entry of the stream's candidate v at v mod 128
    __shared__ uint4 s_ring[kTile / 64][kRing];
    __shared__ uint32_t s_rem[kTile / 64][kRing];  // the entries' rem (chunk_perm)
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6, sub = lane & (LG - 1), grp = lane / LG;
    const uint64_t below = ((1ull << (LG * grp)) - 1ull) & kHeads;  // heads of the lower groups
    const int k = sp.k;
    const int nchunks = ix.stride / kChunk;
    // chunk order: quarters in the ring entry's order, chunks of a quarter in
    // natural order; the running distance is tested against limit * marg,
    // which proves the result key (compensated, natural order) above the limit
    const int olg = sp.order_lg;
    const bool ord = olg >= 0;
    const int omask = ord ? (1 << olg) - 1 : 0;
    const int cpq = omask + 1;  // chunks per quarter
    const float marg = sp.marg;
    const long long T = ws.slice_start[ws.n_slices + 1];
    const long long gw = (long long)blockIdx.x * (kTile / 64) + wave, GW = (long long)gridDim.x * (kTile / 64);
    // The wavefront's stream of candidates: list entries startA .. startA +
    // lenA - 1 at stream positions vbase .., then startB .. startB + lenB - 1.
    // A long list is cut into segments of kSeg, the wavefront's first by its
    // index and each next one taken from a counter when the ring reaches it
    // (wavefronts that meet costly candidates take fewer); a short one into
    // one contiguous range per wavefront, of at least sp.min_range candidates
    // (the wavefronts past them have none).
    const long long nseg = (T + kSeg - 1) / kSeg;
    const bool dyn = nseg >= 2 * GW;
    long long vbase = 0, startA, lenA, startB = 0, lenB = 0;
    bool have_b = !dyn;
    if (dyn) {
        startA = gw * kSeg;
        lenA = kSeg;
    } else {
        const long long GWr = max(1ll, min(GW, T / max(1, sp.min_range)));
        startA = gw < GWr ? T * gw / GWr : T;
        lenA = gw < GWr ? T * (gw + 1) / GWr - startA : 0;
    }
    if (lenA <= 0) return;
    // list index c of stream position v (false: past the stream's end)
    auto vmap = [&](long long v, long long& c) -> bool {
        const long long off = v - vbase;
        if (off < lenA) {
            c = startA + off;
            return true;
        }
        c = startB + (off - lenA);
        return off - lenA < lenB;
    };
    unsigned long long* top = s_top[wave];
    uint4* ring = s_ring[wave];
    uint32_t* rring = s_rem[wave];

    // wavefront state, uniform: the query of the top-k and its k-th distance
    int cur_q = -1;
    float lk = INFINITY;
    int topn = 0;                                     // lane 0
    unsigned long long pub = kInfKey;                 // lane 0: k-th key last published for cur_q
    // refined series and chunks read for query st_q (uniform), per group (the
    // group's lanes hold the same values)
    int st_q = -1;
    uint32_t g_ref = 0u;  // < 2^31 candidates per wavefront
    unsigned long long g_ch = 0ull;
    auto flush_counters = [&]() {
        // sum over the group heads (lanes LG g): xor steps LG .. 32 gather them in lane 0
        uint32_t r = sub == 0 ? g_ref : 0u;
        unsigned long long c = sub == 0 ? g_ch : 0ull;
#pragma unroll
        for (int o = 32; o >= LG; o >>= 1) {
            r += __shfl_xor(r, o, 64);
            c += __shfl_xor(c, o, 64);
        }
        if (lane == 0 && st_q >= 0 && r) {
            atomicAdd(&ws.stats[(int64_t)st_q * kStatSlots + 2], (unsigned long long)r);
            atomicAdd(&ws.stats[(int64_t)st_q * kStatSlots + 3], c);
        }
        g_ref = 0u;
        g_ch = 0ull;
    };

    SliceCursor cur;
    long long mb = 0;  // the ring holds stream positions mb .. mb + 127
    // BSF_k of the query of the entry at ring index snap_idx (this lane's entry
    // of the last window written), requested when the window was written and
    // stored into the ring a round later (snap_due)
    float nsnap;
    int snap_idx = 0;
    bool snap_due = false;
    {
        long long ca, cb;
        const bool va = vmap(lane, ca), vb = vmap(64 + lane, cb);
        const Meta a = load_meta(ws, ca, va, T, cur);
        const Meta b = load_meta(ws, cb, vb, T, cur);
        uint4 ea = ring_entry(a, ord, rring[lane]);
        ea.w = bsf_bits(ws, max(a.q, 0));
        ring[lane] = ea;
        ring[64 + lane] = ring_entry(b, ord, rring[64 + lane]);
        nsnap = bits_to_float(bsf_bits(ws, max(b.q, 0)));
        snap_idx = 64 + lane;
        snap_due = true;
    }
    Meta pend{-1, 0u, 0u};  // the next 64 entries, written to the ring after this round's loads
    bool has_pend = false;
    auto write_snap = [&]() {
        reinterpret_cast<uint32_t*>(&ring[snap_idx])[3] = __float_as_uint(nsnap);
        snap_due = false;
    };
    // pend goes into the ring and the BSF_k of its queries is requested
    auto write_pend = [&]() {
        if (snap_due) write_snap();
        snap_idx = ((int)(mb + 64) & (kRing - 1)) + lane;
        uint32_t rw;
        ring[snap_idx] = ring_entry(pend, ord, rw);
        rring[snap_idx] = rw;
        nsnap = bits_to_float(bsf_bits(ws, max(pend.q, 0)));
        snap_due = true;
        has_pend = false;
    };
    long long next = 0;  // stream position of the next candidate to hand out (uniform)

    // the lane's first point of stored row 0 and of query 0 in each load
    const float* rows_sub = ix.rows + sub * 4;
    const float* qrow_sub = ws.qrow + sub * 4;
    const float* rows16 = ix.rows + (lane & 15) * 4;  // the same for a 16-lane row (result keys)
    const float* qrow16 = ws.qrow + (lane & 15) * 4;
    // slots, each the same in the 4 lanes of its group
    int sq[NS];            // query (-1: empty)
    uint32_t spos[NS];     // stored position of the series
    int sc[NS];            // chunks added so far
    uint32_t sperm[NS];    // order of the quarters
    uint32_t srem[NS];     // bounds of the quarters unread after one and after two (fp16 pair)
    float sthr[NS];        // abandoning limit times marg
    const float* xp[NS];   // the lane's first point of the series and of the query
    const float* qp[NS];
    float sd[NS];          // running distance
    bool fin[NS];          // slot wants a candidate
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        sq[s] = -1;
        spos[s] = 0u;
        sc[s] = 0;
        sperm[s] = kNaturalPerm;
        srem[s] = 0u;
        sthr[s] = INFINITY;
        xp[s] = rows_sub;
        qp[s] = qrow_sub;
        sd[s] = 0.0f;
        fin[s] = true;
    }

    for (;;) {
        // hand out candidates to the slots that want one: slot 0 of every
        // wanting group in group order, then slot 1, ...; a candidate whose
        // lower bound exceeds its limit is skipped and the slot asks again
        for (;;) {
            if (next - mb >= 64) {
                // the ring moves on by 64: the entries now handed out have
                // their BSF_k, and the next 64 entries are loaded (written
                // after this round's loads)
                if (has_pend) write_pend();
                if (snap_due) write_snap();
                mb += 64;
                if (dyn) {
                    if (mb - vbase >= lenA) {
                        // segment A is handed out: B moves up
                        vbase += lenA;
                        startA = startB;
                        lenA = lenB;
                        lenB = 0;
                        have_b = false;
                    }
                    if (!have_b && mb + 64 >= vbase + lenA) {
                        // the entries loaded next lie past segment A: take the next segment
                        uint32_t r = 0u;
                        if (lane == 0) r = atomicAdd(&ws.counters[kCtrRefine], 1u);
                        const long long sg = GW + (long long)__builtin_amdgcn_readfirstlane(r);
                        startB = sg * kSeg;
                        lenB = sg < nseg ? min((long long)kSeg, T - startB) : 0;
                        have_b = true;
                    }
                }
                long long cp;
                const bool vp = vmap(mb + 64 + lane, cp);
                pend = load_meta(ws, cp, vp, T, cur);
                has_pend = true;
            }
            if (has_pend && next + kGroups * NS > mb + 64) {
                // this hand-out reaches the entries still in flight (after many
                // skipped candidates): they are written now
                write_pend();
            }
            int total = 0;
            bool again = false;
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const uint64_t m = __ballot(fin[s]) & kHeads;
                if (!m) continue;
                if (fin[s]) {
                    const int ri = (int)next + total + __popcll(m & below);  // stream position (low bits)
                    const uint4 e = ring[ri & (kRing - 1)];
                    const int q = e.x != 0xffffffffu ? (int)(e.x & 0xffffffu) : -1;  // -1 past the stream's end
                    float lim = __uint_as_float(e.w);
                    if (q == cur_q) lim = fminf(lim, lk);
                    const uint32_t pos = q >= 0 ? e.y : 0u;
                    sq[s] = q;
                    spos[s] = pos;
                    sc[s] = 0;
                    sperm[s] = e.x >> 24;
                    srem[s] = rring[ri & (kRing - 1)];
                    sd[s] = 0.0f;
                    sthr[s] = lim * marg;
                    // one 32 x 32 -> 64-bit multiply each (pos, q and stride are non-negative)
                    xp[s] = rows_sub + (uint64_t)pos * (uint32_t)ix.stride;
                    qp[s] = qrow_sub + (uint64_t)(uint32_t)max(q, 0) * (uint32_t)ix.stride;
                    fin[s] = q >= 0 && __uint_as_float(e.z) > lim;  // skipped: ask again
                    again = again || fin[s];
                }
                total += __popcll(m);
            }
            if (total == 0) break;
            next += total;
            if (!__ballot(again)) break;
        }
        bool any = false;
#pragma unroll
        for (int s = 0; s < NS; ++s) any = any || sq[s] >= 0;
        if (!__ballot(any)) break;
        // one chunk of every slot's series (its next in the slot's order);
        // empty slots read a chunk of row 0
        float4 xa[NS][kNV], qa[NS][kNV];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int c = Q1    ? (int)((sperm[s] >> (2 * sc[s])) & 3u)
                          : ord ? ((int)((sperm[s] >> ((sc[s] >> olg) << 1)) & 3u) << olg) | (sc[s] & omask)
                                : sc[s];
            const float* xb = xp[s] + c * kChunk;
            const float* qb = qp[s] + c * kChunk;
#pragma unroll
            for (int i = 0; i < kNV; ++i) {
                xa[s][i] = *reinterpret_cast<const float4*>(xb + 4 * LG * i);
                qa[s][i] = *reinterpret_cast<const float4*>(qb + 4 * LG * i);
            }
            if (U && sq[s] >= 0 && sub == 0) {
                const int64_t bit = (int64_t)spos[s] * nchunks + c;
                atomicOr(&ws.ubits[bit >> 5], 1u << (bit & 31));
            }
        }
        bool adm[NS];
        bool slow = false;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            adm[s] = false;
            fin[s] = false;
            if (sq[s] >= 0) {
                sd[s] += group_partial<LG>(qa[s], xa[s]);
                sc[s] += 1;
                // cascade: after the first and the second quarter, the bounds of
                // the quarters still unread are added to the running distance
                float rest = 0.0f;
                if (Q1) {
                    rest = (float)__builtin_bit_cast(half2_t, srem[s]).x;
                    srem[s] >>= 16;
                } else if (ord) {
                    const half2_t h = __builtin_bit_cast(half2_t, srem[s]);
                    rest = sc[s] == cpq ? (float)h.x : (sc[s] == 2 * cpq ? (float)h.y : 0.0f);
                }
                const bool over = sd[s] + rest > sthr[s];
                fin[s] = over || sc[s] == nchunks;
                adm[s] = fin[s] && !over;
                slow = slow || adm[s] || (fin[s] && sq[s] != st_q);
            }
        }
        if (snap_due) write_snap();
        if (has_pend) write_pend();

        if (!__ballot(slow)) {
            // common round: nothing admitted, every retired candidate of st_q
#pragma unroll
            for (int s = 0; s < NS; ++s)
                if (fin[s]) {
                    g_ref += 1u;
                    g_ch += (unsigned long long)sc[s];
                }
            continue;
        }
        // a series completed within its limit gets its result key distance,
        // the compensated one in natural chunk order that every kernel keys
        // the pair with: read again by one 16-lane row of the wavefront, up
        // to four series per pass
        float kv[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            kv[s] = sd[s];
            uint64_t m = __ballot(adm[s]) & kHeads;
            while (m) {
                // the batch: the lowest four admitted groups, row j of the
                // wavefront taking the j-th
                uint64_t batch = 0ull, r = m;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const uint64_t lo = r & (~r + 1ull);
                    batch |= lo;
                    r ^= lo;
                }
                m = r;
                const int row = lane >> 4;
                int src = -1;
                {
                    uint64_t b = batch;
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int l = b ? __builtin_ctzll(b) : -1;
                        if (j == row) src = l;
                        b &= b - 1ull;
                    }
                }
                float v = 0.0f;
                const int sl = max(src, 0);
                const uint32_t kpos = (uint32_t)__shfl((int)spos[s], sl, 64);
                const int kq = __shfl(max(sq[s], 0), sl, 64);
                if (src >= 0)
                    v = key_distance(rows16 + (uint64_t)kpos * (uint32_t)ix.stride,
                                     qrow16 + (uint64_t)(uint32_t)kq * (uint32_t)ix.stride, nchunks);
                // the group whose head is the j-th of the batch takes row j's value
                const int j = __popcll(batch & ((1ull << (LG * grp)) - 1ull));
                const float vj = __shfl(v, 16 * min(j, 3), 64);
                if ((batch >> (LG * grp)) & 1ull) {
                    kv[s] = vj;
                    sc[s] += nchunks;  // chunks read again
                }
            }
        }
        // retirements one by one, in slot order
        int new_q = cur_q;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            uint64_t m = __ballot(fin[s]) & kHeads;
            while (m) {
                const int l = __builtin_ctzll(m);
                m &= m - 1ull;
                const int kq = __builtin_amdgcn_readlane(sq[s], l);
                if (kq != st_q) {
                    flush_counters();
                    st_q = kq;
                }
                if (grp == l / LG) {
                    g_ref += 1u;
                    g_ch += (unsigned long long)sc[s];
                }
                if (__builtin_amdgcn_readlane((int)adm[s], l)) {
                    const float v = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(kv[s]), l));
                    const uint32_t kp = (uint32_t)__builtin_amdgcn_readlane((int)spos[s], l);
                    if (lane == 0) {
                        if (kq != new_q) {
                            flush_topk(ws, new_q, k, top, topn);
                            new_q = kq;
                            topn = 0;
                        }
                        topk_insert(top, topn, k, ((unsigned long long)__float_as_uint(v) << 32) | ix.ids[kp]);
                    }
                }
            }
        }
        float new_lk = INFINITY;
        if (lane == 0) {
            if (new_q != cur_q) pub = kInfKey;
            if (new_q >= 0 && topn == k) {
                const unsigned long long kk = top[k - 1];
                new_lk = bits_to_float((uint32_t)(kk >> 32));
                // the key bound only decreases: every improvement of this
                // wavefront's k-th key is published, without reading the
                // global value back (a load here would hold up the next round)
                if (kk < pub) {
                    atomicMin(&ws.bkey[new_q], kk);
                    pub = kk;
                }
            }
        }
        cur_q = __builtin_amdgcn_readlane(new_q, 0);
        lk = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(new_lk), 0));
#pragma unroll
        for (int s = 0; s < NS; ++s)
            if (sq[s] == cur_q) sthr[s] = fminf(sthr[s], lk * marg);
    }
    if (lane == 0) flush_topk(ws, cur_q, k, top, topn);
    flush_counters();
}

}  // namespace

// Both forms refine with the plain running distance; the result keys are the
// compensated ones either way.  A short list of the plain form (a few
// queries' LB_SAX candidates) goes to wavefronts 32 candidates or more each:
// one query's list over every wavefront left most of them a handful of
// candidates and had thousands of them append to that query's result pool
// (single-query latency 0.42 -> 0.34 ms at 10M x 256).  The precision form's
// few candidates per query, each refined in full, keep the widest spread.
hipError_t launch_refine(const IndexView& ix, const ScanParams& sp_in, const QueryWs& ws, int device_cus, int form,
                         hipStream_t st) {
    ScanParams sp = sp_in;
    sp.min_range = form == kPlain ? 32 : 1;
#define HS_REFINE(QQ, UU)                                                                     \
    do {                                                                                      \
        auto kern = k_refine<kRefineLanes, kRefineSlots, QQ, UU>;                             \
        hipLaunchKernelGGL(kern, dim3(resident_grid(kern, kTile, 0, device_cus)), dim3(kTile), 0, st, ix, sp, ws); \
    } while (0)
    const bool q1 = sp.order_lg == 0;
    if (ws.ubits) {
        if (q1) HS_REFINE(true, true);
        else HS_REFINE(false, true);
    } else {
        if (q1) HS_REFINE(true, false);
        else HS_REFINE(false, false);
    }
#undef HS_REFINE
    return hipGetLastError();
}

}  // namespace hs
