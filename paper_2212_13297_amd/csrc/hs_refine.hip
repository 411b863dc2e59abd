// Refinement of the candidate list (Hercules Sec. 3.4, step 4): the exact
// float32 squared distance with early abandoning for every candidate, first
// re-checked against the current BSF_k; per-wavefront top-k, BSF_k published
// with atomicMin, results appended to the per-query pool.
//
// Wavefronts take runs of consecutive candidates (the list is ordered by
// query, so a run holds long stretches of one query) and never wait for one
// another.  Their 16-lane groups refine a few series each, one 64-point chunk
// per round, in the order of the series' LB_SAX quarter bounds, abandoning a
// series as soon as its running distance, plus the bounds of its unread
// quarters, exceeds the limit, and taking the next candidate in its place.
#include "hs_device.h"

namespace hs {
namespace {

constexpr int kRefineSlots = 4;  // candidates in flight per 16-lane group
constexpr int kSeg = 512;        // candidates per segment of a long list (a multiple of 64, >= 128)
constexpr uint32_t kNaturalPerm = 0xE4u;  // quarters 0, 1, 2, 3

struct Meta {
    int q;
    uint32_t pos;
    uint32_t part;  // LB_SAX by quarters, four bytes
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

// The value a byte of the packed quarter bounds stands for.
__device__ __forceinline__ float quarter_value(uint32_t byte) {
    return (float)__builtin_bit_cast(_Float16, (uint16_t)(byte << 8));
}

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

// Ring entry (q | perm << 24, pos, lbs, bsf): lbs = LB_SAX / (1 + slack)
// rounded down, from the exact float64 sum of the four packed partials (each
// at most the float32 one), so lbs > limit implies LB_SAX > limit (1 + slack);
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

// F: distance form.  NS: candidates in flight per 16-lane group.
//
// A wavefront refines a stream of candidates: one contiguous range of a short
// list, or segments of kSeg of a long one, its first by its index and each
// next one from a counter when its ring reaches it (so wavefronts that meet
// costly candidates take fewer segments).  Each of its four groups keeps NS
// slots; a round loads one 64-point chunk of every slot's series (and the
// query's chunk), adds the chunk's partial to the slot's running distance,
// and retires the slots whose distance exceeds their limit (abandoned) or
// whose series is complete.  Retired slots take the next candidates of the
// stream at once, so every round reads NS useful chunks per group however
// early candidates are abandoned.
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
template <int F, int NS, bool Q1, bool U>
__global__ void __launch_bounds__(256, 4) k_refine(IndexView ix, ScanParams sp, QueryWs ws) {
    constexpr int kRing = 128;
    __shared__ unsigned long long s_top[kTile / 64][HS_KMAX];
    // ring_entry of the stream's candidate v at v mod 128
    __shared__ uint4 s_ring[kTile / 64][kRing];
    __shared__ uint32_t s_rem[kTile / 64][kRing];  // the entries' rem (chunk_perm)
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6, sub = t & 15, grp = (t >> 4) & 3;
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
    // one contiguous range per wavefront.
    const long long nseg = (T + kSeg - 1) / kSeg;
    const bool dyn = nseg >= 2 * GW;
    long long vbase = 0, startA, lenA, startB = 0, lenB = 0;
    bool have_b = !dyn;
    if (dyn) {
        startA = gw * kSeg;
        lenA = kSeg;
    } else {
        startA = T * gw / GW;
        lenA = T * (gw + 1) / GW - startA;
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
    // refined series and chunks read for query st_q (uniform), per group
    int st_q = -1;
    uint32_t g_ref = 0u;  // < 2^31 candidates per wavefront
    unsigned long long g_ch = 0ull;
    auto flush_counters = [&]() {
        unsigned long long r = 0ull, c = 0ull;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            r += (uint32_t)__builtin_amdgcn_readlane(g_ref, 16 * g);
            c += ((unsigned long long)(uint32_t)__builtin_amdgcn_readlane((uint32_t)(g_ch >> 32), 16 * g) << 32) |
                 (uint32_t)__builtin_amdgcn_readlane((uint32_t)g_ch, 16 * g);
        }
        if (lane == 0 && st_q >= 0 && r) {
            atomicAdd(&ws.stats[(int64_t)st_q * 8 + 2], r);
            atomicAdd(&ws.stats[(int64_t)st_q * 8 + 3], c);
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

    const float* rows_sub = ix.rows + sub * 4;  // the lane's first point of stored row 0 and of query 0
    const float* qrow_sub = ws.qrow + sub * 4;
    // slots, each the same in the 16 lanes of its group
    int sq[NS];            // query (-1: empty)
    int sc[NS];            // chunks added so far
    uint32_t sperm[NS];    // order of the quarters
    uint32_t srem[NS];     // bounds of the quarters unread after one and after two (fp16 pair)
    float sthr[NS];        // abandoning limit times marg
    const float* xp[NS];   // the lane's first point of the series and of the query
    const float* qp[NS];
    Dist<F> sd[NS];
    bool fin[NS];          // slot wants a candidate
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        sq[s] = -1;
        sc[s] = 0;
        sperm[s] = kNaturalPerm;
        srem[s] = 0u;
        sthr[s] = INFINITY;
        xp[s] = rows_sub;
        qp[s] = qrow_sub;
        fin[s] = true;
    }

    for (;;) {
        // hand out candidates to the slots that want one, in slot order
        // (group g, slot s) -> g NS + s; a candidate whose LB_SAX exceeds its
        // limit is skipped and the slot asks again
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
            if (has_pend && next + 4 * NS > mb + 64) {
                // this hand-out reaches the entries still in flight (after many
                // skipped candidates): they are written now
                write_pend();
            }
            int rank[NS], nf = 0;
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                rank[s] = nf;
                nf += fin[s] ? 1 : 0;
            }
            const int f0 = __builtin_amdgcn_readlane(nf, 0), f1 = __builtin_amdgcn_readlane(nf, 16),
                      f2 = __builtin_amdgcn_readlane(nf, 32), f3 = __builtin_amdgcn_readlane(nf, 48);
            const int total = f0 + f1 + f2 + f3;
            if (total == 0) break;
            const int goff = (int)next + (grp > 0 ? f0 : 0) + (grp > 1 ? f1 : 0) + (grp > 2 ? f2 : 0);
            bool again = false;
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                if (!__ballot(fin[s])) continue;
                if (fin[s]) {
                    const int ri = goff + rank[s];  // stream position
                    const uint4 e = ring[ri & (kRing - 1)];
                    const int q = e.x != 0xffffffffu ? (int)(e.x & 0xffffffu) : -1;  // -1 past the stream's end
                    float lim = __uint_as_float(e.w);
                    if (q == cur_q) lim = fminf(lim, lk);
                    const uint32_t pos = q >= 0 ? e.y : 0u;
                    sq[s] = q;
                    sc[s] = 0;
                    sperm[s] = e.x >> 24;
                    srem[s] = rring[ri & (kRing - 1)];
                    sd[s] = Dist<F>{};
                    sthr[s] = lim * marg;
                    // one 32 x 32 -> 64-bit multiply each (pos, q and stride are non-negative)
                    xp[s] = rows_sub + (uint64_t)pos * (uint32_t)ix.stride;
                    qp[s] = qrow_sub + (uint64_t)(uint32_t)max(q, 0) * (uint32_t)ix.stride;
                    fin[s] = q >= 0 && __uint_as_float(e.z) > lim;  // skipped: ask again
                    again = again || fin[s];
                }
            }
            next += total;
            if (!__ballot(again)) break;
        }
        bool any = false;
#pragma unroll
        for (int s = 0; s < NS; ++s) any = any || sq[s] >= 0;
        if (!__ballot(any)) break;

        // one chunk of every slot's series (its next in the slot's order);
        // empty slots read a chunk of row 0
        float4 x[NS], qv[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int c = Q1    ? (int)((sperm[s] >> (2 * sc[s])) & 3u)
                          : ord ? ((int)((sperm[s] >> ((sc[s] >> olg) << 1)) & 3u) << olg) | (sc[s] & omask)
                                : sc[s];
            x[s] = *reinterpret_cast<const float4*>(xp[s] + c * kChunk);
            qv[s] = *reinterpret_cast<const float4*>(qp[s] + c * kChunk);
            if (U && sq[s] >= 0 && sub == 0) {
                const int64_t bit = (int64_t)((xp[s] - rows_sub) / ix.stride) * nchunks + c;
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
                sd[s].add(qv[s], x[s]);
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
                const bool over = sd[s].value() + rest > sthr[s];
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
        // the pair with: read again unless the running sum already is that
        // (precision form, natural order)
        float kv[NS];
        {
            bool rc[NS], anyrc = false;
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                kv[s] = sd[s].value();
                rc[s] = adm[s] && (F == kPlain || sperm[s] != kNaturalPerm);
                anyrc = anyrc || rc[s];
            }
            if (__ballot(anyrc)) {
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    if (!__ballot(rc[s])) continue;
                    if (rc[s]) {
                        kv[s] = key_distance(xp[s], qp[s], nchunks);
                        sc[s] += nchunks;  // chunks read again
                    }
                }
            }
        }
        // retirements one by one, in slot order
        int new_q = cur_q;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const uint64_t b = __ballot(fin[s]);
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                if (!((b >> (16 * g)) & 1ull)) continue;
                const int kq = __builtin_amdgcn_readlane(sq[s], 16 * g);
                if (kq != st_q) {
                    flush_counters();
                    st_q = kq;
                }
                if (grp == g) {
                    g_ref += 1u;
                    g_ch += (unsigned long long)sc[s];
                }
                if (__builtin_amdgcn_readlane((int)adm[s], 16 * g)) {
                    const float v = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(kv[s]), 16 * g));
                    // stored position of the series, from the lane's pointer (sub * 4 < stride)
                    const uint32_t kp = (uint32_t)__builtin_amdgcn_readlane(
                        (int)(uint32_t)((xp[s] - ix.rows) / ix.stride), 16 * g);
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
        cur_q = __shfl(new_q, 0, 64);
        lk = __shfl(new_lk, 0, 64);
#pragma unroll
        for (int s = 0; s < NS; ++s)
            if (sq[s] == cur_q) sthr[s] = fminf(sthr[s], lk * marg);
    }
    if (lane == 0) flush_topk(ws, cur_q, k, top, topn);
    flush_counters();
}

}  // namespace

hipError_t launch_refine(const IndexView& ix, const ScanParams& sp, const QueryWs& ws, int device_cus, int form,
                         hipStream_t st) {
#define HS_REFINE(FF, NS, QQ, UU)                                                                 \
    k_refine<FF, NS, QQ, UU><<<dim3(resident_grid(k_refine<FF, NS, QQ, UU>, kTile, 0, device_cus)), dim3(kTile), 0, \
                               st>>>(ix, sp, ws)
    const bool q1 = sp.order_lg == 0;
    if (ws.ubits) {
        if (form == kComp) {
            if (q1) HS_REFINE(kComp, kRefineSlots, true, true);
            else HS_REFINE(kComp, kRefineSlots, false, true);
        } else {
            if (q1) HS_REFINE(kPlain, kRefineSlots, true, true);
            else HS_REFINE(kPlain, kRefineSlots, false, true);
        }
    } else if (form == kComp) {
        if (q1) HS_REFINE(kComp, kRefineSlots, true, false);
        else HS_REFINE(kComp, kRefineSlots, false, false);
    } else {
        if (q1) HS_REFINE(kPlain, kRefineSlots, true, false);
        else HS_REFINE(kPlain, kRefineSlots, false, false);
    }
#undef HS_REFINE
    return hipGetLastError();
}

}  // namespace hs
