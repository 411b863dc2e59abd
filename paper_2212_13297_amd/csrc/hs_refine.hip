// Refinement of the candidate list (Hercules Sec. 3.4, step 4): the exact
// float32 squared distance with early abandoning for every candidate, first
// re-checked against the current BSF_k; per-wavefront top-k, BSF_k published
// with atomicMin, results appended to the per-query pool.
//
// Every wavefront owns a contiguous range of the candidate list (regions are
// ordered by query, so a range holds long runs of one query) and never waits
// for another wavefront.  Its 16-lane groups refine a few series each, one
// 64-point chunk per round, abandoning a series as soon as its running
// distance exceeds the limit and taking the next candidate in its place.
#include "hs_device.h"

namespace hs {
namespace {

constexpr int kRefineSlots = 4;  // candidates in flight per 16-lane group

struct Meta {
    int q;
    uint32_t pos;
    float lb;
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
// step across a slice end loads the prefix again.  A lane past cend reads
// entry cend - 1 and marks it invalid, so the loads do not depend on c.
struct SliceCursor {
    int s = 0;
    long long begin = 0, end = 0;
};

__device__ __forceinline__ Meta load_meta(const QueryWs& ws, long long c, long long cend, SliceCursor& cur) {
    const long long cc = min(c, cend - 1);
    if (cc >= cur.end) {
        cur.s = slice_of(ws, cc, cur.s);
        cur.begin = ws.slice_start[cur.s];
        cur.end = ws.slice_start[cur.s + 1];
    }
    const long long e = (long long)cur.s * ws.slice_cap + (cc - cur.begin);
    Meta m;
    m.q = (int)ws.slice_q[e];
    m.pos = ws.slice_pos[e];
    m.lb = ws.slice_lb[e];
    if (c >= cend) m.q = -1;
    return m;
}

__device__ __forceinline__ uint4 ring_entry(const Meta& m) {
    return make_uint4((uint32_t)m.q, m.pos, __float_as_uint(__double2float_rd((double)m.lb / (1.0 + kSlack))), 0u);
}

// F: distance form.  NS: candidates in flight per 16-lane group.
//
// Every wavefront owns a contiguous range of the candidate list.  Each of its
// four groups keeps NS slots; a round loads one 64-point chunk of every
// slot's series (and the query's chunk), adds the chunk's partial to the
// slot's running distance, and retires the slots whose distance exceeds
// their limit (abandoned) or whose series is complete.  Retired slots take
// the next candidates of the range at once, so every round reads NS useful
// chunks per group however early candidates are abandoned.
//
// The candidates' metadata pass through a ring of 128 entries in LDS per
// wavefront (the next 64 are loaded while the current ones are handed out).
// A slot's limit is the smaller of the last BSF_k read for its query and the
// wavefront's own k-th distance; an older BSF_k is only a looser limit.
// Counters accumulate per group in registers; only rounds that complete a
// series within its limit, or retire a candidate of another query, go
// through lane 0, which alone keeps the wavefront's top-k in LDS and
// publishes its improvements with atomicMin.
template <int F, int NS>
__global__ void __launch_bounds__(256) k_refine(IndexView ix, ScanParams sp, QueryWs ws) {
    constexpr int kRing = 128;
    __shared__ unsigned long long s_top[kTile / 64][HS_KMAX];
    // (q, pos, lbs, -) of candidate i at (i - cbeg) mod 128, lbs = LB_SAX / (1 + slack)
    // rounded down: lbs > limit implies LB_SAX > limit (1 + slack), the skip test
    __shared__ uint4 s_ring[kTile / 64][kRing];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6, sub = t & 15, grp = (t >> 4) & 3;
    const int k = sp.k;
    const int nchunks = ix.stride / kChunk;
    const long long T = ws.slice_start[ws.n_slices + 1];
    const long long gw = (long long)blockIdx.x * (kTile / 64) + wave, GW = (long long)gridDim.x * (kTile / 64);
    const long long cbeg = T * gw / GW, cend = T * (gw + 1) / GW;
    if (cbeg >= cend) return;
    const int nrel = (int)(cend - cbeg);  // candidates of this wavefront (< 2^31)
    unsigned long long* top = s_top[wave];
    uint4* ring = s_ring[wave];

    // wavefront state, uniform: the query of the top-k and its k-th distance
    int cur_q = -1;
    float lk = INFINITY;
    int topn = 0;                                     // lane 0
    float pub = INFINITY;                             // lane 0: k-th distance last published for cur_q
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
    long long mb = cbeg;  // the ring holds candidates mb .. mb + 127
    int bq, pq;           // query of the last BSF_k read and of the one in flight
    float bv, pv;
    {
        const Meta a = load_meta(ws, mb + lane, cend, cur);
        const Meta b = load_meta(ws, mb + 64 + lane, cend, cur);
        ring[lane] = ring_entry(a);
        ring[64 + lane] = ring_entry(b);
        bq = pq = __builtin_amdgcn_readfirstlane(a.q);
        bv = pv = bits_to_float(load_relaxed(&ws.bsf[max(bq, 0)]));
    }
    Meta pend{-1, 0u, 0.0f};  // the next 64 entries, written to the ring after this round's loads
    bool has_pend = false;
    long long next = cbeg;  // next candidate to hand out (uniform)

    // slots, each the same in the 16 lanes of its group
    int sq[NS];            // query (-1: empty)
    uint32_t spos[NS];     // stored position of the series
    int sc[NS];            // chunks added so far
    float sthr[NS];        // abandoning limit
    const float* xp[NS];   // the lane's first point of the series and of the query
    const float* qp[NS];
    Dist<F> sd[NS];
    bool fin[NS];          // slot wants a candidate
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        sq[s] = -1;
        spos[s] = 0u;
        sc[s] = 0;
        sthr[s] = INFINITY;
        xp[s] = ix.rows + sub * 4;
        qp[s] = ws.qrow + sub * 4;
        fin[s] = true;
    }

    for (;;) {
        // hand out candidates to the slots that want one, in slot order
        // (group g, slot s) -> g NS + s; a candidate whose LB_SAX exceeds its
        // limit is skipped and the slot asks again
        for (;;) {
            if (next - mb >= 64) {
                // the ring moves on by 64: the next 64 entries are loaded (and
                // written after this round's loads), the BSF_k read at the last
                // move is taken over and the next one is issued
                if (has_pend) {
                    ring[((int)(mb + 64 - cbeg) & (kRing - 1)) + lane] = ring_entry(pend);
                    has_pend = false;
                }
                mb += 64;
                pend = load_meta(ws, mb + 64 + lane, cend, cur);
                has_pend = true;
                bq = pq;
                bv = pv;
                pq = __builtin_amdgcn_readfirstlane((int)ring[(int)(mb - cbeg) & (kRing - 1)].x);
                pv = bits_to_float(load_relaxed(&ws.bsf[max(pq, 0)]));
            }
            if (has_pend && next + 4 * NS > mb + 64) {
                // this hand-out reaches the entries still in flight (after many
                // skipped candidates): they are written now
                ring[((int)(mb + 64 - cbeg) & (kRing - 1)) + lane] = ring_entry(pend);
                has_pend = false;
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
            const int goff = (int)(next - cbeg) + (grp > 0 ? f0 : 0) + (grp > 1 ? f1 : 0) + (grp > 2 ? f2 : 0);
            bool again = false;
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                if (!__ballot(fin[s])) continue;
                if (fin[s]) {
                    const int ri = goff + rank[s];  // candidate cbeg + ri
                    const uint4 e = ring[ri & (kRing - 1)];
                    const int q = ri < nrel ? (int)e.x : -1;
                    float lim = q == bq ? bv : INFINITY;
                    if (q == cur_q) lim = fminf(lim, lk);
                    const uint32_t pos = q >= 0 ? e.y : 0u;
                    sq[s] = q;
                    spos[s] = pos;
                    sc[s] = 0;
                    sd[s] = Dist<F>{};
                    sthr[s] = lim;
                    xp[s] = ix.rows + (int64_t)pos * ix.stride + sub * 4;
                    qp[s] = ws.qrow + (int64_t)max(q, 0) * ix.stride + sub * 4;
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

        // one chunk of every slot's series; empty slots read chunk 0 of row 0
        float4 x[NS], qv[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            x[s] = *reinterpret_cast<const float4*>(xp[s] + sc[s] * kChunk);
            qv[s] = *reinterpret_cast<const float4*>(qp[s] + sc[s] * kChunk);
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
                const bool over = sd[s].value() > sthr[s];
                fin[s] = over || sc[s] == nchunks;
                adm[s] = fin[s] && !over;
                slow = slow || adm[s] || (fin[s] && sq[s] != st_q);
            }
        }
        if (has_pend) {
            ring[((int)(mb + 64 - cbeg) & (kRing - 1)) + lane] = ring_entry(pend);
            has_pend = false;
        }

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
                    const float v = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(sd[s].value()), 16 * g));
                    const uint32_t kp = (uint32_t)__builtin_amdgcn_readlane(spos[s], 16 * g);
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
            if (new_q != cur_q) pub = INFINITY;
            if (new_q >= 0 && topn == k) {
                const uint32_t kb = (uint32_t)(top[k - 1] >> 32);
                new_lk = bits_to_float(kb);
                // BSF_k only decreases: every improvement of this wavefront's
                // k-th distance is published, without reading the global value
                // back (a load here would hold up the next round)
                if (new_lk < pub) {
                    atomicMin(&ws.bsf[new_q], kb);
                    pub = new_lk;
                }
            }
        }
        cur_q = __shfl(new_q, 0, 64);
        lk = __shfl(new_lk, 0, 64);
#pragma unroll
        for (int s = 0; s < NS; ++s)
            if (sq[s] == cur_q) sthr[s] = fminf(sthr[s], lk);
    }
    if (lane == 0) flush_topk(ws, cur_q, k, top, topn);
    flush_counters();
}

}  // namespace

hipError_t launch_refine(const IndexView& ix, const ScanParams& sp, const QueryWs& ws, int device_cus, int form,
                         hipStream_t st) {
#define HS_REFINE(FF, NS) \
    k_refine<FF, NS><<<dim3(resident_grid(k_refine<FF, NS>, kTile, 0, device_cus)), dim3(kTile), 0, st>>>(ix, sp, ws)
    if (form == kComp) HS_REFINE(kComp, kRefineSlots);
    else HS_REFINE(kPlain, kRefineSlots);
#undef HS_REFINE
    return hipGetLastError();
}

}  // namespace hs
