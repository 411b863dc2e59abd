// Refinement of the candidate list (Hercules Sec. 3.4, step 4): the exact
// float32 squared distance with early abandoning for every candidate, first
// re-checked against the current BSF_k; per-wavefront top-k, BSF_k published
// with atomicMin, results appended to the per-query pool.
//
// Every wavefront owns a contiguous range of the candidate list (regions are
// ordered by query, so a range holds long runs of one query) and never waits
// for another wavefront: the metadata of its next 4 NC candidates is loaded
// while the current ones are refined, each 16-lane group refines NC series at
// a time (CB 64-point chunks of each loaded together), and the admitted
// results reach lane 0 by shuffles; lane 0 alone keeps the wavefront's top-k
// in LDS.
#include "hs_device.h"

namespace hs {
namespace {

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

// Candidate c of the list; lanes 0..15 call this for c = base + lane.  The
// lane keeps its slice's first entry and end in registers: only a step across
// a slice end loads the prefix again.
struct SliceCursor {
    int s = 0;
    long long begin = 0, end = 0;
};

__device__ __forceinline__ Meta load_meta(const QueryWs& ws, long long c, long long cend, SliceCursor& cur) {
    Meta m{-1, 0u, 0.0f};
    if (c < cend) {
        if (c >= cur.end) {
            cur.s = slice_of(ws, c, cur.s);
            cur.begin = ws.slice_start[cur.s];
            cur.end = ws.slice_start[cur.s + 1];
        }
        const long long e = (long long)cur.s * ws.slice_cap + (c - cur.begin);
        m.q = (int)ws.slice_q[e];
        m.pos = ws.slice_pos[e];
        m.lb = ws.slice_lb[e];
    }
    return m;
}

// F: distance form.  NC: series in flight per 16-lane group; CB: 64-point
// chunks loaded together per series between two abandoning checks.
template <int F, int NC, int CB>
__global__ void __launch_bounds__(256) k_refine(IndexView ix, ScanParams sp, QueryWs ws) {
    constexpr int kStep = 4 * NC;  // candidates per wavefront step: 4 groups x NC
    __shared__ unsigned long long s_top[kTile / 64][HS_KMAX];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6, sub = t & 15, grp = (t >> 4) & 3;
    const int k = sp.k;
    const int nchunks = ix.stride / kChunk;
    const long long T = ws.slice_start[ws.n_slices + 1];
    const long long gw = (long long)blockIdx.x * (kTile / 64) + wave, GW = (long long)gridDim.x * (kTile / 64);
    const long long cbeg = T * gw / GW, cend = T * (gw + 1) / GW;
    unsigned long long* top = s_top[wave];

    // wavefront state, uniform: the query of the top-k and its k-th distance
    int cur_q = -1;
    float lk = INFINITY;
    int topn = 0;                                     // lane 0
    float pub = INFINITY;                             // lane 0: k-th distance last published for cur_q
    int st_q = -1;                                    // lane 0: counters of st_q
    unsigned long long st_ref = 0, st_ch = 0;

    SliceCursor cur;  // lane's slice (end 0: found on the first load)
    Meta m = lane < kStep ? load_meta(ws, cbeg + lane, cend, cur) : Meta{-1, 0u, 0.0f};
    float mb = m.q >= 0 ? bits_to_float(load_relaxed(&ws.bsf[m.q])) : 0.0f;
    for (long long cb = cbeg; cb < cend; cb += kStep) {
        // next step's metadata in flight while this step is refined
        const Meta nm = lane < kStep ? load_meta(ws, cb + kStep + lane, cend, cur) : Meta{-1, 0u, 0.0f};

        unsigned long long res[NC];  // admitted keys of this group (group-uniform), ~0 = none
        int resq[NC];
        unsigned chs[NC];            // chunks read per candidate (0: not refined)
        float nmb = 0.0f;           // next step's BSF_k, loaded behind this step's first rows
        {
            int q[NC];
            uint32_t pos[NC];
            float thr[NC];
            Dist<F> d[NC];
            bool alive[NC], refined[NC];
            unsigned ch[NC];
#pragma unroll
            for (int j = 0; j < NC; ++j) {
                const int src = grp * NC + j;
                q[j] = __shfl(m.q, src, 64);
                pos[j] = __shfl(m.pos, src, 64);
                const float lb = __shfl(m.lb, src, 64);
                thr[j] = __shfl(mb, src, 64);
                if (q[j] == cur_q) thr[j] = fminf(thr[j], lk);
                refined[j] = q[j] >= 0 && (double)lb <= prune_limit(thr[j]);
                alive[j] = refined[j];
                ch[j] = 0u;
            }
            for (int c = 0; c < nchunks; c += CB) {
                float4 x[NC][CB];
#pragma unroll
                for (int j = 0; j < NC; ++j) {
                    if (alive[j]) {
                        const float* xr = ix.rows + (int64_t)pos[j] * ix.stride + sub * 4 + c * kChunk;
#pragma unroll
                        for (int b = 0; b < CB; ++b)
                            x[j][b] = c + b < nchunks ? *reinterpret_cast<const float4*>(xr + b * kChunk)
                                                      : make_float4(0.f, 0.f, 0.f, 0.f);
                    }
                }
                if (c == 0 && nm.q >= 0) nmb = bits_to_float(load_relaxed(&ws.bsf[nm.q]));
                // the group's candidates almost always share a query: its chunks are
                // loaded once and reloaded only for a candidate of another query
                const float* q0 = ws.qrow + (int64_t)q[0] * ix.stride + sub * 4 + c * kChunk;
                float4 qa[CB];
#pragma unroll
                for (int b = 0; b < CB; ++b)
                    qa[b] = (q[0] >= 0 && c + b < nchunks) ? *reinterpret_cast<const float4*>(q0 + b * kChunk)
                                                          : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
                for (int j = 0; j < NC; ++j) {
                    if (alive[j]) {
                        const float* qr = ws.qrow + (int64_t)q[j] * ix.stride + sub * 4 + c * kChunk;
#pragma unroll
                        for (int b = 0; b < CB; ++b) {
                            if (c + b < nchunks) {
                                const float4 a = q[j] != q[0] ? *reinterpret_cast<const float4*>(qr + b * kChunk) : qa[b];
                                d[j].add(a, x[j][b]);
                                ch[j] += 1u;
                            }
                        }
                        if (d[j].value() > thr[j]) alive[j] = false;
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < NC; ++j) {
                chs[j] = refined[j] ? ch[j] : 0u;
                res[j] = (refined[j] && alive[j]) ? (((unsigned long long)__float_as_uint(d[j].value()) << 32) | ix.ids[pos[j]])
                                                  : ~0ull;
                resq[j] = q[j];
            }
        }

        // lane 0 takes the 4 groups' results and counters one by one
        int new_q = cur_q;
        float new_lk = lk;
#pragma unroll
        for (int i = 0; i < kStep; ++i) {
            const unsigned long long key = __shfl(res[i % NC], (i / NC) * 16, 64);
            const int kq = __shfl(resq[i % NC], (i / NC) * 16, 64);
            const unsigned kch = __shfl(chs[i % NC], (i / NC) * 16, 64);
            if (lane == 0) {
                if (key != ~0ull) {
                    if (kq != new_q) {
                        flush_topk(ws, new_q, k, top, topn);
                        new_q = kq;
                        topn = 0;
                    }
                    topk_insert(top, topn, k, key);
                }
                if (kch) {  // counters, one update per change of query
                    if (kq != st_q) {
                        if (st_q >= 0) {
                            atomicAdd(&ws.stats[(int64_t)st_q * 8 + 2], st_ref);
                            atomicAdd(&ws.stats[(int64_t)st_q * 8 + 3], st_ch);
                        }
                        st_q = kq;
                        st_ref = st_ch = 0;
                    }
                    st_ref += 1;
                    st_ch += kch;
                }
            }
        }
        if (lane == 0) {
            new_lk = INFINITY;
            if (new_q != cur_q) pub = INFINITY;
            if (new_q >= 0 && topn == k) {
                const uint32_t kb = (uint32_t)(top[k - 1] >> 32);
                new_lk = bits_to_float(kb);
                // BSF_k only decreases: every improvement of this wavefront's
                // k-th distance is published, without reading the global value
                // back (a load here would hold up the next step)
                if (new_lk < pub) {
                    atomicMin(&ws.bsf[new_q], kb);
                    pub = new_lk;
                }
            }
        }
        cur_q = __shfl(new_q, 0, 64);
        lk = __shfl(new_lk, 0, 64);
        m = nm;
        mb = nmb;
    }
    if (lane == 0) {
        flush_topk(ws, cur_q, k, top, topn);
        if (st_q >= 0) {
            atomicAdd(&ws.stats[(int64_t)st_q * 8 + 2], st_ref);
            atomicAdd(&ws.stats[(int64_t)st_q * 8 + 3], st_ch);
        }
    }
}

}  // namespace

hipError_t launch_refine(const IndexView& ix, const ScanParams& sp, const QueryWs& ws, int device_cus, int form,
                         hipStream_t st) {
    // series of at least 256 points: two in flight per group, four chunks
    // (1 KB of a row) per load; shorter series: four in flight, two chunks
#define HS_REFINE(FF, NC, CB) \
    k_refine<FF, NC, CB><<<dim3(resident_grid(k_refine<FF, NC, CB>, kTile, 0, device_cus)), dim3(kTile), 0, st>>>(ix, sp, ws)
    const bool wide = ix.stride >= 4 * kChunk;
    if (form == kComp) {
        if (wide) HS_REFINE(kComp, 2, 4);
        else HS_REFINE(kComp, 4, 2);
    } else {
        if (wide) HS_REFINE(kPlain, 2, 4);
        else HS_REFINE(kPlain, 4, 2);
    }
#undef HS_REFINE
    return hipGetLastError();
}

}  // namespace hs
