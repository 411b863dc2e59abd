// Refinement of the candidate list (Hercules Sec. 3.4, step 4): the exact
// float32 squared distance with early abandoning for every candidate, first
// re-checked against the current BSF_k; per-wavefront top-k, BSF_k published
// with atomicMin, results appended to the per-query pool.
//
// Every wavefront owns a contiguous range of the candidate list (regions are
// ordered by query, so a range holds long runs of one query) and never waits
// for another wavefront: the metadata of its next 16 candidates is loaded
// while the current ones are refined, each 16-lane group refines four series
// at a time (their next two 64-point chunks loaded together), and the
// admitted results reach lane 0 by shuffles; lane 0 alone keeps the
// wavefront's top-k in LDS.
#include "hs_device.h"

namespace hs {
namespace {

constexpr int kStep = 16;  // candidates per wavefront step: 4 groups x 4

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

template <int F>
__global__ void __launch_bounds__(256) k_refine(IndexView ix, ScanParams sp, QueryWs ws) {
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
    int st_q = -1;                                    // lane 0: counters of st_q
    unsigned long long st_ref = 0, st_ch = 0;

    SliceCursor cur;  // lane's slice (end 0: found on the first load)
    Meta m = lane < kStep ? load_meta(ws, cbeg + lane, cend, cur) : Meta{-1, 0u, 0.0f};
    float mb = m.q >= 0 ? bits_to_float(load_relaxed(&ws.bsf[m.q])) : 0.0f;
    for (long long cb = cbeg; cb < cend; cb += kStep) {
        // next step's metadata in flight while this step is refined
        const Meta nm = lane < kStep ? load_meta(ws, cb + kStep + lane, cend, cur) : Meta{-1, 0u, 0.0f};

        unsigned long long res[4];  // admitted keys of this group (group-uniform), ~0 = none
        int resq[4];
        unsigned chs[4];            // chunks read per candidate (0: not refined)
        float nmb = 0.0f;           // next step's BSF_k, loaded behind this step's first rows
        {
            int q[4];
            uint32_t pos[4];
            float thr[4];
            Dist<F> d[4];
            bool alive[4], refined[4];
            unsigned ch[4] = {0u, 0u, 0u, 0u};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int src = grp * 4 + j;
                q[j] = __shfl(m.q, src, 64);
                pos[j] = __shfl(m.pos, src, 64);
                const float lb = __shfl(m.lb, src, 64);
                thr[j] = __shfl(mb, src, 64);
                if (q[j] == cur_q) thr[j] = fminf(thr[j], lk);
                refined[j] = q[j] >= 0 && (double)lb <= prune_limit(thr[j]);
                alive[j] = refined[j];
            }
            for (int c = 0; c < nchunks; c += 2) {
                const bool two = c + 1 < nchunks;
                float4 x0[4], x1[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (alive[j]) {
                        const float* xr = ix.rows + (int64_t)pos[j] * ix.stride + sub * 4 + c * kChunk;
                        x0[j] = *reinterpret_cast<const float4*>(xr);
                        x1[j] = two ? *reinterpret_cast<const float4*>(xr + kChunk) : make_float4(0.f, 0.f, 0.f, 0.f);
                    }
                }
                if (c == 0 && nm.q >= 0) nmb = bits_to_float(load_relaxed(&ws.bsf[nm.q]));
                // the group's candidates almost always share a query: its chunks are
                // loaded once and reloaded only for a candidate of another query
                const float* q0 = ws.qrow + (int64_t)q[0] * ix.stride + sub * 4 + c * kChunk;
                float4 qa = make_float4(0.f, 0.f, 0.f, 0.f), qb = qa;
                if (q[0] >= 0) {
                    qa = *reinterpret_cast<const float4*>(q0);
                    if (two) qb = *reinterpret_cast<const float4*>(q0 + kChunk);
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (alive[j]) {
                        float4 a = qa, b = qb;
                        if (q[j] != q[0]) {
                            const float* qr = ws.qrow + (int64_t)q[j] * ix.stride + sub * 4 + c * kChunk;
                            a = *reinterpret_cast<const float4*>(qr);
                            if (two) b = *reinterpret_cast<const float4*>(qr + kChunk);
                        }
                        d[j].add(a, x0[j]);
                        if (two) d[j].add(b, x1[j]);
                        ch[j] += two ? 2u : 1u;
                        if (d[j].value() > thr[j]) alive[j] = false;
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
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
        for (int i = 0; i < 16; ++i) {
            const unsigned long long key = __shfl(res[i & 3], (i >> 2) * 16, 64);
            const int kq = __shfl(resq[i & 3], (i >> 2) * 16, 64);
            const unsigned kch = __shfl(chs[i & 3], (i >> 2) * 16, 64);
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
            if (new_q >= 0 && topn == k) {
                const uint32_t kb = (uint32_t)(top[k - 1] >> 32);
                new_lk = bits_to_float(kb);
                if (new_lk < bits_to_float(load_relaxed(&ws.bsf[new_q]))) atomicMin(&ws.bsf[new_q], kb);
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
    if (form == kComp)
        k_refine<kComp><<<dim3(resident_grid(k_refine<kComp>, kTile, 0, device_cus)), dim3(kTile), 0, st>>>(ix, sp, ws);
    else
        k_refine<kPlain><<<dim3(resident_grid(k_refine<kPlain>, kTile, 0, device_cus)), dim3(kTile), 0, st>>>(ix, sp, ws);
    return hipGetLastError();
}

}  // namespace hs
