// Precision form of the query path.  It computes the same exact k-NN as the
// plain method (Hercules Sec. 3.4); only the per-series filter changes.  A
// bf16 or fp16 copy x~ of every stored series feeds a matrix-core pass that
// computes q~.x~ for every (query, series) pair of the candidate leaves, in
// float32.  From it a rigorous lower bound of the true squared distance
// follows (triangle inequality plus the accumulation error bound):
//
//   sqrt(d(q, x)) >= sqrt(d(q~, x~)) - eps_q - eps_x,   eps = ||v - v~||_2
//   d(q~, x~) = ||q~||^2 + ||x~||^2 - 2 q~.x~
//            >= (1 - g) (||q~||^2 + ||x~||^2) - 2 acc,  |acc - q~.x~| <= g ||q~|| ||x~||
//
// with g = K u' / (1 - K u'), K the accumulation length and u' = 2^-23 (twice
// the float32 unit roundoff, so any rounding of the matrix core's additions is
// covered; bf16 x bf16 and fp16 x fp16 products are exact in float32) and
// 2 ||q~|| ||x~|| <= ||q~||^2 + ||x~||^2.  A pair is dropped only when that
// bound exceeds BSF_k (1 + slack); a float32 test with proven margins discards
// the clear cases, every pair it keeps is decided in float64, and the float64
// bound travels with the candidate to the refinement (compensated float32).
#include <algorithm>

#include "hs_device.h"

namespace hs {
namespace {

typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

constexpr int kKBlock = 256;           // K elements staged per block
constexpr int kKSteps = kKBlock / 16;  // 32x32x16 steps per block
constexpr int kLdsRow = kKBlock + 8;   // 16-bit elements per staged row (padded against bank conflicts)

template <int KIND>
struct Low;

template <>
struct Low<kShadowBf16> {
    typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 v8;
    static __device__ __forceinline__ uint16_t encode(float v) {  // round to nearest even (finite v)
        const uint32_t b = __float_as_uint(v);
        return (uint16_t)((b + 0x7fffu + ((b >> 16) & 1u)) >> 16);
    }
    static __device__ __forceinline__ float decode(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
    // the smallest bf16 value >= v (finite v; truncation moves a negative value up)
    static __device__ __forceinline__ uint16_t encode_up(float v) {
        const uint32_t b = __float_as_uint(v);
        return (uint16_t)((b >> 16) + (((b & 0xffffu) != 0u && !(b >> 31)) ? 1u : 0u));
    }
    static __device__ __forceinline__ bool representable(float) { return true; }
    static __device__ __forceinline__ f32x16 mma(uint4 a, uint4 b, f32x16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(v8, a), __builtin_bit_cast(v8, b), c, 0, 0,
                                                      0);
    }
};

template <>
struct Low<kShadowF16> {
    typedef __attribute__((__vector_size__(8 * sizeof(_Float16)))) _Float16 v8;
    static __device__ __forceinline__ uint16_t encode(float v) { return __builtin_bit_cast(uint16_t, (_Float16)v); }
    static __device__ __forceinline__ float decode(uint16_t h) { return (float)__builtin_bit_cast(_Float16, h); }
    // the smallest fp16 value >= v (finite v; +inf past the range)
    static __device__ __forceinline__ uint16_t encode_up(float v) {
        uint16_t h = encode(v);
        if (decode(h) < v) h = h == 0x8000u ? (uint16_t)1u : (h & 0x8000u ? (uint16_t)(h - 1u) : (uint16_t)(h + 1u));
        return h;
    }
    static __device__ __forceinline__ bool representable(float v) { return fabsf(v) <= 65504.0f; }
    static __device__ __forceinline__ f32x16 mma(uint4 a, uint4 b, f32x16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(v8, a), __builtin_bit_cast(v8, b), c, 0, 0,
                                                     0);
    }
};

// Constants of the float32 test.
struct BoundConsts {
    double g;   // accumulation factor g (plus 2^-40 for the float64 norms)
    double m;   // margin factor 3u of the folded constants (u = 2^-24)
    double g2;  // accumulation factor of K + 2 products (the augmented step, series of <= 256 points)
};

// The constants for series of stride K: g for K float32 additions at twice the
// unit roundoff (plus 2^-40 for the float64 norms), m = 3u, g2 for K + 2.
BoundConsts bound_consts(int K) {
    const double u2 = std::ldexp(1.0, -23), Kd = (double)K, K2 = Kd + 2.0;
    return BoundConsts{Kd * u2 / (1.0 - Kd * u2) + std::ldexp(1.0, -40), 3.0 * std::ldexp(1.0, -24),
                       K2 * u2 / (1.0 - K2 * u2) + std::ldexp(1.0, -40)};
}

// The augmented unit of a series for the bounding pass of series of at most
// 256 points.  The matrix cores add a* x 1 + ebar x sTbar to q~.x~, with
// ebar >= eps_x and sTbar >= sT rounded up to the low precision, and
// a* >= -B0 + g2 R, B0 = (||x~||^2 - eps_x^2) / 2 (from the stored values,
// so at most the true one) and R >= ||x~||^2 / 2 + |a*| + ebar^2 / 2 the
// series' share of the accumulation error bound of the K + 2 products.
// Returned as the two low-precision bit patterns (a* low half, ebar high).
template <int KIND>
__device__ __forceinline__ uint32_t augmented_unit(float xn, float eps, const BoundConsts& bc) {
    const uint16_t eb = Low<KIND>::encode_up(eps);
    const double ebar = (double)Low<KIND>::decode(eb), xd = xn;
    const double B0 = 0.5 * (xd - (double)eps * (double)eps);
    // |a*| <= |B0| + g2 R_0 before rounding; twice that covers the rounding
    const double R = 0.5 * xd * (1.0 + 0x1p-38) + 2.0 * (fabs(B0) + bc.g2 * (xd + 2.0 * fabs(B0) + ebar * ebar)) +
                     0.5 * ebar * ebar;
    const double v = -B0 + bc.g2 * R;
    const float av = __double2float_ru(v + fabs(v) * 0x1p-20 + 1e-30);  // >= v whatever its sign
    return (uint32_t)Low<KIND>::encode_up(av) | ((uint32_t)eb << 16);
}

// beta_x of the float32 test from the stored ||x~||^2 and eps_x (float64,
// lowered by 3u M_x, rounded down).
__device__ __forceinline__ float beta_of(float xn, float eps, const BoundConsts& bc) {
    const double xd = xn, ed = eps;
    return __double2float_rd(0.5 * ((1.0 - bc.g) * xd - ed * ed) - bc.m * (xd + ed * ed));
}

// One wavefront per series: the low-precision copy and, in float64,
// ||x~||^2 (stored rounded down), ||x - x~||_2 (stored rounded up) and beta_x.
template <int KIND>
__global__ void __launch_bounds__(256) k_shadow(IndexView ix, int64_t nrows, uint16_t* __restrict__ out,
                                                float4* __restrict__ norms, uint32_t* __restrict__ bad,
                                                BoundConsts bc) {
    const int lane = threadIdx.x & 63;
    const int64_t w0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t r = w0; r < nrows; r += nw) {
        const float* xr = ix.rows + r * ix.stride;
        uint16_t* orow = out + r * ix.stride;
        double s2 = 0.0, e2 = 0.0;
        bool ok = true;
        for (int j = lane; j < ix.stride; j += 64) {
            const float v = xr[j];
            ok = ok && Low<KIND>::representable(v);
            const uint16_t h = Low<KIND>::encode(v);
            const double lv = (double)Low<KIND>::decode(h);
            orow[j] = h;
            s2 += lv * lv;
            const double e = (double)v - lv;
            e2 += e * e;
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            s2 += __shfl_xor(s2, o, 64);
            e2 += __shfl_xor(e2, o, 64);
        }
        if (__ballot(!ok) != 0ull && lane == 0) atomicOr(bad, 1u);
        // float64 sums carry a relative error below 2^-40 for any stride the
        // index accepts; the factors push the stored values past it
        if (lane == 0) {
            const float xn = __double2float_rd(s2 * (1.0 - 0x1p-40));
            const float eps = __double2float_ru(sqrt(e2) * (1.0 + 0x1p-40));
            norms[r] = make_float4(beta_of(xn, eps, bc), eps, xn, __uint_as_float(augmented_unit<KIND>(xn, eps, bc)));
        }
    }
}

__global__ void k_empty_slices(QueryWs ws, int32_t slice0, int32_t slices) {
    for (int e = threadIdx.x; e < slices; e += blockDim.x) ws.slice_cnt[slice0 + e] = 0;
}

// One wavefront per (padded) query: q~, ||q~||^2 and ||q - q~||_2 in float64.
template <int KIND>
__global__ void __launch_bounds__(64) k_query_low(IndexView ix, int32_t Q, QueryWs ws) {
    const int q = blockIdx.x, lane = threadIdx.x;
    uint16_t* orow = ws.qlow + (int64_t)q * ix.stride;
    if (q >= Q) {
        for (int j = lane; j < ix.stride; j += 64) orow[j] = 0;
        return;
    }
    const float* qr = ws.qrow + (int64_t)q * ix.stride;
    double s2 = 0.0, e2 = 0.0;
    bool ok = true;
    for (int j = lane; j < ix.stride; j += 64) {
        const float v = qr[j];
        ok = ok && Low<KIND>::representable(v);
        const uint16_t h = Low<KIND>::encode(v);
        const double lv = (double)Low<KIND>::decode(h);
        orow[j] = h;
        s2 += lv * lv;
        const double e = (double)v - lv;
        e2 += e * e;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        s2 += __shfl_xor(s2, o, 64);
        e2 += __shfl_xor(e2, o, 64);
    }
    // a query outside the fp16 range is reported like a non-finite one
    if (__ballot(!ok) != 0ull && lane == 0 && !(ws.flags[q] & kFlagNonFinite)) {
        ws.flags[q] |= kFlagNonFinite;
        atomicAdd(&ws.counters[kCtrNonFinite], 1u);
    }
    if (lane == 0) ws.qnorm[q] = make_double2(s2 * (1.0 - 0x1p-40), sqrt(e2) * (1.0 + 0x1p-40));
}

// Per part of the copy: the queries whose LB_EAPCA of the part's leaf does
// not exceed their BSF_k (1 + slack), in query order, and the number of
// kBoundQueries-query blocks (work items of the bounding pass) they make.
__global__ void __launch_bounds__(256) k_part_lists(IndexView ix, ScanParams sp, QueryWs ws) {
    __shared__ int s_w[kTile / 64];
    const int64_t p = blockIdx.x;
    const int t = threadIdx.x;
    const int64_t leaf = ix.part_leaf[p];
    uint32_t* list = ws.plist + p * (int64_t)sp.Q;
    int base = 0;
    for (int q0 = 0; q0 < sp.Q; q0 += blockDim.x) {
        const int q = q0 + t;
        bool k = false;
        if (q < sp.Q && !(ws.flags[q] & kFlagNonFinite))
            k = (double)ws.lbe[(int64_t)q * ix.L + leaf] <= prune_limit(bits_to_float(bsf_bits(ws, q)));
        int tot;
        const int off = block_exclusive_scan(k ? 1 : 0, s_w, &tot);
        if (k) list[base + off] = (uint32_t)q;
        base += tot;
    }
    if (t == 0) {
        ws.pcnt[p] = (uint32_t)base;
        ws.pnb[p] = (uint32_t)((base + kBoundQueries - 1) / kBoundQueries);
    }
}

// The bounding pass.  Workgroup = 4 wavefronts x 32 queries: a block of the
// queries that keep one part (a part lies in one leaf); it walks the part in
// tiles of 32 series.  Per tile and K-block the 32 x 256 low-precision series are
// staged in LDS (double buffered: the next stage's global loads are in flight
// during this stage's matrix-core steps).  Every wavefront computes the 32 x 32 block
// acc[series][query] with 16 v_mfma 32x32x16 steps; its query fragments stay
// in registers when the series fit one K-block.
//
// Output layout of the 32x32 block: lane l holds query (l mod 32) and, in
// accumulator r, series 8 (r / 4) + 4 (l / 32) + (r mod 4).
//
// Float32 test.  With sT = sqrt(BSF_k (1 + slack)) + eps_q (rounded up), the
// pair is dropped iff (1 - g)(||q~||^2 + ||x~||^2) - 2 acc > (sT + eps_x)^2,
// i.e. iff acc - beta_x + sT eps_x < alpha_q with
//   alpha_q = ((1 - g)||q~||^2 - sT^2) / 2,  beta_x = ((1 - g)||x~||^2 - eps_x^2) / 2.
// alpha and beta are computed in float64, lowered by 3u M_q and 3u M_x
// (M_q = ||q~||^2 + sT^2, M_x = ||x~||^2 + eps_x^2, u = 2^-24) and rounded
// down.  e = fma(sT, eps_x, acc - beta) carries two float32 roundings, at most
// 2u (M_q + M_x) in all (|acc| <= (||q~||^2 + ||x~||^2) / 2 (1 + g),
// sT eps_x <= (sT^2 + eps_x^2) / 2), below the margin; so e < alpha implies
// the exact condition.  A lane first takes the largest e of its 16 pairs
// (3 operations per pair); only when it reaches alpha are the pairs tested
// one by one and decided in float64.
//
// Series of at most 256 points (ONE) fold the series' terms into the matrix
// cores: one more step adds a* x 1 + ebar x sTbar (the augmented unit), so
// acc >= q~.x~ + a* + eps_x sT up to the error of K + 2 products, at most
// g2 (Q_q + R_x) with Q_q = ||q~||^2 / 2 (1 + 2^-38) + sTbar^2 / 2 in alpha and
// R_x in a*.  Then acc < alpha with
//   alpha_q = (||q~||^2 - sT^2) / 2 - g2 Q_q - 2^-40 (||q~||^2 + sT^2)
// implies the exact condition, and the per-lane test is a max over the 16
// accumulators.  The float64 decision subtracts a* and ebar sTbar again and
// takes the accumulation bound g2 S of the K + 2 products.
template <int KIND, bool ONE>
__global__ void __launch_bounds__(256) k_bound(IndexView ix, ShadowView sv, ScanParams sp, QueryWs ws,
                                               BoundConsts bc) {
#pragma clang fp contract(off)
    __shared__ __attribute__((aligned(16))) uint16_t s_tile[2][kBoundRows * kLdsRow];
    __shared__ float2 s_norm[2][kBoundRows];  // (beta', eps_x) per staged series
    __shared__ float s_xn[2][kBoundRows];     // ||x~||^2 per staged series
    __shared__ float2 s_aug[2][kBoundRows];   // ONE: (a*, ebar) per staged series, decoded
    __shared__ float s_acc[kTile / 64][16 * 64];  // per wavefront: its accumulators, on the rare float64 path
    __shared__ int s_item;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6, j = lane & 31, half = lane >> 5;
    // ONE: the series fit one K-block (stride <= 256) and the query fragments stay in registers
    const int K = ix.stride, nkb = ONE ? 1 : (K + kKBlock - 1) / kKBlock;
    const uint64_t lt_mask = (1ull << lane) - 1ull;

    const int64_t slice = (int64_t)sp.slice0 + (int64_t)blockIdx.x * (kTile / 64) + wave;
    uint32_t* spos = ws.slice_pos + slice * ws.slice_cap;
    uint32_t* sq = ws.slice_q + slice * ws.slice_cap;
    uint32_t* spart = ws.slice_part + slice * ws.slice_cap;
    uint32_t cnt = 0;  // entries in this wavefront's slice (uniform)
    // slices of wavefronts beyond this grid stay empty
    for (int64_t e = (int64_t)gridDim.x * (kTile / 64) + (int64_t)blockIdx.x * kTile + t; e < sp.slices;
         e += (int64_t)gridDim.x * kTile)
        ws.slice_cnt[sp.slice0 + e] = 0;

    // Work items (part p, block b): the queries of p's list (every query whose
    // LB_EAPCA of p's leaf does not exceed its BSF_k) are cut into blocks of
    // kBoundQueries, 32 per wavefront; items are dealt from one counter in
    // part order, so the blocks of a part run about together.  A part's rows
    // are staged once per block: with at most kBoundQueries queries keeping a
    // leaf, once per batch.
    const uint32_t nitems = ws.pbo[sv.parts_n];
    for (;;) {
        __syncthreads();  // every wave has read s_item
        if (t == 0) s_item = (int)atomicAdd(&ws.counters[kCtrBound], 1u);
        __syncthreads();
        const uint32_t it = (uint32_t)s_item;
        if (it >= nitems) break;
        // the part of the item: the last p with pbo[p] <= it
        int64_t plo = 0, phi = sv.parts_n - 1;
        while (plo < phi) {
            const int64_t mid = (plo + phi + 1) >> 1;
            if (ws.pbo[mid] <= it) plo = mid;
            else phi = mid - 1;
        }
        const int64_t p = plo;
        const uint32_t lq = (it - ws.pbo[p]) * kBoundQueries + (uint32_t)(wave * 32 + j);
        {
            // lanes past the part's list read query 0's copy; their results are masked
            const bool qvalid = lq < ws.pcnt[p];
            const int qj = qvalid ? (int)ws.plist[p * (int64_t)sp.Q + lq] : 0;
            float alpha = -3.0e38f, sT = 0.0f, sTb = 0.0f, bsf_j = 0.0f;
            uint4 bq_aug = make_uint4(0, 0, 0, 0);  // ONE: (1, sTbar) at k = 256, 257 (half 0)
            if (qvalid) {
                const double2 qn = ws.qnorm[qj];
                bsf_j = bits_to_float(bsf_bits(ws, qj));
                const double T = prune_limit(bsf_j);
                if (T < 1e300) {  // no BSF_k yet: every pair passes the float32 test
                    sT = __double2float_ru((sqrt(T) + qn.y) * (1.0 + 0x1p-40));
                    const double s2 = (double)sT * (double)sT;
                    if (ONE) {
                        // acc = q~.x~ + a* + ebar sTbar (K + 2 products); the
                        // query's share of their error bound lowers alpha
                        const uint16_t sb = Low<KIND>::encode_up(sT);
                        sTb = Low<KIND>::decode(sb);
                        const double Qs = 0.5 * qn.x * (1.0 + 0x1p-38) + 0.5 * (double)sTb * (double)sTb;
                        alpha = __double2float_rd(0.5 * (qn.x - s2) - bc.g2 * Qs - 0x1p-40 * (qn.x + s2));
                        bq_aug.x = half == 0 ? ((uint32_t)Low<KIND>::encode(1.0f) | ((uint32_t)sb << 16)) : 0u;
                    } else {
                        alpha = __double2float_rd(0.5 * ((1.0 - bc.g) * qn.x - s2) - bc.m * (qn.x + s2));
                    }
                } else if (ONE) {
                    bq_aug.x = half == 0 ? (uint32_t)Low<KIND>::encode(1.0f) : 0u;
                }
            }
            const uint16_t* qlow = ws.qlow + (int64_t)qj * K + 8 * half;
            uint4 bq[kKSteps];
            if (ONE) {
#pragma unroll
                for (int u = 0; u < kKSteps; ++u)
                    bq[u] = u * 16 < K ? *reinterpret_cast<const uint4*>(qlow + u * 16) : make_uint4(0, 0, 0, 0);
            }
            unsigned long long tested = 0, cands = 0, staged = 0;  // staged: pairs the matrix cores evaluated
            bool lost = false;

            {
                const int64_t ps = ix.part_start[p], pe = ix.part_start[p + 1];
                const bool keep = qvalid;  // every listed query keeps the part's leaf
                const bool wkeep = __ballot(keep) != 0ull;
                const int64_t ntiles = (pe - ps + kBoundRows - 1) / kBoundRows;
                const int64_t nst = ntiles * nkb;

                // stage s: tile s / nkb, K-block s % nkb.  Thread t moves uint4
                // number t + 256 i (i < 4) of the 32 x 256 block: row (that / 32),
                // 8-element column (that % 32); rows past the collection are
                // clamped (their results are masked).
                uint4 pa[4];
                float4 na = make_float4(0.f, 0.f, 0.f, 0.f);
                auto stage_load = [&](int64_t s, uint4 (&pre)[4], float4& pn) {
                    // branch-free, from the tile's first row (the copy is padded by
                    // a tile, so no row clamp); columns past K read other values of
                    // the copy that are zeroed when stored
                    const int64_t tr0 = ps + (s / nkb) * kBoundRows;
                    const int kb = (int)(s % nkb);
                    const uint16_t* base = sv.rows + tr0 * K;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int e = t + 256 * i, cc = (e & 31) * 8 + kb * kKBlock;
                        pre[i] = *reinterpret_cast<const uint4*>(base + ((e >> 5) * K + min(cc, K - 8)));
                    }
                    pn = sv.norms[tr0 + (t & (kBoundRows - 1))];
                };
                auto stage_store = [&](int64_t s, const uint4 (&pre)[4], float4 pn) {
                    uint16_t* dst = s_tile[s & 1];
                    const int kb = (int)(s % nkb);
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int e = t + 256 * i, rr = e >> 5, cc = (e & 31) * 8;
                        *reinterpret_cast<uint4*>(dst + rr * kLdsRow + cc) =
                            cc + kb * kKBlock < K ? pre[i] : make_uint4(0, 0, 0, 0);
                    }
                    if (kb == 0 && t < kBoundRows) {
                        s_norm[(s / nkb) & 1][t] = make_float2(pn.x, pn.y);
                        s_xn[(s / nkb) & 1][t] = pn.z;
                        if (ONE) {
                            // the series' augmented unit in its row's padding: (a*, ebar, 0, ...)
                            const uint32_t au = __float_as_uint(pn.w);
                            *reinterpret_cast<uint4*>(dst + t * kLdsRow + kKBlock) = make_uint4(au, 0u, 0u, 0u);
                            s_aug[(s / nkb) & 1][t] = make_float2(Low<KIND>::decode((uint16_t)(au & 0xffffu)),
                                                                  Low<KIND>::decode((uint16_t)(au >> 16)));
                        }
                    }
                };
                stage_load(0, pa, na);
                stage_store(0, pa, na);
                __syncthreads();
                f32x16 acc = {};
                for (int64_t s = 0; s < nst; ++s) {
                    const int64_t tile = s / nkb;
                    const int kb = (int)(s % nkb);
                    // the next stage's loads are in flight during this stage's steps
                    if (s + 1 < nst) stage_load(s + 1, pa, na);
                    if (wkeep) {
                        if (!ONE) {
#pragma unroll
                            for (int u = 0; u < kKSteps; ++u) {
                                const int c = kb * kKBlock + u * 16;
                                bq[u] = c < K ? *reinterpret_cast<const uint4*>(qlow + c) : make_uint4(0, 0, 0, 0);
                            }
                        }
                        // A fragments from LDS in groups of 4, each group's loads
                        // issued while the previous group's steps execute
                        const uint16_t* arow = s_tile[s & 1] + j * kLdsRow + 8 * half;
#pragma unroll
                        for (int u0 = 0; u0 < kKSteps; u0 += 4) {
                            uint4 a[4];
#pragma unroll
                            for (int v = 0; v < 4; ++v) a[v] = *reinterpret_cast<const uint4*>(arow + (u0 + v) * 16);
#pragma unroll
                            for (int v = 0; v < 4; ++v) acc = Low<KIND>::mma(a[v], bq[u0 + v], acc);
                            __builtin_amdgcn_sched_barrier(0);
                        }
                        if (ONE) {
                            // the augmented step: k = 256 .. 271, only (a*, ebar) x (1, sTbar) nonzero
                            const uint4 aa = half == 0 ? *reinterpret_cast<const uint4*>(arow + kKBlock)
                                                       : make_uint4(0, 0, 0, 0);
                            acc = Low<KIND>::mma(aa, bq_aug, acc);
                        }
                    }
                    if (kb == nkb - 1) {
                        if (wkeep) {
                            const int64_t tr0 = ps + tile * kBoundRows;
                            const int nrows = (int)min((int64_t)kBoundRows, pe - tr0);
                            if (half == 0) {
                                staged += (unsigned long long)nrows;
                                if (keep) tested += (unsigned long long)nrows;
                            }
                            const float2* nrm = s_norm[tile & 1];
                            const float* xnr = s_xn[tile & 1];
                            const float2* aug = s_aug[tile & 1];
                            // common path: one test per lane; ONE: the accumulators
                            // already hold acc - beta + sT eps_x, a max suffices;
                            // otherwise 3 operations per pair
                            float mx = -INFINITY;
#pragma unroll
                            for (int r = 0; r < 16; ++r) {
                                if (ONE) {
                                    mx = fmaxf(mx, acc[r]);
                                } else {
                                    const float2 nm = nrm[8 * (r >> 2) + 4 * half + (r & 3)];
                                    mx = fmaxf(mx, fmaf(sT, nm.y, acc[r] - nm.x));
                                }
                            }
                            const bool any = keep && mx >= alpha;
                            uint32_t mask = 0;
                            if (__ballot(any) != 0ull) {
                                // the lanes' exact float32 masks (rows of this part only)
#pragma unroll
                                for (int r = 0; r < 16; ++r) {
                                    const int i = 8 * (r >> 2) + 4 * half + (r & 3);
                                    const float2 nm = nrm[i];
                                    const float e = ONE ? acc[r] : fmaf(sT, nm.y, acc[r] - nm.x);
                                    if (e >= alpha && i < nrows) mask |= 1u << r;
                                }
                                if (!keep) mask = 0;
                            }
                            if (__ballot(mask != 0u) != 0ull) {
                                // rare: the pairs the float32 test kept are decided in
                                // float64; the accumulators go through LDS so that the
                                // loops below index them without unrolling
                                float* sacc = s_acc[wave];
#pragma unroll
                                for (int r = 0; r < 16; ++r) sacc[r * 64 + lane] = acc[r];
                                double2 qn = make_double2(0.0, 0.0);
                                if (mask) qn = ws.qnorm[qj];
                                const double lim = prune_limit(bsf_j);
                                // lower bound of d(q~, x~) for the pair of accumulator r, row i
                                auto pair_d = [&](int r, int i) -> double {
                                    const double ac = (double)sacc[r * 64 + lane];
                                    if (!ONE) return (1.0 - bc.g) * (qn.x + (double)xnr[i]) - 2.0 * ac;
                                    // q~.x~ <= acc - a* - ebar sTbar + g2 S (the K + 2 products)
                                    const double a = aug[i].x, eb = aug[i].y, es = eb * (double)sTb;
                                    const double S = 0.5 * (qn.x + (double)xnr[i]) * (1.0 + 0x1p-38) + fabs(a) + es;
                                    return qn.x + (double)xnr[i] - 2.0 * (ac - a - es + bc.g2 * S);
                                };
                                uint32_t fm = 0;
                                for (int r = 0; r < 16; ++r) {
                                    if (!((mask >> r) & 1u)) continue;
                                    const int i = 8 * (r >> 2) + 4 * half + (r & 3);
                                    const float2 nm = nrm[i];
                                    const double D = pair_d(r, i);
                                    const double lr = fmax(sqrt(fmax(D, 0.0)) - qn.y - (double)nm.y, 0.0);
                                    if (lr * lr <= lim) fm |= 1u << r;
                                }
                                uint32_t total = 0;
                                for (int r = 0; r < 16; ++r) total += (uint32_t)__popcll(__ballot((fm >> r) & 1u));
                                if (total) {
                                    uint32_t* dpos = spos;
                                    uint32_t* dq = sq;
                                    uint32_t* dpart = spart;
                                    uint32_t off = cnt;
                                    const bool own = (int64_t)cnt + total <= ws.slice_cap;
                                    bool ok = true;
                                    if (!own) {
                                        // private slice full: a range of the shared overflow
                                        // slice, as in the LB_SAX filter
                                        long long b = -1;
                                        if (lane == 0) {
                                            uint32_t* oc = &ws.counters[kCtrOvf];
                                            if ((int64_t)load_relaxed(oc) < ws.ovf_cap) {
                                                const uint32_t rr = atomicAdd(oc, total);
                                                if ((int64_t)rr + total <= ws.ovf_cap) b = rr;
                                                else atomicMin(&ws.counters[kCtrOvfEnd], rr);
                                            }
                                        }
                                        b = __shfl(b, 0, 64);
                                        if (b < 0) {
                                            ok = false;
                                            if (fm) lost = true;
                                        } else {
                                            const int64_t ob = (int64_t)ws.n_slices * ws.slice_cap;
                                            dpos = ws.slice_pos + ob;
                                            dq = ws.slice_q + ob;
                                            dpart = ws.slice_part + ob;
                                            off = (uint32_t)b;
                                        }
                                    }
                                    if (ok) {
                                        for (int r = 0; r < 16; ++r) {
                                            const uint64_t bal = __ballot((fm >> r) & 1u);
                                            if ((fm >> r) & 1u) {
                                                const int i = 8 * (r >> 2) + 4 * half + (r & 3);
                                                const float2 nm = nrm[i];
                                                const double D = pair_d(r, i);
                                                const double lr =
                                                    fmax(sqrt(fmax(D, 0.0)) - qn.y - (double)nm.y, 0.0);
                                                const uint32_t slot = off + (uint32_t)__popcll(bal & lt_mask);
                                                dpos[slot] = (uint32_t)(tr0 + i);
                                                dq[slot] = (uint32_t)qj;
                                                // the bound as the first quarter (natural chunk order)
                                                dpart[slot] = pack_quarters(__double2float_rd(lr * lr), 0.0f, 0.0f, 0.0f);
                                            }
                                            off += (uint32_t)__popcll(bal);
                                        }
                                        if (own) cnt += total;
                                        cands += (unsigned long long)__popc(fm);
                                    }
                                }
                            }
                        }
                        acc = f32x16{};
                    }
                    if (s + 1 < nst) stage_store(s + 1, pa, na);
                    __syncthreads();
                }
            }
            // per-query counters: lanes l and l + 32 hold the same query.  The
            // matrix cores also computed the wavefront's lanes past the list:
            // their pairs count with its first query's
            cands += __shfl_down(cands, 32, 64);
            const int nvalid = __popcll(__ballot(qvalid && half == 0));
            if (lane == 0 && nvalid > 0) staged += (unsigned long long)(32 - nvalid) * staged;
            if (half == 0 && qvalid) {
                if (tested) atomicAdd(&ws.stats[(int64_t)qj * kStatSlots + 0], tested);
                if (cands) atomicAdd(&ws.stats[(int64_t)qj * kStatSlots + 6], cands);
                if (staged) atomicAdd(&ws.stats[(int64_t)qj * kStatSlots + 4], staged);
            }
            if (lost) atomicOr(&ws.flags[qj], kFlagCandLost);
        }
    }
    if (lane == 0) ws.slice_cnt[slice] = cnt;
}

}  // namespace

hipError_t launch_shadow(const IndexView& ix, int kind, int64_t nrows, uint16_t* rows, float4* norms,
                         uint32_t* bad_flag, hipStream_t st) {
    if (nrows <= 0) return hipSuccess;
    const int grid = grid_for(nrows * 64, 256, 1 << 16);
    const BoundConsts bc = bound_consts(ix.stride);
    if (kind == kShadowF16)
        k_shadow<kShadowF16><<<dim3(grid), dim3(256), 0, st>>>(ix, nrows, rows, norms, bad_flag, bc);
    else
        k_shadow<kShadowBf16><<<dim3(grid), dim3(256), 0, st>>>(ix, nrows, rows, norms, bad_flag, bc);
    return hipGetLastError();
}

hipError_t launch_query_low(const IndexView& ix, int kind, int32_t Q, const QueryWs& ws, hipStream_t st) {
    if (kind == kShadowF16)
        k_query_low<kShadowF16><<<dim3(ws.Qpad), dim3(64), 0, st>>>(ix, Q, ws);
    else
        k_query_low<kShadowBf16><<<dim3(ws.Qpad), dim3(64), 0, st>>>(ix, Q, ws);
    return hipGetLastError();
}

hipError_t launch_bound(const IndexView& ix, const ShadowView& sv, const ScanParams& sp, const QueryWs& ws,
                        int device_cus, hipStream_t st) {
    // one candidate slice per wavefront; no more workgroups than are resident
    int grid = sp.slices / (kTile / 64);
    if (sv.rows_n <= 0 || sv.parts_n <= 0) {
        // nothing to bound: the pass only marks its slices empty
        hipLaunchKernelGGL(k_empty_slices, dim3(1), dim3(256), 0, st, ws, sp.slice0, sp.slices);
        return hipGetLastError();
    }
    // per part: the queries that keep it, then the first work item of each part
    hipLaunchKernelGGL(k_part_lists, dim3((unsigned)sv.parts_n), dim3(kTile), 0, st, ix, sp, ws);
    hipError_t e = launch_exclusive_scan(ws.pnb, sv.parts_n, ws.pbo, ws.pscan, st);
    if (e != hipSuccess) return e;
    const bool one = ix.stride <= kKBlock;
    int resident;
    if (sv.kind == kShadowF16)
        resident = one ? resident_grid(k_bound<kShadowF16, true>, kTile, 0, device_cus)
                       : resident_grid(k_bound<kShadowF16, false>, kTile, 0, device_cus);
    else
        resident = one ? resident_grid(k_bound<kShadowBf16, true>, kTile, 0, device_cus)
                       : resident_grid(k_bound<kShadowBf16, false>, kTile, 0, device_cus);
    grid = std::max(1, std::min(grid, resident));
    const BoundConsts bc = bound_consts(ix.stride);
    if (sv.kind == kShadowF16) {
        if (one) k_bound<kShadowF16, true><<<dim3(grid), dim3(kTile), 0, st>>>(ix, sv, sp, ws, bc);
        else k_bound<kShadowF16, false><<<dim3(grid), dim3(kTile), 0, st>>>(ix, sv, sp, ws, bc);
    } else {
        if (one) k_bound<kShadowBf16, true><<<dim3(grid), dim3(kTile), 0, st>>>(ix, sv, sp, ws, bc);
        else k_bound<kShadowBf16, false><<<dim3(grid), dim3(kTile), 0, st>>>(ix, sv, sp, ws, bc);
    }
    return hipGetLastError();
}

}  // namespace hs
