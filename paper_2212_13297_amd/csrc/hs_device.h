// Device helpers shared by the query-side kernels (hs_query.hip, hs_scan.hip).
//
// Result keys are (float bits of d << 32 | original id): for d >= 0 the
// unsigned order of the key is the (d, id) lexicographic order.
//
// Distances: 16 lanes own one series; lane l holds points 4l..4l+3 of every
// 64-point chunk.  A chunk's partial is the lane's sequential fma chain over
// its 4 points, summed over the 16 lanes by a xor butterfly (commutative, so
// every lane holds the same value).  Two forms:
//  - the running distance that early abandoning tests: plain float32 partials
//    (or compensated ones in the precision form) added in whatever chunk
//    order the kernel reads;
//  - the result key of a series that completes within its limit: the
//    compensated distance (Dist<kComp>) summed in natural chunk order, whose
//    relative error is below 2^-23 + (4K + 64) 2^-48 for K stored points.
// Every kernel keys its results the same way, so a (query, series) pair
// always gets the same float32 distance, and the abandoning limit carries a
// margin (ScanParams::marg) that covers the running form's larger error.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "hs_internal.h"

namespace hs {
namespace {

__device__ __forceinline__ double gap(double v, double lo, double hi) {
    return v < lo ? lo - v : (v > hi ? v - hi : 0.0);
}

__device__ __forceinline__ float bits_to_float(uint32_t b) { return __uint_as_float(b); }

__device__ __forceinline__ uint32_t load_relaxed(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ unsigned long long load_relaxed64(const unsigned long long* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// BSF_k of query q as float bits: the high word of its result key bound
// (little-endian), read on its own.
__device__ __forceinline__ uint32_t bsf_bits(const QueryWs& ws, int q) {
    return load_relaxed(reinterpret_cast<const uint32_t*>(ws.bkey + q) + 1);
}

// A bound prunes only when it exceeds BSF_k by the relative slack.
__device__ __forceinline__ double prune_limit(float bsf) { return (double)bsf * (1.0 + kSlack); }

// The LB_SAX table in LDS has 16 W16 segment rows: the query's w rows, then
// zero rows for the padding segments (whose stored symbols are 0), so the
// lookups below need no test on w.
template <int W16>
constexpr int lut_floats() {
    return 16 * W16 * kCard;
}

template <int W16>
__device__ __forceinline__ void load_lut(float* s_lut, const float* __restrict__ src, int w, int t, int nt) {
    for (int j = t; j < lut_floats<W16>(); j += nt) s_lut[j] = j < w * kCard ? src[j] : 0.0f;
}

// LB_SAX of one stored series: sum over segments of the query's table entry
// for the series' symbol (words are 16-byte aligned, W16 uint4 per word).
// Branch-free, four partial sums, so the table loads issue together.
template <int W16>
__device__ __forceinline__ float lb_sax_word(const uint4 (&v)[W16], const float* s_lut) {
    float acc[4];
#pragma unroll
    for (int u = 0; u < W16; ++u) {
        const uint32_t parts[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
#pragma unroll
        for (int p = 0; p < 4; ++p) {
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int i = u * 16 + p * 4 + b;
                const float e = s_lut[i * kCard + ((parts[p] >> (8 * b)) & 0xffu)];
                acc[b] = i < 4 ? e : acc[b] + e;  // table entries are >= 0
            }
        }
    }
    return (acc[0] + acc[1]) + (acc[2] + acc[3]);
}

// The same bound split by quarters of the word: a[p] sums the symbols of
// segments [p w/4, (p + 1) w/4) when w = 16 W16 (the bound is
// (a0 + a1) + (a2 + a3)).  The refine reads a series' chunks in the order of
// these partial bounds, largest first.
template <int W16>
__device__ __forceinline__ void lb_sax_quarters(const uint4 (&v)[W16], const float* s_lut, float (&a)[4]) {
    // every table read is issued before the first sum, then each quarter's
    // entries are added as a balanced tree (table entries are >= 0)
    constexpr int kSeg = 16 * W16, kQ = 4 * W16;
    float e[kSeg];
#pragma unroll
    for (int u = 0; u < W16; ++u) {
        const uint32_t parts[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
#pragma unroll
        for (int p = 0; p < 4; ++p) {
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int i = u * 16 + p * 4 + b;
                e[i] = s_lut[i * kCard + ((parts[p] >> (8 * b)) & 0xffu)];
            }
        }
    }
#pragma unroll
    for (int qt = 0; qt < 4; ++qt) {
        float t[kQ];
#pragma unroll
        for (int j = 0; j < kQ; ++j) t[j] = e[qt * kQ + j];
#pragma unroll
        for (int h = kQ / 2; h >= 1; h >>= 1)
#pragma unroll
            for (int j = 0; j < h; ++j) t[j] = t[j] + t[j + h];
        a[qt] = t[0];
    }
}

// Four non-negative float32 values in one word: byte p is the high byte of
// a_p as fp16 rounded toward zero (5 exponent and 2 mantissa bits), so the
// value it stands for, that byte followed by a zero byte, is at most a_p, and
// bytes order as the values do.
__device__ __forceinline__ uint32_t pack_quarters(float a0, float a1, float a2, float a3) {
    const uint32_t h01 = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(a0, a1));
    const uint32_t h23 = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(a2, a3));
    return __builtin_amdgcn_perm(h23, h01, 0x07050301u);  // bytes 1, 3 of h01, then of h23
}

// The value a byte of the packed quarter bounds stands for (at most the
// float32 value it was packed from).
__device__ __forceinline__ float quarter_value(uint32_t byte) {
    return (float)__builtin_bit_cast(_Float16, (uint16_t)(byte << 8));
}

// Raw buffer loads.  A load whose offset lies past the resource's byte size
// returns zeros and reads no memory, so a masked-out load is an ordinary
// instruction with no traffic: loads need no branch around them, every load
// is issued, and the waits before their uses get fixed counts.
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
constexpr uint32_t kNoLoad = 0x80000000u;   // past every resource this library builds (sizes < 2^31)
constexpr int kBufferWord3 = 0x00020000;    // resource word 3 for CDNA raw buffers (32-bit data format)

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, kBufferWord3);
}

__device__ __forceinline__ uint4 buffer_load16(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    const u32x4_t v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0);
    return make_uint4(v.x, v.y, v.z, v.w);
}

template <int W16>
__device__ __forceinline__ void load_word(const uint8_t* __restrict__ wp, uint4 (&v)[W16]) {
#pragma unroll
    for (int u = 0; u < W16; ++u) v[u] = *reinterpret_cast<const uint4*>(wp + 16 * u);
}

// The value of lane l ^ m (m = 1, 2, 4, 8) within a row of 16 lanes, by a
// data-parallel-primitive move (no LDS).  xor 1 and xor 2 are quad
// permutations; for m = 4 and 8 the value must already be the same in each
// aligned group of m lanes (true after the earlier butterfly steps), where
// the half-row mirror (l -> 7 - l in each 8 lanes) and the row mirror
// (l -> 15 - l) pick a lane of the partner group.
template <int M>
__device__ __forceinline__ float row_xor(float v) {
    constexpr int ctrl = M == 1 ? 0xB1 : (M == 2 ? 0x4E : (M == 4 ? 0x141 : 0x140));
    // (the patterns never read outside the row, so bound_ctrl does not change
    // the value; set, it lets the move fuse into the consuming add)
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), ctrl, 0xF, 0xF, true));
}

__device__ __forceinline__ float chunk_partial(float4 q, float4 x) {
    const float t0 = q.x - x.x, t1 = q.y - x.y, t2 = q.z - x.z, t3 = q.w - x.w;
    float p = t0 * t0;
    p = fmaf(t1, t1, p);
    p = fmaf(t2, t2, p);
    p = fmaf(t3, t3, p);
    p += row_xor<1>(p);
    p += row_xor<2>(p);
    p += row_xor<4>(p);
    p += row_xor<8>(p);
    return p;
}

// Knuth's TwoSum: s = fl(a + b) and e such that a + b = s + e exactly.
// Contraction is off: no step may be fused with a product.
__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
#pragma clang fp contract(off)
    s = a + b;
    const float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// Compensated partial of one 64-point chunk (precision form): the chunk's
// squared distance as hi + lo.  Per point, q - x = dv + ev exactly (TwoSum)
// and dv^2 = p + pe exactly (fma); the points' p are summed with TwoSum, every
// rounding residue goes to lo.  The butterfly combines (hi, lo) pairs the same
// way; TwoSum's residue is exact, so all 16 lanes end with identical values.
__device__ __forceinline__ float chunk_partial_comp(float4 q, float4 x, float& lo_out) {
#pragma clang fp contract(off)
    const float qa[4] = {q.x, q.y, q.z, q.w}, xa[4] = {x.x, x.y, x.z, x.w};
    float hi = 0.0f, lo = 0.0f;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        float dv, ev;
        two_sum(qa[v], -xa[v], dv, ev);
        const float p = dv * dv;
        const float pe = fmaf(dv, dv, -p);
        const float r = fmaf(ev, (dv + dv) + ev, pe);  // (dv + ev)^2 - p
        float t, te;
        two_sum(hi, p, t, te);
        hi = t;
        lo += te + r;
    }
    auto step = [&](float oh, float ol) {
        float t, te;
        two_sum(hi, oh, t, te);
        hi = t;
        lo = (lo + ol) + te;
    };
    step(row_xor<1>(hi), row_xor<1>(lo));
    step(row_xor<2>(hi), row_xor<2>(lo));
    step(row_xor<4>(hi), row_xor<4>(lo));
    step(row_xor<8>(hi), row_xor<8>(lo));
    lo_out = lo;
    return hi;
}

// Running squared distance of one (query, series) pair in form F.
template <int F>
struct Dist;

template <>
struct Dist<kPlain> {
    float s = 0.0f;
    __device__ __forceinline__ void add(float4 q, float4 x) { s += chunk_partial(q, x); }
    __device__ __forceinline__ float value() const { return s; }
};

template <>
struct Dist<kComp> {
    float s = 0.0f, c = 0.0f;
    __device__ __forceinline__ void add(float4 q, float4 x) {
#pragma clang fp contract(off)
        float lo, t, te;
        const float hi = chunk_partial_comp(q, x, lo);
        two_sum(s, hi, t, te);
        s = t;
        c += lo + te;
    }
    __device__ __forceinline__ float value() const {
#pragma clang fp contract(off)
        return s + c;
    }
};

// Result key distance of one series: the compensated distance in natural
// chunk order, by the 16 lanes of a group (all 16 active together).  xr / qr
// point at the lane's first point.
__device__ __forceinline__ float key_distance(const float* __restrict__ xr, const float* __restrict__ qr,
                                              int nchunks) {
    Dist<kComp> d;
    for (int c = 0; c < nchunks; ++c)
        d.add(*reinterpret_cast<const float4*>(qr + c * kChunk), *reinterpret_cast<const float4*>(xr + c * kChunk));
    return d.value();
}

// Squared distance of one series, computed by the 16 lanes of a group (all 16
// active together).  xr / qr point at the lane's first point.  Chunks are
// loaded two at a time; after each pair the running sum (form F) is compared
// with thr (the limit times ScanParams::marg) and the series is abandoned once
// it exceeds it.  A series that completes gets its result key distance: the
// running sum itself in the compensated form, else key_distance (the chunks
// are read again).  `chunks` counts the chunks read.
template <int F>
__device__ __forceinline__ float refine_row(const float* __restrict__ xr, const float* __restrict__ qr,
                                           int nchunks, float thr, bool& alive, unsigned& chunks) {
    Dist<F> d;
    alive = true;
    for (int c = 0; c < nchunks; c += 2) {
        const bool two = c + 1 < nchunks;
        const float4 x0 = *reinterpret_cast<const float4*>(xr + c * kChunk);
        float4 x1 = make_float4(0.f, 0.f, 0.f, 0.f);
        if (two) x1 = *reinterpret_cast<const float4*>(xr + (c + 1) * kChunk);
        d.add(*reinterpret_cast<const float4*>(qr + c * kChunk), x0);
        if (two) d.add(*reinterpret_cast<const float4*>(qr + (c + 1) * kChunk), x1);
        chunks += two ? 2u : 1u;
        if (d.value() > thr) {
            alive = false;
            break;
        }
    }
    if (F == kComp || !alive) return d.value();
    chunks += (unsigned)nchunks;
    return key_distance(xr, qr, nchunks);
}

// Insert key into the ascending list top[0..n) of capacity k (one thread).
__device__ __forceinline__ void topk_insert(unsigned long long* top, int& n, int k, unsigned long long key) {
    if (n == k && key >= top[k - 1]) return;
    int p = n < k ? n : k - 1;
    while (p > 0 && top[p - 1] > key) {
        top[p] = top[p - 1];
        --p;
    }
    top[p] = key;
    if (n < k) ++n;
}

// Publish a block's top-k for query q (one thread): tighten the query's key
// bound with its k-th key, then append the entries whose keys do not exceed
// the bound to the pool.  Keys, not distances, are compared, so series tied
// at the k-th distance beyond the k-th id are not appended again and again.
__device__ __forceinline__ void flush_topk(const QueryWs& ws, int q, int k, const unsigned long long* top, int n) {
    if (q < 0 || n == 0) return;
    unsigned long long g = load_relaxed64(&ws.bkey[q]);
    if (n == k && top[k - 1] < g) {
        atomicMin(&ws.bkey[q], top[k - 1]);
        g = top[k - 1];
    }
    int cnt = 0;
    while (cnt < n && top[cnt] <= g) ++cnt;
    if (cnt == 0) return;
    const uint32_t base = atomicAdd(&ws.pool_cnt[q], (uint32_t)cnt);
    for (int j = 0; j < cnt; ++j)
        if (base + j < (uint32_t)ws.P) ws.pool[(int64_t)q * ws.P + base + j] = top[j];
    if (base + cnt > (uint32_t)ws.P) atomicOr(&ws.flags[q], kFlagOverflow);
}

// Exclusive prefix sum over the 64 NW threads of a block (256 by default);
// returns the offset of this thread and writes the block total to *total.
// s_w holds NW ints.
template <int NW = kTile / 64>
__device__ __forceinline__ int block_exclusive_scan(int v, int* s_w, int* total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    if (lane == 63) s_w[wave] = inc;
    __syncthreads();
    int off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        const int c = s_w[i];
        if (i < wave) off += c;
        tot += c;
    }
    *total = tot;
    __syncthreads();
    return off + inc - v;
}

__device__ __forceinline__ uint64_t leaf_key(float lbe, int64_t leaf) {
    return ((uint64_t)__float_as_uint(lbe) << 32) | (uint64_t)(uint32_t)leaf;
}

__device__ __forceinline__ unsigned long long block_min_u64(unsigned long long v, unsigned long long* s_tmp) {
    for (int o = 32; o > 0; o >>= 1) {
        unsigned long long other = __shfl_xor(v, o, 64);
        v = other < v ? other : v;
    }
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) s_tmp[wave] = v;
    __syncthreads();
    unsigned long long r = s_tmp[0];
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) r = s_tmp[i] < r ? s_tmp[i] : r;
    __syncthreads();
    return r;
}

// Contiguous share [lo, hi) of `total` work units for this block.
__device__ __forceinline__ void block_range(int64_t total, int64_t& lo, int64_t& hi) {
    lo = total * (int64_t)blockIdx.x / (int64_t)gridDim.x;
    hi = total * ((int64_t)blockIdx.x + 1) / (int64_t)gridDim.x;
}

inline int grid_for(int64_t work, int block, int cap = 65536) {
    int64_t g = (work + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

inline int w16_of(const IndexView& ix) { return (ix.wstride + 15) / 16; }

// Grid of a persistent kernel: as many workgroups as can be resident at once
// (occupancy from the runtime for this kernel, block size and dynamic LDS),
// so that static work ranges all run concurrently.
template <typename K>
inline int resident_grid(K kernel, int block, size_t dyn_lds, int cus) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, dyn_lds) != hipSuccess || per_cu < 1)
        per_cu = 1;
    return cus * per_cu;
}

}  // namespace
}  // namespace hs

// Persistent launch of KERNEL<W16> with a resident grid of kTile-thread workgroups.
#define HS_LAUNCH_RESIDENT(ix, KERNEL, lds, cus, st, ...)                                                   \
    switch (w16_of(ix)) {                                                                                  \
        case 1: hipLaunchKernelGGL(KERNEL<1>, dim3(resident_grid(KERNEL<1>, kTile, lds, cus)), dim3(kTile), \
                                   lds, st, __VA_ARGS__); break;                                           \
        case 2: hipLaunchKernelGGL(KERNEL<2>, dim3(resident_grid(KERNEL<2>, kTile, lds, cus)), dim3(kTile), \
                                   lds, st, __VA_ARGS__); break;                                           \
        case 3: hipLaunchKernelGGL(KERNEL<3>, dim3(resident_grid(KERNEL<3>, kTile, lds, cus)), dim3(kTile), \
                                   lds, st, __VA_ARGS__); break;                                           \
        default: hipLaunchKernelGGL(KERNEL<4>, dim3(resident_grid(KERNEL<4>, kTile, lds, cus)), dim3(kTile),\
                                    lds, st, __VA_ARGS__); break;                                          \
    }

#define HS_DISPATCH_W16(ix, KERNEL, ...)                                              \
    switch (w16_of(ix)) {                                                            \
        case 1: hipLaunchKernelGGL(KERNEL<1>, __VA_ARGS__); break;                   \
        case 2: hipLaunchKernelGGL(KERNEL<2>, __VA_ARGS__); break;                   \
        case 3: hipLaunchKernelGGL(KERNEL<3>, __VA_ARGS__); break;                   \
        default: hipLaunchKernelGGL(KERNEL<4>, __VA_ARGS__); break;                  \
    }

// The same two dispatches for kernels templated on <W16, F> (F a constant).
#define HS_LAUNCH_RESIDENT_F(ix, KERNEL, F, lds, cus, st, ...)                                        \
    switch (w16_of(ix)) {                                                                            \
        case 1: KERNEL<1, F><<<dim3(resident_grid(KERNEL<1, F>, kTile, lds, cus)), dim3(kTile), lds, st>>>( \
                    __VA_ARGS__); break;                                                             \
        case 2: KERNEL<2, F><<<dim3(resident_grid(KERNEL<2, F>, kTile, lds, cus)), dim3(kTile), lds, st>>>( \
                    __VA_ARGS__); break;                                                             \
        case 3: KERNEL<3, F><<<dim3(resident_grid(KERNEL<3, F>, kTile, lds, cus)), dim3(kTile), lds, st>>>( \
                    __VA_ARGS__); break;                                                             \
        default: KERNEL<4, F><<<dim3(resident_grid(KERNEL<4, F>, kTile, lds, cus)), dim3(kTile), lds, st>>>( \
                     __VA_ARGS__); break;                                                            \
    }

#define HS_DISPATCH_W16_F(ix, KERNEL, F, grid, block, lds, st, ...)                  \
    switch (w16_of(ix)) {                                                            \
        case 1: KERNEL<1, F><<<grid, block, lds, st>>>(__VA_ARGS__); break;          \
        case 2: KERNEL<2, F><<<grid, block, lds, st>>>(__VA_ARGS__); break;          \
        case 3: KERNEL<3, F><<<grid, block, lds, st>>>(__VA_ARGS__); break;          \
        default: KERNEL<4, F><<<grid, block, lds, st>>>(__VA_ARGS__); break;         \
    }
