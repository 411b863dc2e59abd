// Leaf partition on the device (Hercules Sec. 3.2 H-splits, applied top-down
// to the whole batch; Sec. 3.3 builds the tree by inserting series, which a
// batch build replaces).  A node holding more than tau series is split on the
// (segment, statistic) whose midpoint threshold t = (min + max) / 2 separates
// it and whose segment_length * (max - min)^2 is largest (lowest segment first,
// mean before std on ties); series with v < t go left, in their order.  Below
// the leaf level the same splits continue down to 64 series: they only order
// the series inside their leaf (tight 64-series chunk envelopes).
//
// The nodes of one depth are processed together, level by level:
//   classify  leaves are recorded where a node first holds <= tau series;
//             active nodes (a split is tried) get tiles of kTileElems series
//   minmax    per active node: min and max of its 2w statistics
//   count     per active node and candidate: series below the midpoint
//   choose    per node: the first candidate in score order that separates
//   apply     leaf budget, leaves of unsplittable nodes, children counts
//   tile_left / scatter / copyback   the stable partition of every split
//             node's series (ranks from a scan over the tiles' left counts)
//   next      the next level's node list (children, in order)
// Statistics are float32 (the build's per-series mean and std), thresholds
// and scores FP64, exactly as the host partition computes them, so both give
// the same leaves and the same order.
//
// Leaf budget: so that the index's tables fit a size fixed before the build,
// at most `budget` leaves are made.  A node that would split while more
// leaves could follow than the budget allows becomes a leaf at once (its
// series are still ordered by the in-leaf splits).  Nodes are granted splits
// in node order, so the result is deterministic.  The budget binds only for
// pathological partitions (results never depend on it; pruning does).
#include <algorithm>
#include <vector>

#include "hs_host.h"
#include "hs_device.h"

namespace hs {
namespace {

constexpr int kTileElems = 2048;  // series per tile of an active node
constexpr int kScanBlock = 1024;  // elements per block of the exclusive scan

// node type bits
constexpr uint32_t kInLeaf = 1u;   // below the leaf level
constexpr uint32_t kActive = 2u;   // a split is tried at this level
constexpr uint32_t kSplit = 4u;    // split at this level

__device__ __forceinline__ uint32_t fkey(float f) {
    const uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float funkey(uint32_t k) {
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

// ---------------------------------------------------------------- scan
// out[i] = sum of in[0..i), out[n] = total (n + 1 entries).
__global__ void __launch_bounds__(256) k_scan_blocks(const uint32_t* __restrict__ in, int64_t n,
                                                     uint32_t* __restrict__ out, uint32_t* __restrict__ bsum) {
    __shared__ uint32_t s_w[4];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)t * 4;
    uint32_t v[4], loc = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        v[j] = base + j < n ? in[base + j] : 0u;
        loc += v[j];
    }
    uint32_t inc = loc;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    if (lane == 63) s_w[wave] = inc;
    __syncthreads();
    uint32_t off = 0;
    for (int i = 0; i < wave; ++i) off += s_w[i];
    uint32_t run = off + inc - loc;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (base + j < n) out[base + j] = run;
        run += v[j];
    }
    if (t == 255) bsum[blockIdx.x] = off + inc;
}

__global__ void __launch_bounds__(1024) k_scan_sums(uint32_t* __restrict__ bsum, int64_t nb) {
    __shared__ uint32_t s_part[1024];
    const int t = threadIdx.x;
    const int64_t per = (nb + 1023) / 1024;
    const int64_t a = min(nb, (int64_t)t * per), b = min(nb, a + per);
    uint32_t sum = 0;
    for (int64_t i = a; i < b; ++i) sum += bsum[i];
    s_part[t] = sum;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const uint32_t v = t >= o ? s_part[t - o] : 0u;
        __syncthreads();
        s_part[t] += v;
        __syncthreads();
    }
    uint32_t run = s_part[t] - sum;
    for (int64_t i = a; i < b; ++i) {
        const uint32_t c = bsum[i];
        bsum[i] = run;
        run += c;
    }
    if (t == 1023) bsum[nb] = s_part[1023];
}

__global__ void __launch_bounds__(256) k_scan_add(uint32_t* __restrict__ out, int64_t n,
                                                  const uint32_t* __restrict__ bsum) {
    const int64_t i0 = (int64_t)blockIdx.x * kScanBlock;
    const uint32_t add = bsum[blockIdx.x];
    for (int j = threadIdx.x; j < kScanBlock; j += blockDim.x)
        if (i0 + j < n) out[i0 + j] += add;
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = bsum[gridDim.x];
}


// ---------------------------------------------------------------- levels
struct Level {
    // current node list (sorted by start) and the next one
    const int64_t* nb;
    const int64_t* ne;
    const uint32_t* ntype;
    int64_t* nb2;
    int64_t* ne2;
    uint32_t* ntype2;
    int64_t M;           // nodes in the current list
    // per node of the current list
    uint32_t* ntiles;    // tiles (0 unless active); scanned into tile0
    uint32_t* tile0;     // [M + 1] first tile of each node
    uint32_t* mm;        // [M][2w][2] ordered keys of min, max
    uint32_t* cntl;      // [M][2w] series below each candidate's midpoint
    int32_t* choice;     // [M] chosen candidate or -1
    double* thr;         // [M]
    uint32_t* want;      // [M] a split that needs leaf budget; scanned into wrank
    uint32_t* wrank;     // [M + 1]
    uint32_t* nchild;    // [M] children (0 or 2); scanned into child0
    uint32_t* child0;    // [M + 1]
    // per tile
    uint32_t* tleft;     // [tiles] left series of the tile; scanned into tleft0
    uint32_t* tleft0;    // [tiles + 1]
    // series
    float2* st;          // [N][w] statistics in the current order
    uint32_t* id;        // [N] original ids in the current order
    float2* st2;         // scatter buffers
    uint32_t* id2;
    int64_t* leaves;     // [budget] leaf starts (unordered)
    uint32_t* ctr;       // [0] leaves, [1] active pre-leaf nodes
    int64_t N, tau, budget;
    int32_t w;
};

// leaves at the first node holding <= tau series; active nodes and their tiles
__global__ void k_classify(Level lv) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= lv.M) return;
    const int64_t b = lv.nb[i], e = lv.ne[i], cnt = e - b;
    uint32_t ty = lv.ntype[i] & kInLeaf;
    if (!(ty & kInLeaf) && cnt <= lv.tau) {
        const uint32_t s = atomicAdd(&lv.ctr[0], 1u);
        if (s < lv.budget) lv.leaves[s] = b;
        ty |= kInLeaf;
    }
    // a pre-leaf node here holds more than tau >= 1 series
    const bool active = !((ty & kInLeaf) && cnt <= kChunkRows);
    if (active) {
        ty |= kActive;
        if (!(ty & kInLeaf)) atomicAdd(&lv.ctr[1], 1u);
    }
    ((uint32_t*)lv.ntype)[i] = ty;
    lv.ntiles[i] = active ? (uint32_t)((cnt + kTileElems - 1) / kTileElems) : 0u;
    for (int c = 0; c < 2 * lv.w; ++c) {
        lv.mm[(i * 2 * lv.w + c) * 2 + 0] = 0xffffffffu;
        lv.mm[(i * 2 * lv.w + c) * 2 + 1] = 0u;
        lv.cntl[i * 2 * lv.w + c] = 0u;
    }
    lv.choice[i] = -1;
}

// The node of tile `tile`: the last node whose first tile is <= tile.
__device__ __forceinline__ int64_t node_of_tile(const Level& lv, uint32_t tile) {
    int64_t lo = 0, hi = lv.M - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (lv.tile0[mid] <= tile) lo = mid;
        else hi = mid - 1;
    }
    // skip nodes with no tiles that share the first tile index
    while (lo + 1 < lv.M && lv.tile0[lo + 1] <= tile) ++lo;
    return lo;
}

// Thread layout of the tile kernels: candidate c = t % C2 (C2 = 2w
// statistics: mean of segment c / 2 when c is even, std when odd), element
// lane g = t / C2 of G = 256 / C2 lanes.
template <bool COUNT>
__global__ void __launch_bounds__(256) k_tile_stats(Level lv) {
    __shared__ uint32_t s_a[256], s_b[256];
    __shared__ double s_thr[128];
    const uint32_t tiles = lv.tile0[lv.M];
    const int C2 = 2 * lv.w, G = 256 / C2;
    const int t = threadIdx.x, c = t % C2, g = t / C2;
    const bool on = g < G;
    for (uint32_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const int64_t node = node_of_tile(lv, tile);
        const int64_t b = lv.nb[node], e = lv.ne[node];
        const int64_t s0 = b + (int64_t)(tile - lv.tile0[node]) * kTileElems, s1 = min(e, s0 + kTileElems);
        if (COUNT) {
            if (t < C2) {
                const uint32_t* m = lv.mm + (node * C2 + t) * 2;
                s_thr[t] = ((double)funkey(m[0]) + (double)funkey(m[1])) / 2.0;
            }
            __syncthreads();
        }
        uint32_t a = COUNT ? 0u : 0xffffffffu, bb = 0u;
        if (on) {
            const double th = COUNT ? s_thr[c] : 0.0;
            const float* base = reinterpret_cast<const float*>(lv.st);
            for (int64_t r = s0 + g; r < s1; r += G) {
                const float v = base[r * C2 + c];
                if (COUNT) {
                    a += (double)v < th ? 1u : 0u;
                } else {
                    const uint32_t k = fkey(v);
                    a = min(a, k);
                    bb = max(bb, k);
                }
            }
        }
        s_a[t] = a;
        s_b[t] = bb;
        __syncthreads();
        if (t < C2) {
            for (int j = 1; j < G; ++j) {
                if (COUNT) {
                    a += s_a[t + j * C2];
                } else {
                    a = min(a, s_a[t + j * C2]);
                    bb = max(bb, s_b[t + j * C2]);
                }
            }
            if (COUNT) {
                if (a) atomicAdd(&lv.cntl[node * C2 + t], a);
            } else {
                atomicMin(&lv.mm[(node * C2 + t) * 2 + 0], a);
                atomicMax(&lv.mm[(node * C2 + t) * 2 + 1], bb);
            }
        }
        __syncthreads();
    }
}

// The first candidate, in order of score l (max - min)^2 (equal segment
// lengths: range^2) descending, lowest candidate first on ties, that leaves
// both sides non-empty; candidates with an empty range end the search.
__global__ void k_choose(Level lv) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= lv.M) return;
    const uint32_t ty = lv.ntype[i];
    lv.want[i] = 0u;
    if (!(ty & kActive)) return;
    const int C2 = 2 * lv.w;
    const int64_t cnt = lv.ne[i] - lv.nb[i];
    uint8_t order[128];
    double score[128];
    for (int c = 0; c < C2; ++c) {
        const uint32_t* m = lv.mm + (i * C2 + c) * 2;
        const double r = (double)funkey(m[1]) - funkey(m[0]);
        score[c] = r * r;
        // insertion keeps equal scores in candidate order
        int p = c;
        while (p > 0 && score[order[p - 1]] < score[c]) {
            order[p] = order[p - 1];
            --p;
        }
        order[p] = (uint8_t)c;
    }
    for (int j = 0; j < C2; ++j) {
        const int c = order[j];
        const uint32_t* m = lv.mm + (i * C2 + c) * 2;
        const float mn = funkey(m[0]), mx = funkey(m[1]);
        if (!(mx > mn)) break;
        const uint32_t left = lv.cntl[i * C2 + c];
        if (left > 0 && (int64_t)left < cnt) {
            lv.choice[i] = c;
            lv.thr[i] = ((double)mn + (double)mx) / 2.0;
            if (!(ty & kInLeaf)) lv.want[i] = 1u;
            return;
        }
    }
}

// Budget, leaves of nodes that cannot split, children.
__global__ void k_apply(Level lv) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= lv.M) return;
    uint32_t ty = lv.ntype[i];
    lv.nchild[i] = 0u;
    if (!(ty & kActive)) return;
    const int64_t b = lv.nb[i];
    if (lv.choice[i] < 0) {
        if (!(ty & kInLeaf)) {
            const uint32_t s = atomicAdd(&lv.ctr[0], 1u);
            if (s < lv.budget) lv.leaves[s] = b;
        }
        return;
    }
    if (!(ty & kInLeaf)) {
        // splits granted in node order: the leaves already made plus one per
        // active pre-leaf node, plus one per granted split, stay within budget
        const int64_t granted = lv.budget - (int64_t)lv.ctr[2] - (int64_t)lv.ctr[3];
        if ((int64_t)lv.wrank[i] >= granted) {
            const uint32_t s = atomicAdd(&lv.ctr[0], 1u);
            if (s < lv.budget) lv.leaves[s] = b;
            ty |= kInLeaf;
        }
    }
    ((uint32_t*)lv.ntype)[i] = ty | kSplit;
    lv.nchild[i] = 2u;
}

// Left series of each tile of a split node.
__global__ void __launch_bounds__(256) k_tile_left(Level lv) {
    __shared__ uint32_t s_w[4];
    const uint32_t tiles = lv.tile0[lv.M];
    for (uint32_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const int64_t node = node_of_tile(lv, tile);
        uint32_t cnt = 0;
        if (lv.ntype[node] & kSplit) {
            const int64_t s0 = lv.nb[node] + (int64_t)(tile - lv.tile0[node]) * kTileElems;
            const int64_t s1 = min(lv.ne[node], s0 + kTileElems);
            const int c = lv.choice[node];
            const double th = lv.thr[node];
            const float* base = reinterpret_cast<const float*>(lv.st);
            for (int64_t r = s0 + threadIdx.x; r < s1; r += blockDim.x)
                cnt += (double)base[r * 2 * lv.w + c] < th ? 1u : 0u;
        }
        for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
        if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = cnt;
        __syncthreads();
        if (threadIdx.x == 0) lv.tleft[tile] = s_w[0] + s_w[1] + s_w[2] + s_w[3];
        __syncthreads();
    }
}

// Stable partition of every split node into the scatter buffers: left
// series first, each side in its order.
__global__ void __launch_bounds__(256) k_scatter(Level lv) {
    __shared__ uint32_t s_w[4];
    const uint32_t tiles = lv.tile0[lv.M];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (uint32_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const int64_t node = node_of_tile(lv, tile);
        if (!(lv.ntype[node] & kSplit)) continue;  // uniform over the block
        const int64_t b = lv.nb[node], e = lv.ne[node];
        const uint32_t t0 = lv.tile0[node], t1 = lv.tile0[node + 1];
        const int64_t nl = (int64_t)(lv.tleft0[t1] - lv.tleft0[t0]);
        int64_t left_before = (int64_t)(lv.tleft0[tile] - lv.tleft0[t0]);
        const int64_t s0 = b + (int64_t)(tile - t0) * kTileElems, s1 = min(e, s0 + kTileElems);
        const int c = lv.choice[node];
        const double th = lv.thr[node];
        const float* base = reinterpret_cast<const float*>(lv.st);
        for (int64_t r0 = s0; r0 < s1; r0 += blockDim.x) {
            const int64_t r = r0 + threadIdx.x;
            const bool in = r < s1;
            const bool lf = in && (double)base[r * 2 * lv.w + c] < th;
            const uint64_t bal = __ballot(lf);
            if (lane == 0) s_w[wave] = (uint32_t)__popcll(bal);
            __syncthreads();
            uint32_t before = 0, tot = 0;
            for (int i = 0; i < 4; ++i) {
                if (i < wave) before += s_w[i];
                tot += s_w[i];
            }
            const int64_t lrank = left_before + before + (uint32_t)__popcll(bal & ((1ull << lane) - 1ull));
            if (in) {
                const int64_t dest = lf ? b + lrank : b + nl + (r - b) - lrank;
                for (int j = 0; j < lv.w; ++j) lv.st2[dest * lv.w + j] = lv.st[r * lv.w + j];
                lv.id2[dest] = lv.id[r];
            }
            left_before += tot;
            __syncthreads();
        }
    }
}

__global__ void __launch_bounds__(256) k_copyback(Level lv) {
    const uint32_t tiles = lv.tile0[lv.M];
    for (uint32_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const int64_t node = node_of_tile(lv, tile);
        if (!(lv.ntype[node] & kSplit)) continue;
        const int64_t s0 = lv.nb[node] + (int64_t)(tile - lv.tile0[node]) * kTileElems;
        const int64_t s1 = min(lv.ne[node], s0 + kTileElems);
        for (int64_t r = s0 + threadIdx.x; r < s1; r += blockDim.x) lv.id[r] = lv.id2[r];
        for (int64_t j = s0 * lv.w + threadIdx.x; j < s1 * lv.w; j += blockDim.x) lv.st[j] = lv.st2[j];
    }
}

__global__ void k_next(Level lv) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= lv.M || lv.nchild[i] == 0u) return;
    const int64_t b = lv.nb[i], e = lv.ne[i];
    const uint32_t t0 = lv.tile0[i], t1 = lv.tile0[i + 1];
    const int64_t nl = (int64_t)(lv.tleft0[t1] - lv.tleft0[t0]);
    const uint32_t ty = lv.ntype[i] & kInLeaf;
    const int64_t o = lv.child0[i];
    lv.nb2[o] = b;
    lv.ne2[o] = b + nl;
    lv.ntype2[o] = ty;
    lv.nb2[o + 1] = b + nl;
    lv.ne2[o + 1] = e;
    lv.ntype2[o + 1] = ty;
}

// Snapshot of the counters the budget uses this level: ctr[2] = leaves made so
// far, ctr[3] = active pre-leaf nodes.
__global__ void k_budget_snapshot(uint32_t* ctr) {
    if (threadIdx.x == 0) {
        ctr[2] = ctr[0];
        ctr[3] = ctr[1];
        ctr[1] = 0u;
    }
}

__global__ void k_iota(uint32_t* id, int64_t N) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
        id[i] = (uint32_t)i;
}

__global__ void k_root(int64_t* nb, int64_t* ne, uint32_t* ntype, int64_t N, uint32_t* ctr) {
    if (threadIdx.x == 0) {
        nb[0] = 0;
        ne[0] = N;
        ntype[0] = 0u;
        for (int i = 0; i < 8; ++i) ctr[i] = 0u;
    }
}

struct Carve {
    char* cur;
    int64_t used = 0;
    template <typename T>
    T* take(int64_t count) {
        T* p = (T*)cur;
        const int64_t bytes = align_up(count * (int64_t)sizeof(T), 256);
        cur += bytes;
        used += bytes;
        return p;
    }
};

// Active nodes per level hold more than min(tau, 64) series.
int64_t max_active(int64_t N, int64_t tau) {
    const int64_t lim = std::min<int64_t>(tau, kChunkRows);
    return std::min<int64_t>(N, N / (lim + 1) + 1);
}

struct Bufs {
    float2* st;
    float2* st2;
    uint32_t* id;
    uint32_t* id2;
    int64_t* nb[2];
    int64_t* ne[2];
    uint32_t* ntype[2];
    uint32_t *ntiles, *tile0, *mm, *cntl, *want, *wrank, *nchild, *child0, *tleft, *tleft0, *bsum, *ctr;
    int32_t* choice;
    double* thr;
    int64_t* leaves;
    int64_t Mcap, Tcap;
};

int64_t layout(int64_t N, int w, int64_t tau, int64_t budget, char* base, Bufs* b) {
    Carve cv{base};
    Bufs x{};
    const int64_t A = max_active(N, tau);
    const int64_t Mcap = std::max<int64_t>(2 * A, 2);  // a list holds the children of the active nodes
    const int64_t Tcap = N / kTileElems + A + 1;       // tiles of the active nodes
    const int64_t Scap = std::max(Mcap, Tcap) + 1;
    x.st = cv.take<float2>(N * w);
    x.st2 = cv.take<float2>(N * w);
    x.id = cv.take<uint32_t>(N);
    x.id2 = cv.take<uint32_t>(N);
    for (int k = 0; k < 2; ++k) {
        x.nb[k] = cv.take<int64_t>(Mcap);
        x.ne[k] = cv.take<int64_t>(Mcap);
        x.ntype[k] = cv.take<uint32_t>(Mcap);
    }
    x.ntiles = cv.take<uint32_t>(Mcap);
    x.tile0 = cv.take<uint32_t>(Mcap + 1);
    x.mm = cv.take<uint32_t>(Mcap * 4 * w);
    x.cntl = cv.take<uint32_t>(Mcap * 2 * w);
    x.choice = cv.take<int32_t>(Mcap);
    x.thr = cv.take<double>(Mcap);
    x.want = cv.take<uint32_t>(Mcap);
    x.wrank = cv.take<uint32_t>(Mcap + 1);
    x.nchild = cv.take<uint32_t>(Mcap);
    x.child0 = cv.take<uint32_t>(Mcap + 1);
    x.tleft = cv.take<uint32_t>(Tcap);
    x.tleft0 = cv.take<uint32_t>(Tcap + 1);
    x.bsum = cv.take<uint32_t>(Scap / kScanBlock + 2);
    x.leaves = cv.take<int64_t>(budget);
    x.ctr = cv.take<uint32_t>(64);
    x.Mcap = Mcap;
    x.Tcap = Tcap;
    if (b) *b = x;
    return cv.used;
}

inline unsigned blocks_for(int64_t n, int block) { return (unsigned)std::max<int64_t>(1, (n + block - 1) / block); }

}  // namespace

hipError_t exclusive_scan(const uint32_t* in, int64_t n, uint32_t* out, uint32_t* bsum, hipStream_t st) {
    const int64_t nb = std::max<int64_t>(1, (n + kScanBlock - 1) / kScanBlock);
    hipLaunchKernelGGL(k_scan_blocks, dim3((unsigned)nb), dim3(256), 0, st, in, n, out, bsum);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, st, bsum, nb);
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(256), 0, st, out, n, bsum);
    return hipGetLastError();
}

hipError_t launch_exclusive_scan(const uint32_t* in, int64_t n, uint32_t* out, uint32_t* bsum, hipStream_t st) {
    return exclusive_scan(in, n, out, bsum, st);
}

int64_t partition_scratch_bytes(int64_t N, int w, int64_t tau, int64_t budget) {
    return layout(N, w, tau, budget, nullptr, nullptr);
}

float2* partition_stats_buffer(char* scratch, int64_t N, int w, int64_t tau, int64_t budget) {
    Bufs b;
    layout(N, w, tau, budget, scratch, &b);
    return b.st;
}

hs_status partition_device(int64_t N, int w, int64_t tau, int64_t budget, char* scratch, int cus,
                           uint32_t* ids_out, std::vector<int64_t>* leaf_starts, hipStream_t st) {
    Bufs B;
    layout(N, w, tau, budget, scratch, &B);
    const unsigned tile_grid = (unsigned)std::max(1, cus * 8);
    hipLaunchKernelGGL(k_iota, dim3(blocks_for(N, 256 * 4)), dim3(256), 0, st, B.id, N);
    hipLaunchKernelGGL(k_root, dim3(1), dim3(64), 0, st, B.nb[0], B.ne[0], B.ntype[0], N, B.ctr);
    HIP_TRY(hipGetLastError());
    int64_t M = 1;
    int cur = 0;
    uint32_t host_ctr[2] = {0u, 0u};
    auto done = [&](hs_status s) { return s; };
    // every split makes its node's children strictly smaller: at most N levels
    for (int64_t level = 0; M > 0; ++level) {
        if (level > N + 1 || M > B.Mcap)
            return done(fail(HS_EHIP, "partition: node list overflow at level %lld", (long long)level));
        Level lv{};
        lv.nb = B.nb[cur];
        lv.ne = B.ne[cur];
        lv.ntype = B.ntype[cur];
        lv.nb2 = B.nb[cur ^ 1];
        lv.ne2 = B.ne[cur ^ 1];
        lv.ntype2 = B.ntype[cur ^ 1];
        lv.M = M;
        lv.ntiles = B.ntiles;
        lv.tile0 = B.tile0;
        lv.mm = B.mm;
        lv.cntl = B.cntl;
        lv.choice = B.choice;
        lv.thr = B.thr;
        lv.want = B.want;
        lv.wrank = B.wrank;
        lv.nchild = B.nchild;
        lv.child0 = B.child0;
        lv.tleft = B.tleft;
        lv.tleft0 = B.tleft0;
        lv.st = B.st;
        lv.id = B.id;
        lv.st2 = B.st2;
        lv.id2 = B.id2;
        lv.leaves = B.leaves;
        lv.ctr = B.ctr;
        lv.N = N;
        lv.tau = tau;
        lv.budget = budget;
        lv.w = w;
        const unsigned ng = blocks_for(M, 256);
        hipLaunchKernelGGL(k_classify, dim3(ng), dim3(256), 0, st, lv);
        HIP_TRY(exclusive_scan(B.ntiles, M, B.tile0, B.bsum, st));
        hipLaunchKernelGGL(k_tile_stats<false>, dim3(tile_grid), dim3(256), 0, st, lv);
        hipLaunchKernelGGL(k_tile_stats<true>, dim3(tile_grid), dim3(256), 0, st, lv);
        hipLaunchKernelGGL(k_choose, dim3(ng), dim3(256), 0, st, lv);
        HIP_TRY(exclusive_scan(B.want, M, B.wrank, B.bsum, st));
        hipLaunchKernelGGL(k_budget_snapshot, dim3(1), dim3(64), 0, st, B.ctr);
        hipLaunchKernelGGL(k_apply, dim3(ng), dim3(256), 0, st, lv);
        hipLaunchKernelGGL(k_tile_left, dim3(tile_grid), dim3(256), 0, st, lv);
        // tiles of this level: tile0[M] (scan over at most Tcap tiles)
        HIP_TRY(hipMemcpyAsync(host_ctr, B.tile0 + M, 4, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        const int64_t tiles = host_ctr[0];
        if (tiles > B.Tcap)
            return done(fail(HS_EHIP, "partition: tile list overflow at level %lld", (long long)level));
        HIP_TRY(exclusive_scan(B.tleft, tiles, B.tleft0, B.bsum, st));
        hipLaunchKernelGGL(k_scatter, dim3(tile_grid), dim3(256), 0, st, lv);
        hipLaunchKernelGGL(k_copyback, dim3(tile_grid), dim3(256), 0, st, lv);
        HIP_TRY(exclusive_scan(B.nchild, M, B.child0, B.bsum, st));
        hipLaunchKernelGGL(k_next, dim3(ng), dim3(256), 0, st, lv);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(host_ctr, B.child0 + M, 4, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(host_ctr + 1, B.ctr, 4, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        M = host_ctr[0];
        cur ^= 1;
    }
    const int64_t L = host_ctr[1];
    if (L > budget) return done(fail(HS_EHIP, "partition: %lld leaves above the budget %lld", (long long)L,
                                     (long long)budget));
    leaf_starts->resize((size_t)L);
    HIP_TRY(hipMemcpyAsync(leaf_starts->data(), B.leaves, sizeof(int64_t) * L, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(ids_out, B.id, sizeof(uint32_t) * N, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    std::sort(leaf_starts->begin(), leaf_starts->end());
    return done(HS_OK);
}

}  // namespace hs
