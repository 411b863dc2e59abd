// Fused filter + refine per (query, part) item (Hercules Sec. 3.4, steps 3
// and 4 without a candidate list): the path of queries whose candidate list
// or result pool overflowed.  Work is split into contiguous static ranges per
// workgroup; items are ordered by query, so the query row and LB_SAX table
// are reloaded only when the query changes.
#include "hs_device.h"

namespace hs {
namespace {

struct ScanShared {
    unsigned long long top[HS_KMAX];
    unsigned long long res[kTile];
    uint32_t hits[kTile];
    int w[4];
    int nres, topn;
    float thr;  // block-uniform pruning threshold (a valid upper bound of BSF_k)
    unsigned int st_filt, st_ref, st_chunks;
};

template <int W16, int F>
__global__ void __launch_bounds__(256) k_leaf_scan(IndexView ix, ScanParams sp, QueryWs ws) {
    extern __shared__ float s_dyn[];
    __shared__ ScanShared sh;
    float* s_q = s_dyn;                // [stride]
    float* s_lut = s_dyn + ix.stride;  // [16 W16][256]
    const int t = threadIdx.x;
    const int grp = t >> 4, sub = t & 15;
    const int nchunks = ix.stride / kChunk;
    const int k = sp.k;
    int64_t i0, i1;
    block_range(min((int64_t)ws.counters[kCtrItems], ws.item_cap), i0, i1);
    int cur_q = -1;

    for (int64_t idx = i0; idx < i1; ++idx) {
        const uint64_t item = ws.items[idx];
        const int q = (int)(item >> 32);
        const int64_t part = (int64_t)(uint32_t)item;
        if (q != cur_q) {
            for (int j = t; j < ix.stride; j += blockDim.x) s_q[j] = ws.qrow[(int64_t)q * ix.stride + j];
            load_lut<W16>(s_lut, ws.lut + (int64_t)q * ix.w * kCard, ix.w, t, blockDim.x);
            cur_q = q;
        }
        if (t == 0) {
            sh.topn = 0;
            sh.nres = 0;
            sh.st_filt = 0;
            sh.st_ref = 0;
            sh.st_chunks = 0;
            sh.thr = bits_to_float(bsf_bits(ws, q));
        }
        const bool skip_sax = (ws.flags[q] & kFlagSkipSax) != 0;
        const int64_t b = ix.part_start[part], e = ix.part_start[part + 1];
        unsigned int my_filt = 0, my_ref = 0, my_chunks = 0;
        __syncthreads();
        float thr = sh.thr;

        for (int64_t tb = b; tb < e; tb += kTile) {
            const int64_t r = tb + t;
            bool pass = false;
            if (r < e) {
                if (skip_sax) {
                    pass = true;
                } else {
                    uint4 v[W16];
                    load_word<W16>(ix.words + r * ix.wstride, v);
                    const float lb = lb_sax_word<W16>(v, s_lut);
                    ++my_filt;
                    pass = (double)lb <= prune_limit(thr);
                }
            }
            int nh;
            const int off = block_exclusive_scan(pass ? 1 : 0, sh.w, &nh);
            if (pass) sh.hits[off] = (uint32_t)(r - b);
            __syncthreads();
            for (int h = grp; h < nh; h += kTile / 16) {
                const int64_t pos = b + sh.hits[h];
                bool alive;
                const float d = refine_row<F>(ix.rows + pos * ix.stride + sub * 4, s_q + sub * 4, nchunks,
                                              thr * sp.marg, alive, my_chunks);
                if (sub == 0) {
                    ++my_ref;
                    if (alive)
                        sh.res[atomicAdd(&sh.nres, 1)] = ((unsigned long long)__float_as_uint(d) << 32) | ix.ids[pos];
                }
            }
            __syncthreads();
            if (t == 0) {
                int n = sh.topn;
                for (int i = 0; i < sh.nres; ++i) topk_insert(sh.top, n, k, sh.res[i]);
                sh.topn = n;
                sh.nres = 0;
                const float g = bits_to_float(bsf_bits(ws, q));
                const float lk = n == k ? bits_to_float((uint32_t)(sh.top[k - 1] >> 32)) : INFINITY;
                sh.thr = fminf(g, lk);
            }
            __syncthreads();
            thr = sh.thr;
        }

        atomicAdd(&sh.st_filt, my_filt);
        if (sub == 0) {
            atomicAdd(&sh.st_ref, my_ref);
            atomicAdd(&sh.st_chunks, my_chunks);
        }
        __syncthreads();
        if (t == 0) {
            flush_topk(ws, q, k, sh.top, sh.topn);
            unsigned long long* st = ws.stats + (int64_t)q * kStatSlots;
            atomicAdd(&st[1], (unsigned long long)sh.st_filt);
            atomicAdd(&st[2], (unsigned long long)sh.st_ref);
            atomicAdd(&st[3], (unsigned long long)sh.st_chunks);
        }
        __syncthreads();
    }
}

}  // namespace

hipError_t launch_leaf_scan(const IndexView& ix, const ScanParams& sp, const QueryWs& ws, int device_cus, int form,
                            hipStream_t st) {
    const size_t lds = sizeof(float) * ((size_t)ix.stride + (size_t)16 * w16_of(ix) * kCard);
    if (form == kComp) {
        HS_LAUNCH_RESIDENT_F(ix, k_leaf_scan, kComp, lds, device_cus, st, ix, sp, ws);
    } else {
        HS_LAUNCH_RESIDENT_F(ix, k_leaf_scan, kPlain, lds, device_cus, st, ix, sp, ws);
    }
    return hipGetLastError();
}

}  // namespace hs
