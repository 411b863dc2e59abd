/*
 * Oracle (test infrastructure only): FP64 brute-force exact k-NN.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg use
 * this file; the search library never links or calls it.
 *
 * What it computes is the plain definition of a k-NN query under the squared
 * Euclidean distance (Hercules, Sec. 2, k-NN query definition; whole matching
 * with Euclidean distance): for each query the k series with the smallest
 *     d(q, x) = sum_j (double(q_j) - double(x_j))^2,
 * ties broken by the smaller row index, returned in ascending (d, id) order.
 * The sum runs over j = 0..n-1 in order, in FP64, for every (query, series)
 * pair; nothing is pruned, abandoned or reordered.
 *
 * Parallelism (OpenMP) only splits the series range into contiguous parts,
 * each with its own per-query top-k list; the parts are merged at the end by
 * the same (d, id) order, so the result does not depend on the thread count.
 *
 * Return value: 0 on success, -1 on invalid arguments (N < 1, n < 1, Q < 0,
 * k < 1, k > N, null pointers), -2 if scratch memory cannot be allocated.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double d;
    int64_t id;
} pair_t;

static int pair_less(double d, int64_t id, const pair_t* p) {
    return d < p->d || (d == p->d && id < p->id);
}

/* Insert (d, id) into the ascending list top[0..k-1] if it precedes top[k-1]. */
static void topk_insert(pair_t* top, int k, double d, int64_t id) {
    if (!pair_less(d, id, &top[k - 1])) return;
    int i = k - 1;
    while (i > 0 && pair_less(d, id, &top[i - 1])) {
        top[i] = top[i - 1];
        --i;
    }
    top[i].d = d;
    top[i].id = id;
}

int oracle_knn_brute(const float* x, int64_t N, int32_t n, const float* q, int32_t Q, int32_t k,
                     int64_t* ids, double* d2, int32_t threads) {
    if (!x || !q || !ids || !d2 || N < 1 || n < 1 || Q < 0 || k < 1 || (int64_t)k > N) return -1;
    if (Q == 0) return 0;
    int T = 1;
#ifdef _OPENMP
    T = threads > 0 ? threads : omp_get_max_threads();
#endif
    if ((int64_t)T > N) T = (int)N;
    pair_t* all = (pair_t*)malloc(sizeof(pair_t) * (size_t)T * (size_t)Q * (size_t)k);
    if (!all) return -2;
    for (size_t i = 0; i < (size_t)T * (size_t)Q * (size_t)k; ++i) {
        all[i].d = INFINITY;
        all[i].id = INT64_MAX;
    }
    const int64_t BLOCK = 512; /* series per block: each block is reused by every query */

#ifdef _OPENMP
#pragma omp parallel num_threads(T)
#endif
    {
        int t = 0;
#ifdef _OPENMP
        t = omp_get_thread_num();
#endif
        int64_t lo = N * t / T, hi = N * (t + 1) / T;
        pair_t* mine = all + (size_t)t * (size_t)Q * (size_t)k;
        for (int64_t b = lo; b < hi; b += BLOCK) {
            int64_t e = b + BLOCK < hi ? b + BLOCK : hi;
            for (int32_t qi = 0; qi < Q; ++qi) {
                const float* qq = q + (size_t)qi * (size_t)n;
                pair_t* top = mine + (size_t)qi * (size_t)k;
                for (int64_t r = b; r < e; ++r) {
                    const float* xx = x + (size_t)r * (size_t)n;
                    double s = 0.0;
                    for (int32_t j = 0; j < n; ++j) {
                        double diff = (double)qq[j] - (double)xx[j];
                        s += diff * diff;
                    }
                    topk_insert(top, k, s, r);
                }
            }
        }
    }

    /* merge the per-part lists */
    for (int32_t qi = 0; qi < Q; ++qi) {
        pair_t* out = all + (size_t)qi * (size_t)k; /* part 0's list is the accumulator */
        for (int t = 1; t < T; ++t) {
            const pair_t* src = all + ((size_t)t * (size_t)Q + (size_t)qi) * (size_t)k;
            for (int32_t i = 0; i < k; ++i) topk_insert(out, k, src[i].d, src[i].id);
        }
        for (int32_t i = 0; i < k; ++i) {
            ids[(size_t)qi * k + i] = out[i].id;
            d2[(size_t)qi * k + i] = out[i].d;
        }
    }
    free(all);
    return 0;
}

/* FP64 squared distances for given (query, row) pairs, same summation order as
 * above: out[p] = d(q[qidx[p]], x[rows[p]]).  Used to check sampled outputs at
 * sizes where a full brute-force scan would be too slow. */
int oracle_pair_dist(const float* x, int64_t N, int32_t n, const float* q, int32_t Q,
                     const int32_t* qidx, const int64_t* rows, int64_t P, double* out) {
    if (!x || !q || !qidx || !rows || !out || n < 1 || P < 0) return -1;
    for (int64_t p = 0; p < P; ++p) {
        if (qidx[p] < 0 || qidx[p] >= Q || rows[p] < 0 || rows[p] >= N) return -1;
    }
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
    for (int64_t p = 0; p < P; ++p) {
        const float* qq = q + (size_t)qidx[p] * (size_t)n;
        const float* xx = x + (size_t)rows[p] * (size_t)n;
        double s = 0.0;
        for (int32_t j = 0; j < n; ++j) {
            double diff = (double)qq[j] - (double)xx[j];
            s += diff * diff;
        }
        out[p] = s;
    }
    return 0;
}

/* Threads the OpenMP runtime would use for the calls above (threads <= 0). */
int oracle_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
