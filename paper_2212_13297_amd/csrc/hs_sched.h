// Admission scheduler of the serving loop: host logic only (no HIP calls), so
// it is tested on the CPU through the hs_sched_* entry points.
//
// Requests of C collections wait in one FIFO per collection.  Each collection
// has S streams; each stream owns a fixed region of the device budget that
// holds one batch's query workspace and I/O.  A request occupies one of
// max_slots slots from submission until its batch completes (submit reports
// busy when none is free).  When a stream of collection c is idle, next()
// forms a batch from the head of c's FIFO: requests are taken in order while
// the batch still fits the region at the batch's k bucket (k rounded up to a
// power of two, the largest k of the batch); the batch runs with that k and
// Q rounded up to a power of two, the shapes whose captured graphs are reused.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <array>
#include <deque>
#include <vector>

namespace hs {

constexpr int kKBuckets = 8;  // k buckets 1, 2, 4, ..., 128

inline int k_bucket(int k) {
    int b = 0;
    while ((1 << b) < k) ++b;
    return b;
}

inline int pow2_ceil(int v) {
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

struct SchedRequest {
    uint64_t tag = 0;
    int32_t coll = 0;
    int32_t k = 1;
    int64_t seq = 0;       // submission order (server-internal key of the query data)
    double t_submit = 0.0;
};

struct SchedBatch {
    int32_t coll = -1;
    int32_t stream = -1;
    int32_t q_pad = 0;    // batch size the kernels run with (power of two >= reqs.size())
    int32_t k_batch = 0;  // k the kernels run with (power of two >= every request's k)
    std::vector<SchedRequest> reqs;
};

class Scheduler {
public:
    // max_q[c][b]: largest batch (a power of two; 0 = none fits) a stream region
    // of collection c holds at k bucket b.
    Scheduler(int colls, int streams, int max_slots, const std::vector<std::array<int, kKBuckets>>& max_q)
        : colls_(colls), streams_(streams), max_slots_(max_slots), max_q_(max_q), pending_(colls),
          busy_(colls * streams, 0), inflight_(colls * streams, 0) {}

    // 0 = queued, 1 = busy (no free slot), 2 = k beyond what the collection's
    // regions hold, 3 = bad collection
    int submit(const SchedRequest& r) {
        if (r.coll < 0 || r.coll >= colls_) return 3;
        if (r.k < 1 || k_bucket(r.k) >= kKBuckets || max_q_[r.coll][k_bucket(r.k)] < 1) return 2;
        if (used_ >= max_slots_) return 1;
        ++used_;
        pending_[r.coll].push_back(r);
        return 0;
    }

    bool next(int coll, int stream, SchedBatch* out) {
        if (coll < 0 || coll >= colls_ || stream < 0 || stream >= streams_) return false;
        const int s = coll * streams_ + stream;
        auto& q = pending_[coll];
        if (busy_[s] || q.empty()) return false;
        out->coll = coll;
        out->stream = stream;
        out->reqs.clear();
        int kb = 0;
        while (!q.empty()) {
            const int nkb = std::max(kb, k_bucket(q.front().k));
            const int cap = max_q_[coll][nkb];
            if ((int)out->reqs.size() + 1 > cap) break;
            out->reqs.push_back(q.front());
            q.pop_front();
            kb = nkb;
        }
        out->q_pad = pow2_ceil((int)out->reqs.size());
        out->k_batch = 1 << kb;
        busy_[s] = 1;
        inflight_[s] = (int)out->reqs.size();
        return true;
    }

    // Withdraw the oldest queued request with this tag (searching every
    // collection): 0 = withdrawn (*out holds it; its slot is free again),
    // 1 = none queued.  A request already in a batch is not queued any more.
    int cancel(uint64_t tag, SchedRequest* out) {
        for (auto& q : pending_) {
            for (auto it = q.begin(); it != q.end(); ++it) {
                if (it->tag != tag) continue;
                if (out) *out = *it;
                q.erase(it);
                --used_;
                return 0;
            }
        }
        return 1;
    }

    void complete(int coll, int stream) {
        if (coll < 0 || coll >= colls_ || stream < 0 || stream >= streams_) return;
        const int s = coll * streams_ + stream;
        if (!busy_[s]) return;
        used_ -= inflight_[s];
        inflight_[s] = 0;
        busy_[s] = 0;
    }

    int in_system() const { return used_; }
    int pending(int coll) const { return (coll >= 0 && coll < colls_) ? (int)pending_[coll].size() : 0; }
    bool busy(int coll, int stream) const { return busy_[coll * streams_ + stream] != 0; }
    int colls() const { return colls_; }
    int streams() const { return streams_; }

private:
    int colls_, streams_, max_slots_;
    std::vector<std::array<int, kKBuckets>> max_q_;
    std::vector<std::deque<SchedRequest>> pending_;
    std::vector<int> busy_, inflight_;
    int used_ = 0;
};

}  // namespace hs
