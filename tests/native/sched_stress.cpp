// Host-only stress of the serving loop's admission scheduler (hs_sched.h),
// built by tests/test_sched_sanitizers.py with AddressSanitizer +
// UndefinedBehaviorSanitizer and, separately, ThreadSanitizer.
//
// Several submitter threads and one dispatcher thread share one Scheduler
// under a mutex, as the server does: submitters submit and sometimes cancel,
// the dispatcher forms batches on idle streams and completes them a little
// later.  Checked at the end: every accepted request ran in exactly one batch
// or was withdrawn, per collection in submission order, in batches that fit
// their region, and no slot is left in use.
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <random>
#include <thread>
#include <vector>

#include "../../paper_2212_13297_amd/csrc/hs_sched.h"

using hs::SchedBatch;
using hs::SchedRequest;
using hs::Scheduler;

namespace {

int fail(const char* what) {
    std::fprintf(stderr, "sched_stress: %s\n", what);
    return 1;
}

}  // namespace

int main() {
    const int C = 3, S = 2, slots = 64, threads = 4, per_thread = 4000;
    std::vector<std::array<int, hs::kKBuckets>> max_q(C);
    for (int c = 0; c < C; ++c)
        for (int b = 0; b < hs::kKBuckets; ++b) max_q[c][b] = b < 6 ? (16 >> (b / 2)) : (c == 0 ? 1 : 0);
    Scheduler sched(C, S, slots, max_q);
    std::mutex mu;
    std::atomic<int> submitters_left{threads};
    std::map<uint64_t, int> ran;        // tag -> batches it ran in
    std::map<uint64_t, int> withdrawn;  // tag -> 1
    std::map<uint64_t, int> coll_of;
    std::vector<std::vector<uint64_t>> order(C);  // submission order per collection (tags)
    std::vector<std::vector<uint64_t>> seen(C);   // batch order per collection
    int bad_fit = 0;

    auto submitter = [&](int id) {
        std::mt19937_64 rng(1234 + id);
        for (int i = 0; i < per_thread; ++i) {
            const uint64_t tag = ((uint64_t)id << 32) | (uint64_t)i;
            SchedRequest r;
            r.tag = tag;
            r.coll = (int)(rng() % C);
            r.k = 1 + (int)(rng() % (r.coll == 0 ? 128 : 32));
            for (;;) {
                std::lock_guard<std::mutex> g(mu);
                const int rc = sched.submit(r);
                if (rc == 0) {
                    coll_of[tag] = r.coll;
                    order[r.coll].push_back(tag);
                    break;
                }
                if (rc != 1) std::abort();
            }
            if (rng() % 7 == 0) {
                std::lock_guard<std::mutex> g(mu);
                SchedRequest w;
                if (sched.cancel(tag, &w) == 0) {
                    if (w.tag != tag) std::abort();
                    withdrawn[tag] = 1;
                }
            }
        }
        submitters_left.fetch_sub(1);
    };

    std::vector<SchedBatch> running(C * S);
    std::vector<int> busy(C * S, 0);
    auto dispatcher = [&]() {
        std::mt19937_64 rng(99);
        for (;;) {
            bool any = false;
            {
                std::lock_guard<std::mutex> g(mu);
                for (int c = 0; c < C; ++c)
                    for (int s = 0; s < S; ++s) {
                        const int i = c * S + s;
                        if (busy[i]) {
                            any = true;
                            if (rng() % 3 == 0) {  // the batch completes
                                sched.complete(c, s);
                                busy[i] = 0;
                            }
                            continue;
                        }
                        SchedBatch b;
                        if (!sched.next(c, s, &b)) continue;
                        any = true;
                        if ((int)b.reqs.size() > max_q[c][hs::k_bucket(b.k_batch)]) ++bad_fit;
                        for (auto& r : b.reqs) {
                            ran[r.tag] += 1;
                            seen[c].push_back(r.tag);
                            if (r.k > b.k_batch) ++bad_fit;
                        }
                        busy[i] = 1;
                    }
                if (!any && submitters_left.load() == 0 && sched.in_system() == 0) return;
            }
            std::this_thread::yield();
        }
    };

    std::thread d(dispatcher);
    std::vector<std::thread> ts;
    for (int i = 0; i < threads; ++i) ts.emplace_back(submitter, i);
    for (auto& t : ts) t.join();
    d.join();

    if (bad_fit) return fail("a batch exceeded its region or a request's k");
    if (sched.in_system() != 0) return fail("slots left in use");
    for (auto& kv : coll_of) {
        const int r = ran.count(kv.first) ? ran[kv.first] : 0;
        const int w = withdrawn.count(kv.first) ? 1 : 0;
        if (r + w != 1) return fail("a request neither ran once nor was withdrawn");
    }
    for (int c = 0; c < C; ++c) {
        std::vector<uint64_t> expect;
        for (auto t : order[c])
            if (!withdrawn.count(t)) expect.push_back(t);
        if (expect != seen[c]) return fail("batch order differs from submission order");
    }
    std::printf("sched_stress ok: %zu requests, %zu withdrawn\n", coll_of.size(), withdrawn.size());
    return 0;
}
