// Serving form: a continuous-batching request loop over several collections.
//
// hs_submit queues a request (host copy of the query, k, tag) if one of
// max_slots slots is free.  A dispatcher thread forms a batch whenever a
// stream of the request's collection is idle (hs_sched.h), copies its queries
// to pinned memory and launches the whole query path as one captured HIP
// graph, cached per (stream, batch size, k): host-to-device copy of the
// queries, steps 1-4 and the merge, device-to-host copies of the results and
// of the overflow counters.  Batches of different collections, and of the
// same collection on its other streams, run concurrently on the device while
// new requests keep arriving; a request never waits for a batch it is not in.
// When a graph's event has completed, the dispatcher finishes the rare
// overflow rounds eagerly, then hands out one completion per request (its
// first k of the batch's sorted top-k_batch, which are its exact top-k).
//
// Every batch's device state (query rows, LB tables, BSF_k, pools, candidate
// lists) lives in the stream's fixed region of the caller's budget buffer, so
// captured graphs stay valid from batch to batch.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <utility>
#include <vector>

#include "hs_host.h"
#include "hs_sched.h"

using namespace hs;

namespace {

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct GraphEntry {
    hipGraphExec_t exec = nullptr;
    KnnCall call;
};

struct StreamSlot {
    int coll = 0;
    int index = 0;  // stream index within the collection
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    char* region = nullptr;
    int64_t region_bytes = 0;
    int qmax = 0;
    float* q_dev = nullptr;
    int64_t* ids_dev = nullptr;
    float* d2_dev = nullptr;
    double* err_dev = nullptr;
    char* ws_dev = nullptr;
    int64_t ws_bytes = 0;
    float* q_host = nullptr;  // pinned
    int64_t* ids_host = nullptr;
    float* d2_host = nullptr;
    double* err_host = nullptr;
    uint32_t* redo_host = nullptr;
    bool busy = false;
    SchedBatch batch;
    GraphEntry* running = nullptr;
    int k_run = 0;
    double t_launch = 0.0;
    std::map<std::pair<int, int>, GraphEntry> graphs;
};

// I/O part of a region for q queries of length n: queries, ids, d2, err.
int64_t io_bytes(int q, int n) {
    return align_up((int64_t)q * n * 4, 256) + align_up((int64_t)q * HS_KMAX * 8, 256) +
           align_up((int64_t)q * HS_KMAX * 4, 256) + align_up((int64_t)q * HS_KMAX * 8, 256);
}

}  // namespace

struct hs_server {
    int device = 0;
    int C = 0;
    int S = 1;
    std::vector<hs_index*> idx;
    std::vector<int> form;  // 0 plain, 1 precision
    std::vector<StreamSlot> slots;
    Scheduler* sched = nullptr;
    std::mutex mu;
    std::condition_variable cv;
    std::unordered_map<int64_t, std::vector<float>> qdata;
    std::deque<hs_completion> done;
    int64_t seq = 0;
    std::atomic<bool> stop{false};
    std::thread th;
    std::string error;  // first dispatcher failure (guarded by mu)
    int64_t launched_batches = 0, launched_queries = 0, padded_queries = 0, graphs_built = 0;
};

namespace {

void record_error(hs_server* s, const std::string& msg) {
    std::lock_guard<std::mutex> g(s->mu);
    if (s->error.empty()) s->error = msg;
}

// Capture (once per shape) and launch the graph of slot's current batch.
hs_status launch_batch(hs_server* s, StreamSlot& sl) {
    hs_index* idx = s->idx[sl.coll];
    const int n = idx->view.n;
    const SchedBatch& b = sl.batch;
    const int k_run = (int)std::min<int64_t>(b.k_batch, idx->view.N);
    const int qp = b.q_pad;
    auto key = std::make_pair(qp, k_run);
    auto it = sl.graphs.find(key);
    if (it == sl.graphs.end()) {
        GraphEntry ge;
        hs_status st = knn_prepare(idx, qp, k_run, sl.ws_dev, sl.ws_bytes, s->form[sl.coll] != 0, &ge.call);
        if (st) return st;
        HIP_TRY(hipStreamBeginCapture(sl.st, hipStreamCaptureModeThreadLocal));
        hipError_t e = hipMemcpyAsync(sl.q_dev, sl.q_host, (size_t)qp * n * 4, hipMemcpyHostToDevice, sl.st);
        hs_status hs_st = e == hipSuccess ? HS_OK : fail(HS_EHIP, "capture: %s", hipGetErrorString(e));
        if (!hs_st)
            hs_st = knn_enqueue(ge.call, sl.q_dev, sl.ids_dev, sl.d2_dev, sl.err_dev,
                                nullptr, sl.st, sl.redo_host, nullptr);
        if (!hs_st) {
            e = hipMemcpyAsync(sl.ids_host, sl.ids_dev, (size_t)qp * k_run * 8, hipMemcpyDeviceToHost, sl.st);
            if (e == hipSuccess)
                e = hipMemcpyAsync(sl.d2_host, sl.d2_dev, (size_t)qp * k_run * 4, hipMemcpyDeviceToHost, sl.st);
            if (e == hipSuccess)
                e = hipMemcpyAsync(sl.err_host, sl.err_dev, (size_t)qp * k_run * 8, hipMemcpyDeviceToHost, sl.st);
            if (e != hipSuccess) hs_st = fail(HS_EHIP, "capture: %s", hipGetErrorString(e));
        }
        hipGraph_t graph = nullptr;
        e = hipStreamEndCapture(sl.st, &graph);
        if (hs_st) {
            if (graph) (void)hipGraphDestroy(graph);
            return hs_st;
        }
        HIP_TRY(e);
        e = hipGraphInstantiate(&ge.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        HIP_TRY(e);
        it = sl.graphs.emplace(key, ge).first;
        s->graphs_built++;
    }
    sl.running = &it->second;
    sl.k_run = k_run;
    HIP_TRY(hipGraphLaunch(it->second.exec, sl.st));
    HIP_TRY(hipEventRecord(sl.ev, sl.st));
    sl.t_launch = now_s();
    return HS_OK;
}

// The slot's graph has completed: overflow rounds, then completions.
// failed: the batch could not be launched (its requests complete with that status).
void finish_batch(hs_server* s, StreamSlot& sl, hs_status failed = HS_OK) {
    const SchedBatch& b = sl.batch;
    const int k_run = sl.k_run;
    const int qp = b.q_pad;
    hs_status status = failed;
    std::string msg;
    if (failed) {
        msg = "batch launch failed";
    } else if (sl.redo_host[1]) {
        status = HS_EINVAL;
        msg = "non-finite query in a batch";
    } else if (sl.redo_host[0]) {
        const KnnCall& c = sl.running->call;
        status = knn_finish(c, sl.ids_dev, sl.d2_dev, sl.err_dev, nullptr, sl.st, nullptr);
        hipError_t e = hipSuccess;
        if (!status) e = hipMemcpyAsync(sl.ids_host, sl.ids_dev, (size_t)qp * k_run * 8, hipMemcpyDeviceToHost, sl.st);
        if (!status && e == hipSuccess)
            e = hipMemcpyAsync(sl.d2_host, sl.d2_dev, (size_t)qp * k_run * 4, hipMemcpyDeviceToHost, sl.st);
        if (!status && e == hipSuccess)
            e = hipMemcpyAsync(sl.err_host, sl.err_dev, (size_t)qp * k_run * 8, hipMemcpyDeviceToHost, sl.st);
        if (!status && e == hipSuccess) e = hipStreamSynchronize(sl.st);
        if (!status && e != hipSuccess) status = fail(HS_EHIP, "overflow round: %s", hipGetErrorString(e));
        if (status) msg = hs_last_error();
    }
    const double t_done = now_s();
    std::vector<hs_completion> out(b.reqs.size());
    for (size_t i = 0; i < b.reqs.size(); ++i) {
        hs_completion& c = out[i];
        std::memset(&c, 0, sizeof c);
        const SchedRequest& r = b.reqs[i];
        c.tag = r.tag;
        c.coll = r.coll;
        c.k = r.k;
        c.status = status;
        c.batch = (int32_t)b.reqs.size();
        c.t_submit = r.t_submit;
        c.t_launch = sl.t_launch;
        c.t_done = t_done;
        for (int j = 0; j < r.k; ++j) {
            c.ids[j] = sl.ids_host[i * k_run + j];
            c.d2[j] = sl.d2_host[i * k_run + j];
            c.err[j] = sl.err_host[i * k_run + j];
        }
    }
    std::lock_guard<std::mutex> g(s->mu);
    if (status && s->error.empty()) s->error = msg;
    for (auto& c : out) s->done.push_back(c);
    s->sched->complete(sl.coll, sl.index);
    sl.batch.reqs.clear();  // hs_cancel looks for running requests here (under mu)
    sl.busy = false;
    sl.running = nullptr;
}

void dispatcher(hs_server* s) {
    if (hipSetDevice(s->device) != hipSuccess) {
        record_error(s, "dispatcher: hipSetDevice failed");
        return;
    }
    int rr = 0;
    while (true) {
        bool progress = false, inflight = false;
        for (auto& sl : s->slots) {
            if (!sl.busy) continue;
            const hipError_t e = hipEventQuery(sl.ev);
            if (e == hipSuccess) {
                finish_batch(s, sl);
                progress = true;
            } else if (e == hipErrorNotReady) {
                inflight = true;
            } else {
                record_error(s, std::string("dispatcher: ") + hipGetErrorString(e));
                (void)hipStreamSynchronize(sl.st);
                finish_batch(s, sl, HS_EHIP);
            }
        }
        if (s->stop.load() && !inflight) {
            std::lock_guard<std::mutex> g(s->mu);
            bool any = false;
            for (auto& sl : s->slots) any = any || sl.busy;
            if (!any) break;
        }
        if (!s->stop.load()) {
            for (int cc = 0; cc < s->C; ++cc) {
                const int c = (rr + cc) % s->C;
                for (int j = 0; j < s->S; ++j) {
                    StreamSlot& sl = s->slots[c * s->S + j];
                    if (sl.busy) continue;
                    {
                        std::lock_guard<std::mutex> g(s->mu);
                        if (!s->sched->next(c, j, &sl.batch)) continue;
                        const int n = s->idx[c]->view.n;
                        for (size_t i = 0; i < sl.batch.reqs.size(); ++i) {
                            auto f = s->qdata.find(sl.batch.reqs[i].seq);
                            std::memcpy(sl.q_host + i * n, f->second.data(), sizeof(float) * n);
                            s->qdata.erase(f);
                        }
                        for (int i = (int)sl.batch.reqs.size(); i < sl.batch.q_pad; ++i)
                            std::memcpy(sl.q_host + (size_t)i * n, sl.q_host, sizeof(float) * n);
                        s->launched_batches++;
                        s->launched_queries += (int64_t)sl.batch.reqs.size();
                        s->padded_queries += sl.batch.q_pad;
                    }
                    sl.busy = true;
                    const hs_status st = launch_batch(s, sl);
                    if (st) {
                        record_error(s, std::string("launch: ") + hs_last_error());
                        // complete the requests with the error
                        sl.redo_host[0] = sl.redo_host[1] = 0;
                        for (int i = 0; i < sl.batch.q_pad * HS_KMAX; ++i) {
                            sl.ids_host[i] = -1;
                            sl.d2_host[i] = INFINITY;
                        }
                        sl.k_run = std::max(1, sl.batch.k_batch);
                        finish_batch(s, sl, st);
                    }
                    progress = true;
                }
            }
            rr = (rr + 1) % std::max(1, s->C);
        }
        if (!progress) {
            std::unique_lock<std::mutex> g(s->mu);
            bool busy_any = false;
            for (auto& sl : s->slots) busy_any = busy_any || sl.busy;
            if (busy_any)
                s->cv.wait_for(g, std::chrono::microseconds(20));
            else if (!s->stop.load() && s->sched->in_system() == 0)
                s->cv.wait_for(g, std::chrono::milliseconds(5));
        }
    }
}

void destroy_server(hs_server* s) {
    for (auto& sl : s->slots) {
        for (auto& kv : sl.graphs)
            if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
        if (sl.ev) (void)hipEventDestroy(sl.ev);
        if (sl.st) (void)hipStreamDestroy(sl.st);
        if (sl.q_host) (void)hipHostFree(sl.q_host);
        if (sl.ids_host) (void)hipHostFree(sl.ids_host);
        if (sl.d2_host) (void)hipHostFree(sl.d2_host);
        if (sl.err_host) (void)hipHostFree(sl.err_host);
        if (sl.redo_host) (void)hipHostFree(sl.redo_host);
    }
    delete s->sched;
    delete s;
}

}  // namespace

struct hs_sched {
    Scheduler* s = nullptr;
    SchedBatch scratch;
    int max_batch = 0;  // largest max_q entry
};

extern "C" {

double hs_server_now(void) { return now_s(); }

hs_status hs_server_create(hs_index* const* colls, const int32_t* forms, int32_t C, void* budget_dev,
                           int64_t budget_bytes, const hs_server_config* cfg, hs_server** out) {
    if (!out) return fail(HS_EINVAL, "out is NULL");
    *out = nullptr;
    if (!colls || C < 1 || !budget_dev || !cfg) return fail(HS_EINVAL, "NULL argument or C < 1");
    if (cfg->streams_per_coll < 1 || cfg->streams_per_coll > 8)
        return fail(HS_EINVAL, "streams_per_coll=%d out of range [1, 8]", cfg->streams_per_coll);
    if (cfg->max_slots < 1) return fail(HS_EINVAL, "max_slots=%d < 1", cfg->max_slots);
    if (cfg->max_batch < 1 || cfg->max_batch > 1024 || (cfg->max_batch & (cfg->max_batch - 1)))
        return fail(HS_EINVAL, "max_batch=%d must be a power of two in [1, 1024]", cfg->max_batch);
    for (int c = 0; c < C; ++c) {
        if (!colls[c]) return fail(HS_EINVAL, "collection %d is NULL", c);
        const int f = forms ? forms[c] : 0;
        if (f != 0 && f != 1) return fail(HS_EINVAL, "form %d of collection %d unknown", f, c);
        if (f == 1 && colls[c]->shadow.kind == 0)
            return fail(HS_EINVAL, "collection %d: precision form without a low-precision copy", c);
    }
    hs_server* s = new (std::nothrow) hs_server();
    if (!s) return fail(HS_ENOMEM, "host allocation failed");
    s->C = C;
    s->S = cfg->streams_per_coll;
    s->idx.assign(colls, colls + C);
    for (int c = 0; c < C; ++c) s->form.push_back(forms ? forms[c] : 0);
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return fail(HS_EHIP, "hipGetDevice failed");
    }
    const int64_t region = (budget_bytes / (C * s->S)) / 256 * 256;
    std::vector<std::array<int, kKBuckets>> max_q(C);
    s->slots.resize((size_t)C * s->S);
    char* base = (char*)budget_dev;
    auto bail = [&](hs_status code) {
        destroy_server(s);
        return code;
    };
    for (int c = 0; c < C; ++c) {
        hs_index* ix = colls[c];
        const int n = ix->view.n;
        int qmax = cfg->max_batch;
        while (qmax >= 1 && io_bytes(qmax, n) + ws_layout(ix, qmax, 1, nullptr, nullptr) > region) qmax >>= 1;
        if (qmax < 1)
            return bail(fail(HS_ENOMEM, "budget region %lld bytes too small for one query of collection %d",
                             (long long)region, c));
        const int kcap = (int)std::min<int64_t>(HS_KMAX, ix->view.N);
        for (int b = 0; b < kKBuckets; ++b) {
            const int lo = b == 0 ? 1 : (1 << (b - 1)) + 1;  // smallest k of bucket b
            max_q[c][b] = lo <= kcap ? qmax : 0;
        }
        for (int j = 0; j < s->S; ++j) {
            StreamSlot& sl = s->slots[c * s->S + j];
            sl.coll = c;
            sl.index = j;
            sl.region = base + (int64_t)(c * s->S + j) * region;
            sl.region_bytes = region;
            sl.qmax = qmax;
            char* cur = sl.region;
            sl.q_dev = (float*)cur;
            cur += align_up((int64_t)qmax * n * 4, 256);
            sl.ids_dev = (int64_t*)cur;
            cur += align_up((int64_t)qmax * HS_KMAX * 8, 256);
            sl.d2_dev = (float*)cur;
            cur += align_up((int64_t)qmax * HS_KMAX * 4, 256);
            sl.err_dev = (double*)cur;
            cur += align_up((int64_t)qmax * HS_KMAX * 8, 256);
            sl.ws_dev = cur;
            sl.ws_bytes = region - (cur - sl.region);
            if (hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) != hipSuccess ||
                hipHostMalloc((void**)&sl.q_host, (size_t)qmax * n * 4, hipHostMallocDefault) != hipSuccess ||
                hipHostMalloc((void**)&sl.ids_host, (size_t)qmax * HS_KMAX * 8, hipHostMallocDefault) != hipSuccess ||
                hipHostMalloc((void**)&sl.d2_host, (size_t)qmax * HS_KMAX * 4, hipHostMallocDefault) != hipSuccess ||
                hipHostMalloc((void**)&sl.err_host, (size_t)qmax * HS_KMAX * 8, hipHostMallocDefault) != hipSuccess ||
                hipHostMalloc((void**)&sl.redo_host, 256, hipHostMallocDefault) != hipSuccess)
                return bail(fail(HS_EHIP, "stream or pinned-memory setup failed"));
        }
    }
    s->sched = new (std::nothrow) Scheduler(C, s->S, cfg->max_slots, max_q);
    if (!s->sched) return bail(fail(HS_ENOMEM, "host allocation failed"));
    try {
        s->th = std::thread(dispatcher, s);
    } catch (...) {
        return bail(fail(HS_ENOMEM, "cannot start the dispatcher thread"));
    }
    *out = s;
    return HS_OK;
}

hs_status hs_submit(hs_server* s, int32_t coll, const float* q_host, int32_t k, uint64_t tag) {
    if (!s || !q_host) return fail(HS_EINVAL, "NULL argument");
    if (coll < 0 || coll >= s->C) return fail(HS_EINVAL, "collection %d out of range [0, %d)", coll, s->C);
    hs_index* ix = s->idx[coll];
    if (k < 1 || k > HS_KMAX || (int64_t)k > ix->view.N)
        return fail(HS_EINVAL, "k=%d out of range for collection %d", k, coll);
    const int n = ix->view.n;
    const bool f16 = s->form[coll] && ix->shadow.kind == kShadowF16;
    for (int j = 0; j < n; ++j) {
        if (!std::isfinite(q_host[j])) return fail(HS_EINVAL, "query holds NaN or Inf");
        if (f16 && std::fabs(q_host[j]) > 65504.0f) return fail(HS_EINVAL, "query beyond the fp16 range");
    }
    std::vector<float> data(q_host, q_host + n);
    {
        std::lock_guard<std::mutex> g(s->mu);
        if (!s->error.empty()) return fail(HS_EHIP, "server failed: %s", s->error.c_str());
        SchedRequest r;
        r.tag = tag;
        r.coll = coll;
        r.k = k;
        r.seq = s->seq;
        r.t_submit = now_s();
        const int rc = s->sched->submit(r);
        if (rc == 1) return fail(HS_EBUSY, "all %d slots in use", s->sched->in_system());
        if (rc != 0) return fail(HS_EINVAL, "request rejected (k=%d, collection %d)", k, coll);
        s->qdata.emplace(s->seq, std::move(data));
        s->seq++;
    }
    s->cv.notify_one();
    return HS_OK;
}

hs_status hs_cancel(hs_server* s, uint64_t tag) {
    if (!s) return fail(HS_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> g(s->mu);
    SchedRequest r;
    if (s->sched->cancel(tag, &r) != 0) {
        // launched (it completes normally) or unknown; a slot's batch is
        // formed and cleared under mu
        for (auto& sl : s->slots)
            for (auto& q : sl.batch.reqs)
                if (q.tag == tag) return fail(HS_EBUSY, "request %llu is running", (unsigned long long)tag);
        return fail(HS_EINVAL, "no queued request with tag %llu", (unsigned long long)tag);
    }
    s->qdata.erase(r.seq);
    hs_completion c;
    std::memset(&c, 0, sizeof c);
    c.tag = r.tag;
    c.coll = r.coll;
    c.k = r.k;
    c.status = HS_ECANCEL;
    c.t_submit = r.t_submit;
    c.t_done = now_s();
    s->done.push_back(c);
    return HS_OK;
}

hs_status hs_poll(hs_server* s, hs_completion* out, int32_t max, int32_t* got) {
    if (!s || !got || (max > 0 && !out)) return fail(HS_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> g(s->mu);
    int n = 0;
    while (n < max && !s->done.empty()) {
        out[n++] = s->done.front();
        s->done.pop_front();
    }
    *got = n;
    return HS_OK;
}

hs_status hs_server_info(hs_server* s, hs_server_stats* out) {
    if (!s || !out) return fail(HS_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> g(s->mu);
    std::memset(out, 0, sizeof *out);
    out->in_system = s->sched->in_system();
    out->batches = s->launched_batches;
    out->queries = s->launched_queries;
    out->padded_queries = s->padded_queries;
    out->graphs = s->graphs_built;
    out->failed = s->error.empty() ? 0 : 1;
    return HS_OK;
}

hs_status hs_server_destroy(hs_server* s) {
    if (!s) return HS_OK;
    s->stop.store(true);
    s->cv.notify_all();
    if (s->th.joinable()) s->th.join();
    destroy_server(s);
    return HS_OK;
}

// ---- the scheduler alone (host only)

hs_status hs_sched_create(int32_t C, int32_t streams, int32_t max_slots, const int32_t* max_q, hs_sched** out) {
    if (!out || !max_q) return fail(HS_EINVAL, "NULL argument");
    *out = nullptr;
    if (C < 1 || streams < 1 || max_slots < 1) return fail(HS_EINVAL, "C, streams and max_slots must be >= 1");
    std::vector<std::array<int, kKBuckets>> mq(C);
    int mb = 0;
    for (int c = 0; c < C; ++c)
        for (int b = 0; b < kKBuckets; ++b) {
            const int v = max_q[c * kKBuckets + b];
            if (v < 0 || (v & (v - 1))) return fail(HS_EINVAL, "max_q[%d][%d]=%d is not 0 or a power of two", c, b, v);
            mq[c][b] = v;
            mb = std::max(mb, v);
        }
    hs_sched* h = new (std::nothrow) hs_sched();
    if (!h) return fail(HS_ENOMEM, "host allocation failed");
    h->max_batch = mb;
    h->s = new (std::nothrow) Scheduler(C, streams, max_slots, mq);
    if (!h->s) {
        delete h;
        return fail(HS_ENOMEM, "host allocation failed");
    }
    *out = h;
    return HS_OK;
}

hs_status hs_sched_submit(hs_sched* h, int32_t coll, int32_t k, uint64_t tag) {
    if (!h) return fail(HS_EINVAL, "NULL argument");
    SchedRequest r;
    r.tag = tag;
    r.coll = coll;
    r.k = k;
    const int rc = h->s->submit(r);
    if (rc == 1) return fail(HS_EBUSY, "all slots in use");
    if (rc != 0) return fail(HS_EINVAL, "request rejected (k=%d, collection %d)", k, coll);
    return HS_OK;
}

hs_status hs_sched_next(hs_sched* h, int32_t coll, int32_t stream, int32_t* q_pad, int32_t* k_batch, uint64_t* tags,
                        int32_t max_tags, int32_t* count) {
    if (!h || !q_pad || !k_batch || !count || (max_tags > 0 && !tags)) return fail(HS_EINVAL, "NULL argument");
    *count = 0;
    *q_pad = 0;
    *k_batch = 0;
    if (max_tags < h->max_batch) return fail(HS_EINVAL, "max_tags=%d below the largest batch %d", max_tags, h->max_batch);
    if (!h->s->next(coll, stream, &h->scratch)) return HS_OK;
    const int m = (int)h->scratch.reqs.size();
    for (int i = 0; i < m; ++i) tags[i] = h->scratch.reqs[i].tag;
    *count = m;
    *q_pad = h->scratch.q_pad;
    *k_batch = h->scratch.k_batch;
    return HS_OK;
}

hs_status hs_sched_cancel(hs_sched* h, uint64_t tag) {
    if (!h) return fail(HS_EINVAL, "NULL argument");
    if (h->s->cancel(tag, nullptr) != 0) return fail(HS_EINVAL, "no queued request with tag %llu", (unsigned long long)tag);
    return HS_OK;
}

hs_status hs_sched_complete(hs_sched* h, int32_t coll, int32_t stream) {
    if (!h) return fail(HS_EINVAL, "NULL argument");
    h->s->complete(coll, stream);
    return HS_OK;
}

hs_status hs_sched_in_system(hs_sched* h, int32_t* n) {
    if (!h || !n) return fail(HS_EINVAL, "NULL argument");
    *n = h->s->in_system();
    return HS_OK;
}

hs_status hs_sched_destroy(hs_sched* h) {
    if (!h) return HS_OK;
    delete h->s;
    delete h;
    return HS_OK;
}

}  // extern "C"
