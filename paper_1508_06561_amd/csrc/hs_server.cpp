// hs_server.cpp -- serving loop of the C ABI (include/hs.h): queries are
// submitted one at a time from any thread; each of a few worker threads owns
// a batch handle and a stream and runs continuous batching -- whenever it is
// free it takes the waiting queries, oldest first, that fit its batch's
// footprint (device memory: count and total letters within the handle's
// buffers; LDS: queries that keep four profile copies are not batched with
// ones that need the one-copy layout), searches them as one batch on its
// stream and publishes each query's results.  With
// two workers, queries that arrive while one batch is on the device start at
// once beside it.  Every result equals a separate hs_search of that query:
// batching never changes results.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "hs.h"

namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

struct Pending {
    uint64_t tag;
    int lds_class;          // profile copies its batch can keep (4 or 1)
    std::string query;
    hs_params params;
    bool own_matrix;
    int8_t matrix[HS_NSYM * HS_NSYM];
    Clock::time_point t_submit;
};

struct Done {
    int rc;
    std::string err;
    std::vector<hs_hit> hits;
    std::vector<hs_aln> alns;
    std::vector<uint32_t> ops;
    hs_server_timing timing;
};

}  // namespace

// The library's per-thread error message (hs_last_error), and the LDS class
// of a query in a batch, both in hs_lib.hip.
namespace hs_internal {
void set_error(const std::string& msg);
int batch_lds_class(int32_t qlen);
}

namespace {

int sfail(int code, const std::string& msg) {
    hs_internal::set_error(msg);
    return code;
}

}  // namespace

struct hs_server;

namespace {

// One worker: a batch handle, a stream and the thread that drives them.
struct Worker {
    hs_batch* batch = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};   // around each batch's kernels
    std::thread thread;
};

}  // namespace

struct hs_server {
    const hs_db* db = nullptr;
    std::vector<Worker> workers;
    int device = 0;
    int32_t max_batch = 0, max_qlen = 0, k = 0, n_aln = 0;
    int64_t max_residues = 0;
    std::thread worker;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool stop = false;
    std::deque<Pending> queue;
    std::unordered_set<uint64_t> inflight;   // tags taken by the worker, results not yet published
    std::unordered_map<uint64_t, Done> done;
    std::deque<uint64_t> done_order;
    int64_t n_batches = 0, n_served = 0;
    Clock::time_point t0 = Clock::now();

    void run(Worker& wk);
};

void hs_server::run(Worker& wk) {
    (void)hipSetDevice(device);
    hs_batch* batch = wk.batch;
    hipStream_t stream = wk.stream;
    std::vector<Pending> cur;
    std::vector<char> residues;
    std::vector<int64_t> offsets;
    std::vector<hs_params> params;
    std::vector<hs_hit> hits;
    std::vector<int32_t> n_hits, n_alns;
    std::vector<hs_aln> alns;
    std::vector<uint32_t> ops;
    for (;;) {
        cur.clear();
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_work.wait(lk, [&] { return stop || !queue.empty(); });
            if (stop) return;
            // admission, first come first served, while the batch's footprint
            // allows: device memory (queries and letters within the batch
            // handle's buffers) and LDS -- a query whose profile needs the
            // one-copy layout starts a batch of its own class rather than
            // taking a batch of shorter queries down to one copy with it
            int64_t res = 0;
            while (!queue.empty() && (int32_t)cur.size() < max_batch &&
                   res + (int64_t)queue.front().query.size() <= max_residues &&
                   (cur.empty() || queue.front().lds_class == cur[0].lds_class)) {
                res += (int64_t)queue.front().query.size();
                inflight.insert(queue.front().tag);
                cur.push_back(std::move(queue.front()));
                queue.pop_front();
            }
        }
        const Clock::time_point t_start = Clock::now();
        const int32_t nq = (int32_t)cur.size();
        residues.clear();
        offsets.assign(1, 0);
        params.resize((size_t)nq);
        int64_t ops_cap = 0;
        for (int32_t i = 0; i < nq; ++i) {
            Pending& p = cur[(size_t)i];
            residues.insert(residues.end(), p.query.begin(), p.query.end());
            offsets.push_back((int64_t)residues.size());
            params[(size_t)i] = p.params;
            params[(size_t)i].matrix = p.own_matrix ? p.matrix : nullptr;
            ops_cap += (int64_t)n_aln * (2 * (int64_t)p.query.size() + 2);
        }
        hits.resize((size_t)nq * k);
        n_hits.resize((size_t)nq);
        n_alns.assign((size_t)nq, 0);
        alns.resize((size_t)nq * (size_t)(n_aln > 0 ? n_aln : 1));
        ops.resize((size_t)(ops_cap > 0 ? ops_cap : 1));
        int64_t used = 0;
        int rc = hs_batch_set(batch, nq, residues.data(), offsets.data(), params.data(), nq, stream);
        const Clock::time_point t_set = Clock::now();
        if (!rc) {
            (void)hipEventRecord(wk.ev[0], stream);
            rc = hs_batch_run(batch, stream);
            (void)hipEventRecord(wk.ev[1], stream);
        }
        const Clock::time_point t_run = Clock::now();
        if (!rc)
            rc = hs_batch_results(batch, stream, hits.data(), n_hits.data(), alns.data(),
                                  n_alns.data(), ops.data(), ops_cap, &used);
        const std::string err = rc ? hs_last_error() : "";
        const Clock::time_point t_done = Clock::now();
        float gpu_ms = 0.f;
        if (!rc && hipEventElapsedTime(&gpu_ms, wk.ev[0], wk.ev[1]) != hipSuccess) gpu_ms = -1.f;
        {
            std::lock_guard<std::mutex> lk(mu);
            for (int32_t i = 0; i < nq; ++i) {
                Done d;
                d.rc = rc;
                d.err = err;
                d.timing.queue_ms = ms_between(cur[(size_t)i].t_submit, t_start);
                d.timing.total_ms = ms_between(cur[(size_t)i].t_submit, t_done);
                d.timing.batch_ms = ms_between(t_start, t_done);
                d.timing.set_ms = ms_between(t_start, t_set);
                d.timing.run_ms = ms_between(t_set, t_run);
                d.timing.results_ms = ms_between(t_run, t_done);
                d.timing.gpu_ms = gpu_ms;
                d.timing.batch_size = nq;
                d.timing.submit_ms = ms_between(t0, cur[(size_t)i].t_submit);
                if (!rc) {
                    const int32_t nh = n_hits[(size_t)i];
                    d.hits.assign(hits.begin() + (size_t)i * k, hits.begin() + (size_t)i * k + nh);
                    if (n_aln > 0) {
                        const int32_t na = n_alns[(size_t)i];
                        const hs_aln* a = alns.data() + (size_t)i * n_aln;
                        const int64_t o0 = na ? a[0].ops_off : 0;
                        const int64_t o1 = na ? a[na - 1].ops_off + a[na - 1].n_ops : 0;
                        d.alns.assign(a, a + na);
                        for (hs_aln& x : d.alns) x.ops_off -= o0;
                        d.ops.assign(ops.begin() + o0, ops.begin() + o1);
                    }
                }
                done[cur[(size_t)i].tag] = std::move(d);
                done_order.push_back(cur[(size_t)i].tag);
                inflight.erase(cur[(size_t)i].tag);
            }
            ++n_batches;
            n_served += nq;
        }
        cv_done.notify_all();
    }
}

extern "C" {

int hs_server_create_workers(const hs_db* db, int32_t max_batch, int32_t max_qlen,
                             int64_t max_residues, int32_t k, int32_t n_aln, int32_t n_workers,
                             hs_server** out) {
    if (!out) return sfail(HS_EINVAL, "out is NULL");
    if (n_workers < 1 || n_workers > HS_MAX_SERVER_WORKERS)
        return sfail(HS_EINVAL, "n_workers must lie in [1, HS_MAX_SERVER_WORKERS]");
    // a query longer than max_residues could never be admitted: it would stay
    // at the head of the queue and block every query behind it
    if (max_qlen > 0 && max_residues < max_qlen)
        return sfail(HS_EINVAL, "max_residues must be at least max_qlen");
    hs_server* s = new hs_server();
    s->workers.resize((size_t)n_workers);
    int rc = HS_OK;
    for (Worker& wk : s->workers) {   // the first batch handle validates the arguments
        if (rc) break;
        rc = hs_batch_create(db, max_batch, max_qlen, max_residues, k, n_aln, &wk.batch);
        if (!rc && hipStreamCreateWithFlags(&wk.stream, hipStreamNonBlocking) != hipSuccess)
            rc = sfail(HS_EDEVICE, "stream creation failed");
        if (!rc && (hipEventCreate(&wk.ev[0]) != hipSuccess || hipEventCreate(&wk.ev[1]) != hipSuccess))
            rc = sfail(HS_EDEVICE, "event creation failed");
    }
    if (!rc && hipGetDevice(&s->device) != hipSuccess) rc = sfail(HS_EDEVICE, "no current device");
    if (rc) {
        for (Worker& wk : s->workers) {
            for (hipEvent_t e : wk.ev)
                if (e) (void)hipEventDestroy(e);
            if (wk.stream) (void)hipStreamDestroy(wk.stream);
            if (wk.batch) hs_batch_free(wk.batch);
        }
        delete s;
        return rc;
    }
    s->db = db;
    s->max_batch = max_batch;
    s->max_qlen = max_qlen;
    s->max_residues = max_residues;
    s->k = k;
    s->n_aln = n_aln;
    for (Worker& wk : s->workers) {
        Worker* w = &wk;
        wk.thread = std::thread([s, w] { s->run(*w); });
    }
    *out = s;
    return HS_OK;
}

int hs_server_create(const hs_db* db, int32_t max_batch, int32_t max_qlen, int64_t max_residues,
                     int32_t k, int32_t n_aln, hs_server** out) {
    return hs_server_create_workers(db, max_batch, max_qlen, max_residues, k, n_aln, 2, out);
}

int hs_server_free(hs_server* s) {
    if (!s) return HS_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    for (Worker& wk : s->workers)
        if (wk.thread.joinable()) wk.thread.join();
    for (Worker& wk : s->workers) {
        (void)hipStreamSynchronize(wk.stream);
        for (hipEvent_t e : wk.ev)
            if (e) (void)hipEventDestroy(e);
        (void)hipStreamDestroy(wk.stream);
        hs_batch_free(wk.batch);
    }
    delete s;
    return HS_OK;
}

int hs_server_submit(hs_server* s, const char* query, int32_t qlen, const hs_params* params,
                     uint64_t tag) {
    if (!s) return sfail(HS_EINVAL, "server is NULL");
    if (!query || !params) return sfail(HS_EINVAL, "NULL query or params");
    if (qlen < 1 || qlen > s->max_qlen || qlen > s->max_residues)
        return sfail(HS_EINVAL, "qlen must lie in [1, max_qlen] and fit max_residues");
    if (int rc = hs_params_check(params)) return rc;
    std::vector<uint8_t> codes((size_t)qlen);
    if (hs_encode(query, qlen, codes.data())) return HS_EINVAL;
    Pending p;
    p.tag = tag;
    p.lds_class = hs_internal::batch_lds_class(qlen);
    p.query.assign(query, (size_t)qlen);
    p.params = *params;
    p.own_matrix = params->matrix != nullptr;
    if (p.own_matrix) std::memcpy(p.matrix, params->matrix, sizeof(p.matrix));
    p.params.matrix = nullptr;
    p.t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->done.count(tag)) return sfail(HS_EINVAL, "tag already holds an unclaimed result");
        if (s->inflight.count(tag)) return sfail(HS_EINVAL, "tag already being searched");
        for (const Pending& q : s->queue)
            if (q.tag == tag) return sfail(HS_EINVAL, "tag already pending");
        s->queue.push_back(std::move(p));
    }
    s->cv_work.notify_one();
    return HS_OK;
}

int hs_server_poll(hs_server* s, uint64_t* tags, int32_t max_tags, int32_t* n_tags,
                   int32_t timeout_ms) {
    if (!s || !tags || !n_tags || max_tags < 1) return sfail(HS_EINVAL, "bad arguments to hs_server_poll");
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->done_order.empty() && timeout_ms > 0)
        s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms),
                            [&] { return !s->done_order.empty(); });
    int32_t n = 0;
    while (n < max_tags && !s->done_order.empty()) {
        tags[n++] = s->done_order.front();
        s->done_order.pop_front();
    }
    *n_tags = n;
    return HS_OK;
}

int hs_server_result(hs_server* s, uint64_t tag, hs_hit* hits, int32_t* n_hits, hs_aln* alns,
                     int32_t* n_alns, uint32_t* ops, int64_t ops_cap, int64_t* ops_used,
                     hs_server_timing* timing) {
    if (!s || !hits || !n_hits) return sfail(HS_EINVAL, "bad arguments to hs_server_result");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->done.find(tag);
    if (it == s->done.end()) return sfail(HS_EINVAL, "no finished query with this tag");
    Done& d = it->second;
    if (d.rc) {
        const int rc = d.rc;
        hs_internal::set_error(d.err);
        s->done.erase(it);
        return rc;
    }
    if (s->n_aln > 0) {
        if (!alns || !n_alns || !ops_used) return sfail(HS_EINVAL, "NULL alignment outputs");
        *ops_used = (int64_t)d.ops.size();
        if ((int64_t)d.ops.size() > ops_cap) return sfail(HS_ENOSPC, "ops buffer too small");
        std::memcpy(alns, d.alns.data(), sizeof(hs_aln) * d.alns.size());
        *n_alns = (int32_t)d.alns.size();
        if (!d.ops.empty()) std::memcpy(ops, d.ops.data(), sizeof(uint32_t) * d.ops.size());
    }
    std::memcpy(hits, d.hits.data(), sizeof(hs_hit) * d.hits.size());
    *n_hits = (int32_t)d.hits.size();
    if (timing) *timing = d.timing;
    s->done.erase(it);
    return HS_OK;
}

int hs_server_stats(hs_server* s, int64_t* pending, int64_t* batches, int64_t* served) {
    if (!s) return sfail(HS_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    if (pending) *pending = (int64_t)s->queue.size();
    if (batches) *batches = s->n_batches;
    if (served) *served = s->n_served;
    return HS_OK;
}

}  // extern "C"
