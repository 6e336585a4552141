// qms_server.cpp -- the request loop: sort requests arrive one by one, are
// admitted against an HBM budget, grouped into batches and sorted with the
// batched QuickMergesort path on the server's own stream.
//
// Threads: callers submit and poll; one worker admits, batches, launches and
// completes.  Admission is FIFO: a request waits until the bytes of all
// admitted, unfinished requests plus its own fit in the budget; no request is
// dropped (a request larger than the whole budget is rejected at submit).
// Batching is greedy: whenever the worker is idle it takes every admitted
// request of the oldest request's dtype (up to max_batch) into one batch, so
// batches stay small under light load and grow with the queue.
// Ordering: a submit records an event on the caller's stream; the batch that
// holds the request waits for it on the server's stream, so keys still being
// written by work the caller enqueued before the submit are sorted only once
// that work has run.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "qms.h"
#include "qms_host.hpp"

using namespace qms;
using Clock = std::chrono::steady_clock;

namespace {

struct Request {
    uint64_t ticket;
    uint32_t *keys;
    uint64_t n;
    int dt;
    Clock::time_point t_submit, t_done;
    int status;  // QMS_PENDING, QMS_OK or an error code
    hipEvent_t ready;  // recorded on the caller's stream at submit
};

inline uint64_t request_bytes(uint64_t n, int dt) { return n * (dtype_wide(dt) ? 8 : 4); }

}  // namespace

struct qms_server {
    qms_server_config cfg;
    hipStream_t stream = nullptr;
    std::mutex mu;
    std::vector<hipEvent_t> free_events;  // recycled submit events
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> waiting;    // submitted, not yet admitted (FIFO)
    std::deque<Request *> admitted;   // admitted, not yet in a batch
    std::unordered_map<uint64_t, Request *> by_ticket;
    uint64_t next_ticket = 1;
    uint64_t admitted_bytes = 0;
    uint64_t in_flight = 0;           // requests admitted and not finished
    qms_server_stats stats;
    bool stop = false;
    std::thread worker;

    void admit_locked() {
        while (!waiting.empty()) {
            Request *r = waiting.front();
            const uint64_t b = request_bytes(r->n, r->dt);
            if (admitted_bytes + b > cfg.hbm_budget_bytes) break;
            waiting.pop_front();
            admitted_bytes += b;
            if (admitted_bytes > stats.peak_admitted_bytes) stats.peak_admitted_bytes = admitted_bytes;
            admitted.push_back(r);
        }
    }

    void run() {
        (void)hipSetDevice(cfg.device);
        std::vector<Request *> batch;
        std::vector<HostSeg> segs;
        // the worker holds its stream's workspace while it runs
        WorkspaceLease ws;
        for (;;) {
            {
                std::unique_lock<std::mutex> lock(mu);
                cv_work.wait(lock, [&] { return stop || !admitted.empty(); });
                if (admitted.empty() && stop) return;
                const int dt = admitted.front()->dt;
                batch.clear();
                const uint32_t cap = cfg.max_batch ? cfg.max_batch : 4096;
                for (auto it = admitted.begin(); it != admitted.end() && batch.size() < cap;) {
                    if ((*it)->dt == dt) {
                        batch.push_back(*it);
                        it = admitted.erase(it);
                    } else {
                        ++it;
                    }
                }
            }
            segs.clear();
            int rc = ws.get() ? QMS_OK : get_workspace(cfg.device, stream, &ws);
            for (Request *r : batch) {
                segs.push_back(HostSeg{r->keys, nullptr, r->n});
                if (rc == QMS_OK) {
                    hipError_t e = hipStreamWaitEvent(stream, r->ready, 0);
                    if (e != hipSuccess) rc = hip_error(e, "server: waiting for the submit event");
                }
            }
            if (rc == QMS_OK)
                rc = sort_segments(batch.front()->dt, false, segs.data(), segs.size(), *ws, stream,
                                   false);
            if (rc == QMS_OK) {
                hipError_t e = hipStreamSynchronize(stream);
                if (e != hipSuccess) rc = hip_error(e, "server batch");
            } else {
                // the events may still be waited on by enqueued work
                (void)hipStreamSynchronize(stream);
            }
            const Clock::time_point now = Clock::now();
            {
                std::lock_guard<std::mutex> lock(mu);
                for (Request *r : batch) {
                    r->t_done = now;
                    r->status = rc == QMS_OK ? QMS_OK : rc;
                    free_events.push_back(r->ready);
                    r->ready = nullptr;
                    admitted_bytes -= request_bytes(r->n, r->dt);
                    --in_flight;
                    stats.completed += 1;
                    stats.completed_keys += r->n;
                }
                stats.batches += 1;
                admit_locked();
            }
            cv_done.notify_all();
        }
    }
};

extern "C" {

int qms_server_create(const qms_server_config *cfg, qms_server **out) {
    try {
        if (!cfg || !out) return set_error(QMS_ERR_INVALID, "NULL config or handle");
        *out = nullptr;
        if (cfg->hbm_budget_bytes == 0) return set_error(QMS_ERR_INVALID, "zero HBM budget");
        int ndev = 0;
        hipError_t e = hipGetDeviceCount(&ndev);
        if (e != hipSuccess) return hip_error(e, "hipGetDeviceCount");
        if (cfg->device < 0 || cfg->device >= ndev) return set_error(QMS_ERR_INVALID, "bad device");
        qms_server *s = new qms_server();
        s->cfg = *cfg;
        std::memset(&s->stats, 0, sizeof(s->stats));
        DeviceScope scope(cfg->device);
        e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            delete s;
            return hip_error(e, "server stream");
        }
        {
            // allocate the stream's workspace now, so that a failure is
            // reported here; the worker takes it when it starts
            WorkspaceLease lease;
            int rc = get_workspace(cfg->device, s->stream, &lease);
            if (rc != QMS_OK) {
                (void)hipStreamDestroy(s->stream);
                delete s;
                return rc;
            }
        }
        s->worker = std::thread([s] { s->run(); });
        *out = s;
        return QMS_OK;
    } catch (...) {
        return set_error(QMS_ERR_NOMEM, "host exception in qms_server_create");
    }
}

int qms_server_submit(qms_server *s, void *d_keys, uint64_t n, int dt, hipStream_t stream,
                      uint64_t *ticket_out) {
    try {
        if (!s || !ticket_out) return set_error(QMS_ERR_INVALID, "NULL server or ticket");
        if (!dtype_known(dt)) return set_error(QMS_ERR_UNSUPPORTED, "unknown dtype");
        if (n >= (1ull << 32)) return set_error(QMS_ERR_UNSUPPORTED, "n must be below 2^32");
        if (request_bytes(n, dt) > s->cfg.hbm_budget_bytes)
            return set_error(QMS_ERR_BUDGET, "request larger than the HBM budget");
        hipEvent_t ev = nullptr;
        if (n > 1) {
            if (!d_keys) return set_error(QMS_ERR_INVALID, "NULL keys with n > 1");
            int dev = -1;
            int rc = check_device_ptr(d_keys, "keys", &dev, dtype_wide(dt) ? 8 : 4);
            if (rc != QMS_OK) return rc;
            if (dev != s->cfg.device)
                return set_error(QMS_ERR_INVALID, "keys not on the server's device");
            {
                std::lock_guard<std::mutex> lock(s->mu);
                if (!s->free_events.empty()) {
                    ev = s->free_events.back();
                    s->free_events.pop_back();
                }
            }
            DeviceScope scope(s->cfg.device);
            hipError_t e = hipSuccess;
            if (!ev) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
            if (e == hipSuccess) e = hipEventRecord(ev, stream);
            if (e != hipSuccess) {
                if (ev) {
                    std::lock_guard<std::mutex> lock(s->mu);
                    s->free_events.push_back(ev);
                }
                (void)hipGetLastError();
                return hip_error(e, "server: recording the submit event on the caller's stream");
            }
        }
        Request *r = new Request{0, (uint32_t *)d_keys, n, dt, Clock::now(), {}, QMS_PENDING, ev};
        {
            std::lock_guard<std::mutex> lock(s->mu);
            if (s->stop) {
                if (ev) s->free_events.push_back(ev);
                delete r;
                return set_error(QMS_ERR_INVALID, "server is shutting down");
            }
            r->ticket = s->next_ticket++;
            s->by_ticket[r->ticket] = r;
            if (n <= 1) {  // nothing to sort
                r->t_done = r->t_submit;
                r->status = QMS_OK;
                s->stats.completed += 1;
                s->stats.completed_keys += n;
            } else {
                ++s->in_flight;
                const bool fits = s->waiting.empty() &&
                                  s->admitted_bytes + request_bytes(n, dt) <= s->cfg.hbm_budget_bytes;
                if (!fits) s->stats.waited_for_budget += 1;
                s->waiting.push_back(r);
                s->admit_locked();
            }
            *ticket_out = r->ticket;
        }
        s->cv_work.notify_one();
        return QMS_OK;
    } catch (...) {
        return set_error(QMS_ERR_NOMEM, "host exception in qms_server_submit");
    }
}

int qms_server_poll(qms_server *s, uint64_t ticket, double *latency_s_out) {
    try {
        if (!s) return set_error(QMS_ERR_INVALID, "NULL server");
        std::lock_guard<std::mutex> lock(s->mu);
        auto it = s->by_ticket.find(ticket);
        if (it == s->by_ticket.end()) return set_error(QMS_ERR_INVALID, "unknown or retired ticket");
        Request *r = it->second;
        if (r->status == QMS_PENDING) return QMS_PENDING;
        const int st = r->status;
        if (latency_s_out)
            *latency_s_out = std::chrono::duration<double>(r->t_done - r->t_submit).count();
        s->by_ticket.erase(it);
        delete r;
        if (st != QMS_OK) return set_error(st, "the batch holding this request failed");
        return QMS_OK;
    } catch (...) {
        return set_error(QMS_ERR_NOMEM, "host exception in qms_server_poll");
    }
}

int qms_server_get_stats(qms_server *s, qms_server_stats *out) {
    if (!s || !out) return set_error(QMS_ERR_INVALID, "NULL server or stats");
    std::lock_guard<std::mutex> lock(s->mu);
    *out = s->stats;
    return QMS_OK;
}

int qms_server_destroy(qms_server *s) {
    try {
        if (!s) return QMS_OK;
        {
            std::unique_lock<std::mutex> lock(s->mu);
            // drain: wait until every admitted or waiting request has finished
            s->cv_done.wait(lock, [&] { return s->in_flight == 0; });
            s->stop = true;
        }
        s->cv_work.notify_all();
        if (s->worker.joinable()) s->worker.join();
        (void)hipStreamSynchronize(s->stream);
        for (auto &kv : s->by_ticket) delete kv.second;
        for (hipEvent_t ev : s->free_events) (void)hipEventDestroy(ev);
        // the workspace is keyed by this stream; release it with the stream
        (void)release_workspace(s->cfg.device, s->stream);
        (void)hipStreamDestroy(s->stream);
        delete s;
        return QMS_OK;
    } catch (...) {
        return set_error(QMS_ERR_NOMEM, "host exception in qms_server_destroy");
    }
}

}  // extern "C"
