// Request loop: resident series, admission by HBM footprint, continuous
// batching over several HIP streams, latency statistics.
//
// A worker thread owns the GPU side.  Each turn it (1) retires batches whose
// completion event has fired, (2) while a stream slot is free and requests
// are pending, forms one batch from the pending queue in arrival order,
// bounded by the remaining HBM budget, and launches it, and (3) sleeps
// briefly.  Requests that arrive while earlier batches are on the GPU are
// admitted into the next batch as soon as a slot and memory free up; that
// batch runs on another stream, so its blocks start as the earlier kernel's
// persistent blocks drain.  A batch is sized before anything is allocated;
// the queue front waits for memory (rather than failing) while other batches
// hold it, and admission is retried only once a batch has retired.  Each
// estimate's result does not depend on the batch it ran in (exact counts,
// fixed-order sums).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <thread>
#include <unordered_map>

#include "runtime.h"

namespace mte {

namespace {

using Clock = std::chrono::steady_clock;

struct Series {
    std::unique_ptr<DevBuf> buf;
    int P = 0;
    int64_t T = 0;
    int pending = 0;
    int32_t std_sid = -1;   // its per-node z-scored copy, made on first use
    bool cancelled = false; // mte_serve_cancel: new requests are refused
};

struct Req {
    uint64_t ticket = 0;
    mte_request r{};
    std::vector<int32_t> nodes, lags;
    Clock::time_point t_submit, t_done;
    // the admission that launched it: its start and the end of its enqueue
    Clock::time_point t_admit, t_launch;
    int batch_reqs = 0;            // requests in that batch
    int state = 0;                 // 0 queued, 1 on the GPU, 2 done
    bool waited = false;           // held at the queue front for memory
    int status = MTE_OK;
    std::string error;
    std::vector<double> result;    // 1 + S
};

struct Slot {
    bool busy = false;
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    std::unique_ptr<Batch> batch;
    std::vector<std::shared_ptr<Req>> reqs;
    DevBuf out;
    HostBuf hout;
    size_t bytes = 0;
};

constexpr int kSlots = 3;
constexpr size_t kMaxBatchRequests = 512;
// Device memory of one batch at most (MTE_BATCH_BYTES_MAX overrides), above
// which a batch of several requests is halved: requests with lists of their
// own (a served mix of unrelated conditioning sets) made batches of 85-128
// requests and 70-120 GB in a burst of 768, whose blocks the allocator's
// cache could not supply, and the re-allocation of tens of GB stretched such
// bursts from 0.22 s to 2.4-4.9 s; batches of about ten requests already
// keep the device busy.
constexpr size_t kMaxBatchBytes = size_t(16) << 30;

class Server {
public:
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::unordered_map<int32_t, Series> series;
    int32_t next_sid = 0;
    std::deque<std::shared_ptr<Req>> queue;
    std::unordered_map<uint64_t, std::shared_ptr<Req>> reqs;
    uint64_t next_ticket = 1;
    Slot slots[kSlots];
    int active_slots = kSlots;     // MTE_SERVE_SLOTS (1..3) limits the batches in flight
    std::thread worker;
    bool running = false, stop = false;
    size_t bytes_in_flight = 0;
    bool mem_blocked = false;      // the queue front waits for a batch to retire
    // statistics
    int64_t submitted = 0, completed = 0, rejected = 0, batches = 0, estimates = 0, batch_reqs = 0;
    int64_t waited = 0;            // requests admitted after waiting for memory
    // latency of each completed request and its phases: queued (submit to the
    // start of the admission that launched it), host (that admission: sizing,
    // preparing and enqueueing the batch) and device (launch to the retirement
    // that found the batch done)
    struct Lat {
        double total, queue, host, device;
        int64_t n;
        int batch;
    };
    std::vector<Lat> latencies;
    size_t peak_bytes = 0;

    int start_locked() {
        if (running) return MTE_OK;
        int rc = ensure_init();
        if (rc) return rc;
        for (auto &s : slots) {
            if (!s.stream) MTE_HIP(hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking));
            if (!s.done) MTE_HIP(hipEventCreateWithFlags(&s.done, hipEventDisableTiming));
        }
        active_slots = kSlots;
        if (const char *v = std::getenv("MTE_SERVE_SLOTS")) {
            const int n = std::atoi(v);
            if (n >= 1 && n <= kSlots) active_slots = n;
        }
        stop = false;
        running = true;
        const int dev = ctx().device;
        worker = std::thread([this, dev] { loop(dev); });
        return MTE_OK;
    }

    void finish_req(const std::shared_ptr<Req> &q, int status, const char *msg) {
        q->status = status;
        if (msg) q->error = msg;
        q->state = 2;
        q->t_done = Clock::now();
        auto it = series.find(q->r.sid);
        if (it != series.end()) it->second.pending--;
        if (status == MTE_OK) {
            completed++;
            estimates += (int64_t)q->result.size();
            auto sec = [](Clock::duration d) { return std::chrono::duration<double>(d).count(); };
            latencies.push_back(Lat{sec(q->t_done - q->t_submit), sec(q->t_admit - q->t_submit),
                                    sec(q->t_launch - q->t_admit), sec(q->t_done - q->t_launch), q->r.N,
                                    q->batch_reqs});
        } else {
            rejected++;
        }
    }

    // Retire finished slots (called with mu held).
    void retire() {
        for (auto &s : slots) {
            if (!s.busy) continue;
            hipError_t e = hipEventQuery(s.done);
            if (e == hipErrorNotReady) continue;
            int status = e == hipSuccess ? MTE_OK : MTE_EDEVICE;
            if (status == MTE_OK && s.batch->check_error(s.stream) != MTE_OK) status = MTE_EDEVICE;
            const double *h = static_cast<const double *>(s.hout.p);
            size_t pos = 0;
            for (auto &q : s.reqs) {
                const size_t E = (size_t)q->r.S + 1;
                if (status == MTE_OK) q->result.assign(h + pos, h + pos + E);
                pos += E;
                finish_req(q, status, status ? "kernel failure" : nullptr);
            }
            s.reqs.clear();
            s.batch.reset();
            bytes_in_flight -= s.bytes;
            s.bytes = 0;
            s.busy = false;
            mem_blocked = false;
            cv_done.notify_all();
        }
    }

    JobSpec spec_for(const Req &q, double *out) {
        const Series &se = series.at(q.r.sid);
        JobSpec sp;
        const int d = q.r.dx + q.r.dy + q.r.dz;
        for (int c = 0; c < d; ++c)
            sp.cols[c] = se.buf->as<float>() + (size_t)q.nodes[c] * se.T + (q.r.t0 - q.lags[c]);
        sp.n = (int)q.r.N;
        sp.dx = q.r.dx;
        sp.dy = q.r.dy;
        sp.dz = q.r.dz;
        sp.k = q.r.k;
        sp.theiler = q.r.theiler;
        sp.keys.resize((size_t)q.r.S + 1);
        sp.keys[0] = EstKey{0, 1, 0};
        for (int s = 0; s < q.r.S; ++s)
            sp.keys[(size_t)s + 1] = EstKey{surrogate_key(q.r.seed, q.r.cand, (uint32_t)s), 0, 0};
        sp.out = out;
        return sp;
    }

    // The queue front waits for memory: admission is retried after the
    // next retirement.
    void block_front() {
        mem_blocked = true;
        if (!queue.empty()) queue.front()->waited = true;
    }

    // Drop the first n queued requests with a status (mu held).
    void fail_front(size_t n, int status, const char *msg) {
        for (size_t i = 0; i < n; ++i) finish_req(queue[i], status, msg);
        queue.erase(queue.begin(), queue.begin() + (long)n);
        cv_done.notify_all();
    }

    // The requests that would share the front request's neighbour-list set
    // (same series, rows, Y and Z columns and window) are moved up behind it,
    // keeping their order, so that a batch holds few list sets (mu held).
    // The front request itself never moves.
    void group_front() {
        if (queue.size() < 2) return;
        const Req &f = *queue.front();
        auto same_set = [&](const Req &q) {
            if (q.r.sid != f.r.sid || q.r.N != f.r.N || q.r.t0 != f.r.t0 || q.r.dy != f.r.dy || q.r.dz != f.r.dz ||
                q.r.theiler != f.r.theiler)
                return false;
            for (int c = 0; c < q.r.dy + q.r.dz; ++c)
                if (q.nodes[q.r.dx + c] != f.nodes[f.r.dx + c] || q.lags[q.r.dx + c] != f.lags[f.r.dx + c])
                    return false;
            return true;
        };
        const size_t lim = std::min(queue.size(), 4 * kMaxBatchRequests);
        std::stable_partition(queue.begin() + 1, queue.begin() + (long)lim,
                              [&](const std::shared_ptr<Req> &q) { return same_set(*q); });
    }

    // Form and launch one batch on slot s from the queue front (mu held).
    // The batch is sized first (Batch::prepare in measuring mode); it is
    // halved while it does not fit beside the batches in flight, a single
    // request that exceeds the whole budget is rejected, and one that only
    // needs memory held by others waits.  An allocation that fails while other
    // batches hold memory makes the front wait as well.
    void admit(Slot &s) {
        if (mem_blocked) return;
        const Clock::time_point t_admit = Clock::now();
        const size_t budget = ctx().budget;
        static const size_t batch_cap = [] {
            const char *v = std::getenv("MTE_BATCH_BYTES_MAX");
            const long long b = v && *v ? std::atoll(v) : 0;
            return b > 0 ? (size_t)b : kMaxBatchBytes;
        }();
        group_front();
        size_t take = std::min(queue.size(), kMaxBatchRequests);
        while (take > 0) {
            size_t n_out = 0;
            for (size_t i = 0; i < take; ++i) n_out += (size_t)queue[i]->r.S + 1;
            int rc = s.out.ensure(sizeof(double) * n_out);
            if (rc == MTE_OK) rc = s.hout.ensure(sizeof(double) * n_out);
            if (rc != MTE_OK) {
                if (bytes_in_flight > 0) return block_front();
                return fail_front(take, rc, "output buffer allocation failed");
            }
            std::vector<JobSpec> specs;
            size_t pos = 0;
            for (size_t i = 0; i < take; ++i) {
                specs.push_back(spec_for(*queue[i], s.out.as<double>() + pos));
                pos += (size_t)queue[i]->r.S + 1;
            }
            TileChoice tc;
            size_t need = 0;
            auto b = std::make_unique<Batch>();
            rc = choose_tiles(specs, s.stream, kTuneNone, &tc);
            if (rc == MTE_OK) rc = b->prepare(specs, tc, s.stream, &need);
            if (rc != MTE_OK) return fail_front(take, rc, "batch preparation failed");
            const size_t bytes = need + sizeof(double) * n_out;
            if (take > 1 && bytes > batch_cap) {
                take /= 2;
                continue;
            }
            if (bytes_in_flight + bytes > budget) {
                if (take > 1) {
                    take /= 2;
                    continue;
                }
                if (bytes > budget) return fail_front(1, MTE_ENOMEM, "request exceeds the HBM budget");
                return block_front();
            }
            rc = b->prepare(specs, tc, s.stream);
            if (rc == MTE_ENOMEM) {
                if (bytes_in_flight > 0) return block_front();
                if (take > 1) {
                    take /= 2;
                    continue;
                }
            }
            if (rc != MTE_OK) return fail_front(take, rc, "batch preparation failed");
            rc = b->enqueue(s.stream, false);
            if (rc == MTE_OK && hipMemcpyAsync(s.hout.p, s.out.p, sizeof(double) * n_out,
                                               hipMemcpyDeviceToHost, s.stream) != hipSuccess)
                rc = MTE_EDEVICE;
            if (rc == MTE_OK && hipEventRecord(s.done, s.stream) != hipSuccess) rc = MTE_EDEVICE;
            if (rc != MTE_OK) {
                (void)hipStreamSynchronize(s.stream);
                return fail_front(take, MTE_EDEVICE, "launch failed");
            }
            s.reqs.assign(queue.begin(), queue.begin() + (long)take);
            queue.erase(queue.begin(), queue.begin() + (long)take);
            const Clock::time_point t_launch = Clock::now();
            for (auto &q : s.reqs) {
                q->state = 1;
                q->t_admit = t_admit;
                q->t_launch = t_launch;
                q->batch_reqs = (int)take;
                if (q->waited) waited++;
            }
            s.batch = std::move(b);
            s.bytes = bytes;
            s.busy = true;
            bytes_in_flight += bytes;
            peak_bytes = std::max(peak_bytes, bytes_in_flight);
            batches++;
            batch_reqs += (int64_t)s.reqs.size();
            return;
        }
    }

    // Refuse new requests on the series and finish its queued ones with
    // MTE_ECANCELED (mu held); batches on the GPU complete.
    void cancel(int32_t sid) {
        for (auto it = queue.begin(); it != queue.end();) {
            if ((*it)->r.sid == sid) {
                finish_req(*it, MTE_ECANCELED, "cancelled");
                it = queue.erase(it);
            } else {
                ++it;
            }
        }
        if (!queue.empty() && mem_blocked) queue.front()->waited = true;
        cv_done.notify_all();
    }

    void loop(int dev) {
        (void)hipSetDevice(dev);
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            retire();
            bool any_busy = false;
            for (int i = 0; i < active_slots; ++i) {
                Slot &s = slots[i];
                if (!s.busy && !queue.empty()) admit(s);
                any_busy |= s.busy;
            }
            if (stop && !any_busy && queue.empty()) break;
            if (any_busy) {
                lk.unlock();
                std::this_thread::sleep_for(std::chrono::microseconds(20));
                lk.lock();
            } else {
                cv_work.wait_for(lk, std::chrono::milliseconds(5));
            }
        }
    }

    int shutdown() {
        {
            std::lock_guard<std::mutex> lk(mu);
            if (!running) return MTE_OK;
            stop = true;
        }
        cv_work.notify_all();
        worker.join();
        std::lock_guard<std::mutex> lk(mu);
        running = false;
        for (auto &s : slots) {
            if (s.stream) (void)hipStreamDestroy(s.stream);
            if (s.done) (void)hipEventDestroy(s.done);
            s.stream = nullptr;
            s.done = nullptr;
            s.out.reset();
            s.hout.reset();
        }
        series.clear();
        reqs.clear();
        queue.clear();
        return MTE_OK;
    }
};

// Never destroyed: the worker thread may still exist at process exit, and a
// joinable std::thread must not be destroyed (mte_shutdown joins it).
Server &server() {
    static Server *s = new Server;
    return *s;
}

}  // namespace

int serve_shutdown() { return server().shutdown(); }

int select_sources_served(int32_t sid, int P, int64_t T, int target, const int32_t *candidates,
                          int n_candidates, int max_lag_sources, double alpha, const mte_opts *opts,
                          mte_result *out);

int series_shape(int32_t sid, int *P, int64_t *T) {
    Server &sv = server();
    std::lock_guard<std::mutex> lk(sv.mu);
    auto it = sv.series.find(sid);
    if (it == sv.series.end()) return fail(MTE_EINVAL, "unknown series %d", sid);
    *P = it->second.P;
    *T = it->second.T;
    return MTE_OK;
}

// Device copy of a registered series for a caller that reads it directly
// (the Gaussian greedy search); the series counts as in use until unpinned.
int series_pin(int32_t sid, const float **dev, int *P, int64_t *T) {
    Server &sv = server();
    std::lock_guard<std::mutex> lk(sv.mu);
    auto it = sv.series.find(sid);
    if (it == sv.series.end()) return fail(MTE_EINVAL, "unknown series %d", sid);
    it->second.pending++;
    *dev = it->second.buf->as<float>();
    *P = it->second.P;
    *T = it->second.T;
    return MTE_OK;
}

// The z-scored copy of a registered series (mte_standardise), registered
// as a series of its own on first use and released with the original.
int series_standardised(int32_t sid, int32_t *std_sid) {
    Server &sv = server();
    int P;
    int64_t T;
    std::vector<float> host;
    {
        std::lock_guard<std::mutex> lk(sv.mu);
        auto it = sv.series.find(sid);
        if (it == sv.series.end()) return fail(MTE_EINVAL, "unknown series %d", sid);
        if (it->second.cancelled) return fail(MTE_ECANCELED, "series %d was cancelled", sid);
        if (it->second.std_sid >= 0) {
            *std_sid = it->second.std_sid;
            return MTE_OK;
        }
        P = it->second.P;
        T = it->second.T;
        host.resize((size_t)P * T);
        MTE_HIP(hipMemcpy(host.data(), it->second.buf->p, sizeof(float) * host.size(), hipMemcpyDeviceToHost));
    }
    standardise_host(host.data(), 1, P, T, host.data());
    int32_t made = -1;
    int rc = mte_series_register(host.data(), P, T, &made);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(sv.mu);
    auto it = sv.series.find(sid);
    if (it == sv.series.end()) {
        sv.series.erase(made);
        return fail(MTE_EINVAL, "series %d was released", sid);
    }
    if (it->second.std_sid >= 0) {
        sv.series.erase(made);       // another thread made it first
    } else {
        it->second.std_sid = made;
    }
    *std_sid = it->second.std_sid;
    return MTE_OK;
}

void series_unpin(int32_t sid) {
    Server &sv = server();
    std::lock_guard<std::mutex> lk(sv.mu);
    auto it = sv.series.find(sid);
    if (it != sv.series.end()) it->second.pending--;
}

}  // namespace mte

using namespace mte;

extern "C" {

int mte_series_register(const float *data, int P, int64_t T, int32_t *sid_out) {
    if (!data || !sid_out || P < 1 || T < 2) return fail(MTE_EINVAL, "bad series arguments");
    int rc = validate_host_finite(data, (int64_t)P * T, "data");
    if (rc) return rc;
    if ((rc = ensure_init())) return rc;
    auto buf = std::make_unique<DevBuf>();
    if ((rc = buf->ensure(sizeof(float) * (size_t)P * T))) return rc;
    MTE_HIP(hipMemcpy(buf->p, data, sizeof(float) * (size_t)P * T, hipMemcpyHostToDevice));
    Server &sv = server();
    std::lock_guard<std::mutex> lk(sv.mu);
    const int32_t sid = sv.next_sid++;
    Series &s = sv.series[sid];
    s.buf = std::move(buf);
    s.P = P;
    s.T = T;
    *sid_out = sid;
    return MTE_OK;
}

int mte_series_release(int32_t sid) {
    Server &sv = server();
    std::lock_guard<std::mutex> lk(sv.mu);
    auto it = sv.series.find(sid);
    if (it == sv.series.end()) return fail(MTE_EINVAL, "unknown series %d", sid);
    if (it->second.pending > 0) return fail(MTE_EBUSY, "series %d has pending requests", sid);
    const int32_t std_sid = it->second.std_sid;
    if (std_sid >= 0) {
        auto st = sv.series.find(std_sid);
        if (st != sv.series.end() && st->second.pending > 0)
            return fail(MTE_EBUSY, "series %d has pending requests", sid);
        if (st != sv.series.end()) sv.series.erase(st);
    }
    sv.series.erase(sid);
    return MTE_OK;
}

int mte_submit(const mte_request *req, uint64_t *ticket_out) {
    if (!req || !ticket_out || !req->nodes || !req->lags) return fail(MTE_EINVAL, "null argument");
    int rc = validate_dims(req->dx, req->dy, req->dz, req->N, req->k);
    if (!rc) rc = validate_theiler(req->N, req->k, req->theiler);
    if (rc) return rc;
    if (req->S < 0) return fail(MTE_EINVAL, "S must be >= 0");
    Server &sv = server();
    std::lock_guard<std::mutex> lk(sv.mu);
    auto it = sv.series.find(req->sid);
    if (it == sv.series.end()) return fail(MTE_EINVAL, "unknown series %d", req->sid);
    const Series &se = it->second;
    if (se.cancelled) return fail(MTE_ECANCELED, "series %d was cancelled", req->sid);
    const int d = req->dx + req->dy + req->dz;
    for (int c = 0; c < d; ++c) {
        if (req->nodes[c] < 0 || req->nodes[c] >= se.P) return fail(MTE_EINVAL, "node out of range");
        if (req->lags[c] < 0) return fail(MTE_EINVAL, "negative lag");
        if (req->t0 - req->lags[c] < 0 || req->t0 + req->N - 1 - req->lags[c] >= se.T)
            return fail(MTE_EINVAL, "window of column %d leaves the series", c);
    }
    if ((rc = sv.start_locked())) return rc;
    auto q = std::make_shared<Req>();
    q->ticket = sv.next_ticket++;
    q->r = *req;
    q->nodes.assign(req->nodes, req->nodes + d);
    q->lags.assign(req->lags, req->lags + d);
    q->r.nodes = q->nodes.data();
    q->r.lags = q->lags.data();
    q->t_submit = Clock::now();
    sv.reqs[q->ticket] = q;
    sv.queue.push_back(q);
    sv.series[req->sid].pending++;
    sv.submitted++;
    *ticket_out = q->ticket;
    sv.cv_work.notify_one();
    return MTE_OK;
}

int mte_wait(uint64_t ticket, double *cmi_out, double *surr_out, double timeout_s) {
    if (!cmi_out) return fail(MTE_EINVAL, "null output pointer");
    Server &sv = server();
    std::unique_lock<std::mutex> lk(sv.mu);
    auto it = sv.reqs.find(ticket);
    if (it == sv.reqs.end()) return fail(MTE_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    std::shared_ptr<Req> q = it->second;
    auto done = [&] { return q->state == 2; };
    if (timeout_s < 0) sv.cv_done.wait(lk, done);
    else if (!sv.cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), done))
        return fail(MTE_ETIMEOUT, "request %llu still pending", (unsigned long long)ticket);
    sv.reqs.erase(ticket);
    if (q->status != MTE_OK) return fail(q->status, "request failed: %s", q->error.c_str());
    *cmi_out = q->result[0];
    if (surr_out && q->r.S > 0) std::memcpy(surr_out, q->result.data() + 1, sizeof(double) * q->r.S);
    return MTE_OK;
}

int mte_serve_get_stats(mte_serve_stats *out, int reset) {
    if (!out) return fail(MTE_EINVAL, "null argument");
    Server &sv = server();
    std::lock_guard<std::mutex> lk(sv.mu);
    std::memset(out, 0, sizeof *out);
    out->submitted = sv.submitted;
    out->completed = sv.completed;
    out->rejected = sv.rejected;
    out->batches = sv.batches;
    out->estimates = sv.estimates;
    out->mean_batch_requests = sv.batches ? (double)sv.batch_reqs / (double)sv.batches : 0.0;
    out->peak_bytes_in_use = (int64_t)sv.peak_bytes;
    out->budget_bytes = (int64_t)ctx().budget;
    out->waited = sv.waited;
    if (!sv.latencies.empty()) {
        const size_t m = sv.latencies.size();
        auto pct = [&](double Server::Lat::*f, double p) {
            std::vector<double> l(m);
            for (size_t i = 0; i < m; ++i) l[i] = sv.latencies[i].*f;
            std::sort(l.begin(), l.end());
            return l[(size_t)std::min<double>((double)m - 1, std::ceil(p * (double)m) - 1)];
        };
        out->p50_latency_s = pct(&Server::Lat::total, 0.50);
        out->p99_latency_s = pct(&Server::Lat::total, 0.99);
        out->queue_p50_s = pct(&Server::Lat::queue, 0.50);
        out->queue_p99_s = pct(&Server::Lat::queue, 0.99);
        out->host_p50_s = pct(&Server::Lat::host, 0.50);
        out->host_p99_s = pct(&Server::Lat::host, 0.99);
        out->device_p50_s = pct(&Server::Lat::device, 0.50);
        out->device_p99_s = pct(&Server::Lat::device, 0.99);
        // the requests at or above the p99 latency, their phases averaged
        int64_t nt = 0;
        for (const auto &L : sv.latencies) {
            if (L.total < out->p99_latency_s) continue;
            ++nt;
            out->tail_queue_s += L.queue;
            out->tail_host_s += L.host;
            out->tail_device_s += L.device;
            out->tail_mean_n += (double)L.n;
            out->tail_mean_batch_requests += (double)L.batch;
        }
        out->tail_requests = nt;
        out->tail_queue_s /= (double)nt;
        out->tail_host_s /= (double)nt;
        out->tail_device_s /= (double)nt;
        out->tail_mean_n /= (double)nt;
        out->tail_mean_batch_requests /= (double)nt;
    }
    if (reset) {
        sv.submitted = sv.completed = sv.rejected = sv.batches = sv.estimates = sv.batch_reqs = sv.waited = 0;
        sv.latencies.clear();
        sv.peak_bytes = sv.bytes_in_flight;
    }
    return MTE_OK;
}

int mte_serve_cancel(int32_t sid) {
    Server &sv = server();
    std::lock_guard<std::mutex> lk(sv.mu);
    auto it = sv.series.find(sid);
    if (it == sv.series.end()) return fail(MTE_EINVAL, "unknown series %d", sid);
    it->second.cancelled = true;
    sv.cancel(sid);
    const int32_t std_sid = it->second.std_sid;
    auto st = std_sid >= 0 ? sv.series.find(std_sid) : sv.series.end();
    if (st != sv.series.end()) {
        st->second.cancelled = true;
        sv.cancel(std_sid);
    }
    return MTE_OK;
}

int mte_select_sources_sid(int32_t sid, int target, const int32_t *candidates, int n_candidates,
                           int max_lag_sources, double alpha, const mte_opts *opts, mte_result *out) {
    int P = 0;
    int64_t T = 0;
    int rc = series_shape(sid, &P, &T);
    if (rc) return rc;
    return select_sources_served(sid, P, T, target, candidates, n_candidates, max_lag_sources,
                                     alpha, opts, out);
}

}  // extern "C"
