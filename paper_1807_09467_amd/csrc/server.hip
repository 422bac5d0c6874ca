// Serving loop of the rsolve library (include/rsolve_server.h): admission by pool memory and
// slots, one batch worker for sequences within the one-block limits (continuous batching through
// rsolve_solve_batch / rsolve_update_recycle_batch), and large workers with one HIP stream each
// for the rest.  Host code only; every solve runs through the library's own entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <set>
#include <thread>
#include <vector>

#include "../../include/rsolve.h"
#include "../../include/rsolve_server.h"
#include "engine_internal.hpp"

namespace {

using Clock = std::chrono::steady_clock;
constexpr size_t POOL_ALIGN = 256;

double ms_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

struct Req {
    uint64_t tag = 0;
    uint64_t seq_id = 0;
    rsolve_seq* h = nullptr;
    rsolve_csr A{};
    const double* b = nullptr;
    const double* x0 = nullptr;
    double* x = nullptr;
    double tol = 0.0;
    hipEvent_t ev = nullptr;
    Clock::time_point t_submit;
};

struct SeqRec {
    rsolve_seq* h = nullptr;
    size_t off = 0, bytes = 0;
    int64_t n = 0;
    bool small = false;
    int worker = -1;   // index into large workers, -1 = batch worker
    int inflight = 0;
    bool closing = false;
};

// First-fit allocator over the caller's pool, in POOL_ALIGN units, coalescing on release.
struct Pool {
    std::map<size_t, size_t> free_;  // offset -> bytes
    void init(size_t bytes) {
        free_.clear();
        const size_t usable = bytes / POOL_ALIGN * POOL_ALIGN;
        if (usable) free_[0] = usable;
    }
    bool take(size_t bytes, size_t* off) {
        bytes = (bytes + POOL_ALIGN - 1) / POOL_ALIGN * POOL_ALIGN;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes;
            const size_t roff = it->first + bytes;
            free_.erase(it);
            if (rest) free_[roff] = rest;
            return true;
        }
        return false;
    }
    void give(size_t off, size_t bytes) {
        bytes = (bytes + POOL_ALIGN - 1) / POOL_ALIGN * POOL_ALIGN;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t largest() const {
        size_t m = 0;
        for (auto& kv : free_) m = std::max(m, kv.second);
        return m;
    }
};

struct Worker {
    std::thread th;
    hipStream_t stream = nullptr;
    std::deque<Req> q;
    int64_t load = 0;   // sum of n over its sequences
};

bool fits_one_block(const rsolve_config& c, int64_t n) {
    return c.restart_m <= RSOLVE_SMALL_MAX_RESTART && c.recycle_k <= RSOLVE_SMALL_MAX_RECYCLE &&
           n <= RSOLVE_SMALL_MAX_N && c.method <= RSOLVE_DEFL_OBLIQUE && c.precond != RSOLVE_PRECOND_SSOR;
}

}  // namespace

struct rsolve_server {
    rsolve_server_config cfg{};
    int device = 0;
    hipStream_t admin = nullptr;   // stream of sequence creation and destruction
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    Pool pool;
    size_t used = 0;
    std::map<uint64_t, SeqRec> seqs;
    uint64_t next_id = 1;
    Worker batch;
    std::vector<Worker> large;
    std::deque<rsolve_completion> done;
    int pending = 0;
    int64_t completed = 0, batches = 0, batched_solves = 0;
    bool stop = false;

    void post(std::vector<rsolve_completion>& out, const std::vector<uint64_t>& ids) {
        {
            std::lock_guard<std::mutex> lk(mu);
            for (size_t i = 0; i < out.size(); ++i) {
                done.push_back(out[i]);
                auto it = seqs.find(ids[i]);
                if (it != seqs.end()) it->second.inflight--;
            }
            pending -= (int)out.size();
            completed += (int64_t)out.size();
        }
        cv_done.notify_all();
    }

    void batch_loop() {
        (void)hipSetDevice(device);
        std::vector<rsolve_batch_solve_item> items;
        std::vector<rsolve_batch_update_item> upd;
        for (;;) {
            std::vector<Req> take;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_work.wait(lk, [&] { return stop || !batch.q.empty(); });
                if (batch.q.empty()) return;   // stop requested and nothing left
                // the oldest request of each sequence, in arrival order, up to max_batch
                std::set<uint64_t> seen;
                for (auto it = batch.q.begin(); it != batch.q.end();) {
                    if (seen.count(it->seq_id)) {
                        ++it;
                        continue;
                    }
                    seen.insert(it->seq_id);
                    if ((int)take.size() < cfg.max_batch) {
                        take.push_back(*it);
                        it = batch.q.erase(it);
                    } else {
                        ++it;
                    }
                }
            }
            const auto t_start = Clock::now();
            const int cnt = (int)take.size();
            items.assign(cnt, rsolve_batch_solve_item{});
            for (int i = 0; i < cnt; ++i) {
                const Req& r = take[i];
                if (r.ev) (void)hipStreamWaitEvent(batch.stream, r.ev, 0);
                items[i].seq = r.h;
                items[i].A = r.A;
                items[i].b = r.b;
                items[i].x0 = r.x0;
                items[i].x = r.x;
                items[i].tol = r.tol;
            }
            const int rc = rsolve_solve_batch(items.data(), cnt, batch.stream);
            upd.clear();
            std::vector<int> upd_of;
            for (int i = 0; i < cnt; ++i) {
                if (rc != RSOLVE_OK) items[i].status = rc;
                if (items[i].status == RSOLVE_OK || items[i].status == RSOLVE_NOT_CONVERGED) {
                    upd.push_back(rsolve_batch_update_item{take[i].h, nullptr, 0, 0});
                    upd_of.push_back(i);
                }
            }
            const int urc = rsolve_update_recycle_batch(upd.data(), (int32_t)upd.size(), batch.stream);
            for (size_t u = 0; u < upd.size(); ++u) {
                const int st = urc != RSOLVE_OK ? urc : upd[u].status;
                if (st != RSOLVE_OK) items[upd_of[u]].status = st;
            }
            const auto t_end = Clock::now();
            std::vector<rsolve_completion> out(cnt);
            std::vector<uint64_t> ids(cnt);
            for (int i = 0; i < cnt; ++i) {
                rsolve_completion& c = out[i];
                memset(&c, 0, sizeof(c));
                c.tag = take[i].tag;
                c.seq_id = take[i].seq_id;
                c.status = items[i].status;
                c.batched = 1;
                c.stats = items[i].stats;
                c.t_latency_ms = ms_between(take[i].t_submit, t_end);
                c.t_queue_ms = ms_between(take[i].t_submit, t_start);
                ids[i] = take[i].seq_id;
            }
            {
                std::lock_guard<std::mutex> lk(mu);
                batches += 1;
                batched_solves += cnt;
            }
            post(out, ids);
        }
    }

    void large_loop(int w) {
        (void)hipSetDevice(device);
        Worker& me = large[w];
        for (;;) {
            Req r;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_work.wait(lk, [&] { return stop || !me.q.empty(); });
                if (me.q.empty()) return;
                r = me.q.front();
                me.q.pop_front();
            }
            const auto t_start = Clock::now();
            if (r.ev) (void)hipStreamWaitEvent(me.stream, r.ev, 0);
            rsolve_completion c;
            memset(&c, 0, sizeof(c));
            int st = rsolve_solve(r.h, &r.A, r.b, r.x0, r.x, r.tol, &c.stats);
            if (st == RSOLVE_OK || st == RSOLVE_NOT_CONVERGED) {
                const int u = rsolve_update_recycle(r.h, nullptr);
                if (u != RSOLVE_OK) st = u;
            }
            const auto t_end = Clock::now();
            c.tag = r.tag;
            c.seq_id = r.seq_id;
            c.status = st;
            c.batched = 0;
            c.t_latency_ms = ms_between(r.t_submit, t_end);
            c.t_queue_ms = ms_between(r.t_submit, t_start);
            std::vector<rsolve_completion> out{c};
            std::vector<uint64_t> ids{r.seq_id};
            post(out, ids);
        }
    }
};

extern "C" {

int rsolve_server_create(const rsolve_server_config* cfg, rsolve_server** out) {
    if (!out) return RSOLVE_E_INVALID;
    *out = nullptr;
    if (!cfg || !cfg->pool || cfg->pool_bytes < POOL_ALIGN ||
        reinterpret_cast<uintptr_t>(cfg->pool) % POOL_ALIGN != 0 || cfg->large_workers < 1 ||
        cfg->large_workers > 64 || cfg->max_batch < 1 || cfg->max_batch > 256 || cfg->max_sequences < 1 ||
        (cfg->small_fp64 != 0 && cfg->small_fp64 != 1))
        return RSOLVE_E_INVALID;
    rsolve_server* s = new rsolve_server();
    s->cfg = *cfg;
    hipError_t e = hipGetDevice(&s->device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->admin, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->batch.stream, hipStreamNonBlocking);
    s->large.resize(cfg->large_workers);
    for (auto& w : s->large)
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&w.stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        if (s->admin) (void)hipStreamDestroy(s->admin);
        if (s->batch.stream) (void)hipStreamDestroy(s->batch.stream);
        for (auto& w : s->large)
            if (w.stream) (void)hipStreamDestroy(w.stream);
        delete s;
        return RSOLVE_E_DEVICE;
    }
    s->pool.init(cfg->pool_bytes);
    s->batch.th = std::thread([s] { s->batch_loop(); });
    for (int w = 0; w < cfg->large_workers; ++w) s->large[w].th = std::thread([s, w] { s->large_loop(w); });
    *out = s;
    return RSOLVE_OK;
}

int rsolve_server_open(rsolve_server* s, const rsolve_config* cfg, int64_t n, int64_t nnz_max, uint64_t* seq_id) {
    if (!s || !cfg || !seq_id) return RSOLVE_E_INVALID;
    rsolve_config c = *cfg;
    bool small = false;
    if (fits_one_block(c, n)) {
        if (c.precision == RSOLVE_FP64) small = true;
        else if (s->cfg.small_fp64) {
            c.precision = RSOLVE_FP64;
            small = true;
        }
    }
    const size_t bytes = rsolve_workspace_bytes(&c, n, nnz_max);
    if (bytes == 0) return RSOLVE_E_INVALID;
    SeqRec rec;
    uint64_t id = 0;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if ((int)s->seqs.size() >= s->cfg.max_sequences) return RSOLVE_E_BUDGET;
        if (!s->pool.take(bytes, &rec.off)) return RSOLVE_E_BUDGET;
        rec.bytes = bytes;
        rec.n = n;
        rec.small = small;
        rec.closing = true;   // not visible to submit until created
        if (!small) {
            int best = 0;
            for (int w = 1; w < (int)s->large.size(); ++w)
                if (s->large[w].load < s->large[best].load) best = w;
            rec.worker = best;
            s->large[best].load += n;
        }
        id = s->next_id++;
        s->used += bytes;
        s->seqs[id] = rec;
    }
    // the workspace is cleared on the admin stream, then the sequence moves to its worker's stream
    char* base = static_cast<char*>(s->cfg.pool) + rec.off;
    rsolve_seq* h = nullptr;
    (void)hipSetDevice(s->device);
    const int rc = rsolve_create_sequence(&c, n, nnz_max, s->admin, base, bytes, &h);
    // served sequences run tens of steps: the per-pattern build of shared offset lists (a read-back
    // and a host pass over the rows) costs more than the few per cent it saves per product
    if (rc == RSOLVE_OK) rs::seq_set_offset_classes(h, false);
    std::lock_guard<std::mutex> lk(s->mu);
    SeqRec& r = s->seqs[id];
    if (rc != RSOLVE_OK) {
        s->pool.give(r.off, r.bytes);
        s->used -= r.bytes;
        if (r.worker >= 0) s->large[r.worker].load -= r.n;
        s->seqs.erase(id);
        return rc;
    }
    rs::seq_set_stream(h, r.worker >= 0 ? s->large[r.worker].stream : s->batch.stream);
    r.h = h;
    r.closing = false;
    *seq_id = id;
    return RSOLVE_OK;
}

int rsolve_server_submit(rsolve_server* s, uint64_t seq_id, const rsolve_csr* A, const double* b, const double* x0,
                         double* x, double tol, void* ready_event, uint64_t tag) {
    if (!s || !A || !b || !x || !(tol > 0.0)) return RSOLVE_E_INVALID;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->seqs.find(seq_id);
        if (it == s->seqs.end() || it->second.closing || A->n != it->second.n) return RSOLVE_E_INVALID;
        SeqRec& r = it->second;
        Req q;
        q.tag = tag;
        q.seq_id = seq_id;
        q.h = r.h;
        q.A = *A;
        q.b = b;
        q.x0 = x0;
        q.x = x;
        q.tol = tol;
        q.ev = reinterpret_cast<hipEvent_t>(ready_event);
        q.t_submit = Clock::now();
        (r.worker >= 0 ? s->large[r.worker].q : s->batch.q).push_back(q);
        r.inflight++;
        s->pending++;
    }
    s->cv_work.notify_all();
    return RSOLVE_OK;
}

int rsolve_server_poll(rsolve_server* s, rsolve_completion* out, int32_t cap, int32_t* count, int32_t timeout_ms) {
    if (!s || !count || cap < 0 || (cap > 0 && !out)) return RSOLVE_E_INVALID;
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->done.empty() && timeout_ms > 0)
        s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), [&] { return !s->done.empty(); });
    int c = 0;
    while (c < cap && !s->done.empty()) {
        out[c++] = s->done.front();
        s->done.pop_front();
    }
    *count = c;
    return RSOLVE_OK;
}

int rsolve_server_close(rsolve_server* s, uint64_t seq_id) {
    if (!s) return RSOLVE_E_INVALID;
    rsolve_seq* h = nullptr;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->seqs.find(seq_id);
        if (it == s->seqs.end() || it->second.closing) return RSOLVE_E_INVALID;
        if (it->second.inflight > 0) return RSOLVE_E_STATE;
        it->second.closing = true;
        h = it->second.h;
    }
    // nothing of this sequence is queued or running: destroy it away from the worker streams
    (void)hipSetDevice(s->device);
    rs::seq_set_stream(h, s->admin);
    const int rc = rsolve_destroy_sequence(h);
    std::lock_guard<std::mutex> lk(s->mu);
    SeqRec& r = s->seqs[seq_id];
    s->pool.give(r.off, r.bytes);
    s->used -= r.bytes;
    if (r.worker >= 0) s->large[r.worker].load -= r.n;
    s->seqs.erase(seq_id);
    return rc;
}

int rsolve_server_info_get(rsolve_server* s, rsolve_server_info* info) {
    if (!s || !info) return RSOLVE_E_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    info->pool_used = s->used;
    info->pool_largest_free = s->pool.largest();
    info->sequences = (int32_t)s->seqs.size();
    info->pending = s->pending;
    info->completed = s->completed;
    info->batches = s->batches;
    info->batched_solves = s->batched_solves;
    return RSOLVE_OK;
}

int rsolve_server_destroy(rsolve_server* s) {
    if (!s) return RSOLVE_E_INVALID;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->batch.th.joinable()) s->batch.th.join();
    for (auto& w : s->large)
        if (w.th.joinable()) w.th.join();
    (void)hipSetDevice(s->device);
    for (auto& kv : s->seqs) {
        if (!kv.second.h) continue;
        rs::seq_set_stream(kv.second.h, s->admin);
        (void)rsolve_destroy_sequence(kv.second.h);
    }
    s->seqs.clear();
    (void)hipStreamDestroy(s->batch.stream);
    for (auto& w : s->large) (void)hipStreamDestroy(w.stream);
    (void)hipStreamDestroy(s->admin);
    delete s;
    return RSOLVE_OK;
}

}  // extern "C"
