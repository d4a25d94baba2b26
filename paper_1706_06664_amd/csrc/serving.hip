// Serving loop: a request queue in front of one ACE context.
//
// A request is a batch of rows to insert (counting phase of Alg. 1) or to score (query
// phase).  Admission takes one of S slots; each slot owns a HIP stream, the hash
// workspace, device buffers for its rows and outputs, and pinned host staging.  On its
// slot's stream a request runs H2D copy -> hash -> count update (insert) or score + D2H
// copy (score), then records the slot's event.  A completion thread polls the events of
// busy slots, copies staged outputs to the caller, records the latency and frees the slot.
//
// Ordering.  Inserts are integer adds and commute with each other; scores only read the
// counts and commute with each other.  An insert and a score do not commute, so a request
// waits (hipStreamWaitEvent, after its H2D copy) on the events of every request of the other
// kind still in flight when it is admitted.  Requests that completed earlier are already
// visible.  Hence a score sees exactly the inserts admitted before it, whatever S is: the
// results equal those of running the requests one by one in admission order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <mutex>
#include <thread>
#include <vector>

#include "ace_context.h"

using namespace ace;

namespace {

using Clock = std::chrono::steady_clock;

struct Slot {
    hipStream_t s = nullptr;
    hipEvent_t done = nullptr;
    Workspace ws;
    float* Xd = nullptr;       // [max_rows][d] device rows
    float* sd = nullptr;       // [max_rows] device scores
    uint32_t* Td = nullptr;    // [max_rows] device totals
    float* Xh = nullptr;       // pinned staging of the rows
    float* sh = nullptr;       // pinned staging of the outputs
    uint32_t* Th = nullptr;
    // request in flight
    bool busy = false;
    int kind = 0;
    int64_t n = 0;
    uint64_t ticket = 0;
    float* s_user = nullptr;
    uint32_t* T_user = nullptr;
    bool staged_out = false;
    Clock::time_point t_arrive;
};

double ms_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

}  // namespace

struct ace_server_s {
    ace_ctx c = nullptr;
    ace_server_config cfg{};
    std::vector<Slot> slots;
    std::mutex mu;                   // guards slot state, latency records, stats
    std::condition_variable cv;      // a slot became free / busy, or a request completed
    std::mutex submit_mu;            // one submitter at a time
    std::thread completer;
    bool stop = false;
    ace_status err = ACE_OK;         // first device error seen by the completion thread
    size_t bytes = 0;                // device bytes the slots hold (returned to the budget on destroy)
    uint64_t next_ticket = 0;
    uint64_t ticket_base = 0;        // latency records start at this ticket
    std::vector<double> latency_ms;  // per ticket since ticket_base (-1 while in flight)
    std::vector<uint8_t> kind_of;    // per ticket since ticket_base
    std::vector<int64_t> rows_of;
    int64_t inflight = 0;
    int next_slot = 0;
    bool have_first = false;
    Clock::time_point t_first, t_last;
};

namespace {

void completion_loop(ace_server srv) {
    (void)hipSetDevice(srv->c->cfg.device);
    std::vector<int> busy;
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(srv->mu);
            srv->cv.wait(lk, [&] { return srv->stop || srv->inflight > 0; });
            if (srv->stop && srv->inflight == 0) return;
            busy.clear();
            for (int i = 0; i < (int)srv->slots.size(); ++i)
                if (srv->slots[i].busy) busy.push_back(i);
        }
        bool any = false;
        for (int i : busy) {
            Slot& sl = srv->slots[i];
            hipError_t q = hipEventQuery(sl.done);
            if (q == hipErrorNotReady) continue;
            ace_status st = ACE_OK;
            if (q != hipSuccess) {
                (void)hipGetLastError();
                st = ACE_E_DEVICE;
            } else if (sl.kind == ACE_REQ_SCORE && sl.staged_out) {
                if (sl.s_user) std::memcpy(sl.s_user, sl.sh, sizeof(float) * (size_t)sl.n);
                if (sl.T_user) std::memcpy(sl.T_user, sl.Th, sizeof(uint32_t) * (size_t)sl.n);
            }
            const Clock::time_point now = Clock::now();
            {
                std::lock_guard<std::mutex> lk(srv->mu);
                if (st != ACE_OK && srv->err == ACE_OK) srv->err = st;
                if (sl.ticket >= srv->ticket_base) srv->latency_ms[sl.ticket - srv->ticket_base] = ms_between(sl.t_arrive, now);
                srv->t_last = now;
                sl.busy = false;
                --srv->inflight;
            }
            any = true;
        }
        if (any) srv->cv.notify_all();
        else std::this_thread::yield();
    }
}

void free_slot(ace_ctx c, Slot& sl) {
    ws_free(&sl.ws);
    void* dev[] = {sl.Xd, sl.sd, sl.Td};
    for (void* p : dev)
        if (p) (void)hipFree(p);
    void* host[] = {sl.Xh, sl.sh, sl.Th};
    for (void* p : host)
        if (p) (void)hipHostFree(p);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.s) (void)hipStreamDestroy(sl.s);
    sl = Slot();
}

ace_status alloc_slot(ace_ctx c, Slot& sl, int64_t rows) {
    const size_t d = (size_t)c->cfg.d;
    if (hipStreamCreateWithFlags(&sl.s, hipStreamNonBlocking) != hipSuccess) return ACE_E_DEVICE;
    if (hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess) return ACE_E_DEVICE;
    ace_status st = ws_alloc(c, &sl.ws, rows);
    st = st ? st : dev_alloc(c, (void**)&sl.Xd, sizeof(float) * d * (size_t)rows);
    st = st ? st : dev_alloc(c, (void**)&sl.sd, sizeof(float) * (size_t)rows);
    st = st ? st : dev_alloc(c, (void**)&sl.Td, sizeof(uint32_t) * (size_t)rows);
    if (st) return st;
    if (hipHostMalloc((void**)&sl.Xh, sizeof(float) * d * (size_t)rows, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&sl.sh, sizeof(float) * (size_t)rows, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&sl.Th, sizeof(uint32_t) * (size_t)rows, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return ACE_E_NOMEM;
    }
    return ACE_OK;
}

struct DevGuard {
    int prev = -1;
    explicit DevGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        (void)hipSetDevice(dev);
    }
    ~DevGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// Enqueue one admitted request on its slot's stream.  Called with submit_mu held.
ace_status enqueue(ace_server srv, Slot& sl, int kind, const float* X, int64_t n, int32_t flags,
                   const std::vector<hipEvent_t>& waits) {
    ace_ctx c = srv->c;
    const size_t xbytes = sizeof(float) * (size_t)c->cfg.d * (size_t)n;
    const float* src = X;
    if (!(flags & ACE_SUBMIT_PINNED)) {
        std::memcpy(sl.Xh, X, xbytes);
        src = sl.Xh;
    }
    ace_status st = check(c, hipMemcpyAsync(sl.Xd, src, xbytes, hipMemcpyHostToDevice, sl.s));
    for (hipEvent_t e : waits)
        st = st ? st : check(c, hipStreamWaitEvent(sl.s, e, 0));
    st = st ? st : hash_chunk(c, &sl.ws, sl.Xd, n, false, sl.s);
    if (st) return st;
    if (kind == ACE_REQ_INSERT) {
        st = check(c, launch_count_update(sl.ws.codes, n, n, c->cfg.K, c->cfg.L, +1, c->counts, c->S2, c->S3, c->err,
                                          sl.s));
    } else {
        st = check(c, launch_score(sl.ws.codes, n, n, c->cfg.K, c->cfg.L, c->counts, sl.sd, sl.Td, c->mom, sl.s));
        if (st) return st;
        float* so = sl.staged_out ? sl.sh : sl.s_user;
        uint32_t* To = sl.staged_out ? sl.Th : sl.T_user;
        if (so && sl.s_user) st = check(c, hipMemcpyAsync(so, sl.sd, sizeof(float) * n, hipMemcpyDeviceToHost, sl.s));
        if (!st && To && sl.T_user)
            st = check(c, hipMemcpyAsync(To, sl.Td, sizeof(uint32_t) * n, hipMemcpyDeviceToHost, sl.s));
    }
    if (st) return st;
    return check(c, hipEventRecord(sl.done, sl.s));
}

ace_status submit_at(ace_server srv, int32_t kind, const float* X, int64_t n, float* s_host, uint32_t* T_host,
                     int32_t flags, Clock::time_point t_arrive, uint64_t* ticket) {
    ace_ctx c = srv->c;
    if (kind != ACE_REQ_INSERT && kind != ACE_REQ_SCORE) return ACE_E_INVALID;
    if (n < 1 || n > srv->cfg.max_rows || !X) return ACE_E_INVALID;
    if (flags & ~ACE_SUBMIT_PINNED) return ACE_E_INVALID;
    if (c->sticky != ACE_OK) return c->sticky;
    std::lock_guard<std::mutex> sub(srv->submit_mu);
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (srv->err != ACE_OK) return srv->err;
    }
    if (kind == ACE_REQ_INSERT && c->n_total + n > c->cap) return ACE_E_OVERFLOW;
    if (kind == ACE_REQ_SCORE && (u64)c->cfg.L * (u64)c->n_total > 0xFFFFFFFFull) return ACE_E_OVERFLOW;
    if (c->fail_next) {
        c->fail_next = 0;
        c->sticky = ACE_E_DEVICE;
        return ACE_E_DEVICE;
    }
    // Admission: wait for a free slot; collect the events of in-flight requests of the
    // other kind.
    int idx = -1;
    std::vector<hipEvent_t> waits;
    {
        std::unique_lock<std::mutex> lk(srv->mu);
        const int S = (int)srv->slots.size();
        srv->cv.wait(lk, [&] {
            for (int k = 0; k < S; ++k)
                if (!srv->slots[(srv->next_slot + k) % S].busy) return true;
            return false;
        });
        for (int k = 0; k < S; ++k) {
            const int i = (srv->next_slot + k) % S;
            if (!srv->slots[i].busy) {
                idx = i;
                break;
            }
        }
        srv->next_slot = (idx + 1) % S;
        for (auto& o : srv->slots)
            if (o.busy && o.kind != kind) waits.push_back(o.done);
    }
    Slot& sl = srv->slots[idx];
    sl.kind = kind;
    sl.n = n;
    sl.s_user = s_host;
    sl.T_user = T_host;
    sl.staged_out = !(flags & ACE_SUBMIT_PINNED);
    sl.t_arrive = t_arrive;
    DevGuard g(c->cfg.device);
    ace_status st = enqueue(srv, sl, kind, X, n, flags, waits);
    if (st) return st;
    if (kind == ACE_REQ_INSERT) c->n_total += n;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        sl.ticket = srv->next_ticket++;
        srv->latency_ms.push_back(-1.0);
        srv->kind_of.push_back((uint8_t)kind);
        srv->rows_of.push_back(n);
        if (!srv->have_first) {
            srv->have_first = true;
            srv->t_first = t_arrive;
        }
        sl.busy = true;
        ++srv->inflight;
        if (ticket) *ticket = sl.ticket;
    }
    srv->cv.notify_all();
    return ACE_OK;
}

double percentile(std::vector<double>& v, double p) {
    if (v.empty()) return 0.0;
    // nearest-rank percentile
    size_t r = (size_t)std::ceil(p / 100.0 * (double)v.size());
    if (r < 1) r = 1;
    std::nth_element(v.begin(), v.begin() + (r - 1), v.end());
    return v[r - 1];
}

}  // namespace

extern "C" {

ace_status ace_server_create(ace_ctx c, const ace_server_config* cfg, ace_server* out) {
    if (!c || !cfg || !out) return ACE_E_INVALID;
    if (c->sticky != ACE_OK) return c->sticky;
    if (cfg->slots < 1 || cfg->slots > 64 || cfg->max_rows < 1 || cfg->max_rows > ((int64_t)1 << 24)) return ACE_E_INVALID;
    if (cfg->use_graphs != 0 || cfg->reserved != 0) return ACE_E_INVALID;
    if (c->server_attached) return ACE_E_STATE;
    DevGuard g(c->cfg.device);
    ace_server srv = new ace_server_s();
    srv->c = c;
    srv->cfg = *cfg;
    srv->slots.resize(cfg->slots);
    const size_t bytes0 = c->bytes;
    ace_status st = ACE_OK;
    for (auto& sl : srv->slots) {
        st = alloc_slot(c, sl, cfg->max_rows);
        if (st) break;
    }
    srv->bytes = c->bytes - bytes0;
    if (st) {
        for (auto& sl : srv->slots) free_slot(c, sl);
        c->bytes -= srv->bytes;
        delete srv;
        return st;
    }
    c->server_attached = 1;
    srv->completer = std::thread(completion_loop, srv);
    *out = srv;
    return ACE_OK;
}

ace_status ace_server_submit(ace_server srv, int32_t kind, const float* X_host, int64_t n, float* s_host,
                             uint32_t* T_host, int32_t flags, uint64_t* ticket) {
    if (!srv) return ACE_E_INVALID;
    return submit_at(srv, kind, X_host, n, s_host, T_host, flags, Clock::now(), ticket);
}

ace_status ace_server_wait(ace_server srv, uint64_t ticket, double* latency_ms) {
    if (!srv) return ACE_E_INVALID;
    std::unique_lock<std::mutex> lk(srv->mu);
    if (ticket >= srv->next_ticket) return ACE_E_INVALID;
    auto done = [&] {
        if (srv->err != ACE_OK) return true;
        for (auto& sl : srv->slots)
            if (sl.busy && sl.ticket == ticket) return false;
        return true;
    };
    srv->cv.wait(lk, done);
    if (latency_ms)
        *latency_ms = ticket >= srv->ticket_base ? srv->latency_ms[ticket - srv->ticket_base] : -1.0;
    return srv->err;
}

ace_status ace_server_drain(ace_server srv) {
    if (!srv) return ACE_E_INVALID;
    std::lock_guard<std::mutex> sub(srv->submit_mu);
    std::unique_lock<std::mutex> lk(srv->mu);
    srv->cv.wait(lk, [&] { return srv->inflight == 0; });
    return srv->err != ACE_OK ? srv->err : srv->c->sticky;
}

ace_status ace_server_replay(ace_server srv, const ace_request* reqs, int64_t nreq, const float* pool,
                             int64_t pool_rows, int32_t flags, float* s_out, uint32_t* T_out, double* latency_ms) {
    if (!srv || (nreq > 0 && (!reqs || !pool))) return ACE_E_INVALID;
    if (nreq < 0 || pool_rows < 0 || (flags & ~ACE_SUBMIT_PINNED)) return ACE_E_INVALID;
    for (int64_t r = 0; r < nreq; ++r) {
        const ace_request& q = reqs[r];
        if (q.n < 1 || q.row0 < 0 || q.row0 + q.n > pool_rows || q.t_arrival_s < 0) return ACE_E_INVALID;
        if (q.kind == ACE_REQ_SCORE && (s_out || T_out) && q.out0 < 0) return ACE_E_INVALID;
    }
    const size_t d = (size_t)srv->c->cfg.d;
    std::vector<uint64_t> tickets((size_t)nreq);
    const Clock::time_point t0 = Clock::now();
    for (int64_t r = 0; r < nreq; ++r) {
        const ace_request& q = reqs[r];
        Clock::time_point ta = Clock::now();
        if (q.t_arrival_s > 0) {
            ta = t0 + std::chrono::duration_cast<Clock::duration>(std::chrono::duration<double>(q.t_arrival_s));
            while (Clock::now() < ta) std::this_thread::yield();
        }
        float* so = (q.kind == ACE_REQ_SCORE && s_out) ? s_out + q.out0 : nullptr;
        uint32_t* To = (q.kind == ACE_REQ_SCORE && T_out) ? T_out + q.out0 : nullptr;
        ace_status st = submit_at(srv, q.kind, pool + (size_t)q.row0 * d, q.n, so, To, flags, ta, &tickets[r]);
        if (st) {
            (void)ace_server_drain(srv);
            return st;
        }
    }
    ace_status st = ace_server_drain(srv);
    if (latency_ms) {
        std::lock_guard<std::mutex> lk(srv->mu);
        for (int64_t r = 0; r < nreq; ++r)
            latency_ms[r] = tickets[r] >= srv->ticket_base ? srv->latency_ms[tickets[r] - srv->ticket_base] : -1.0;
    }
    return st;
}

ace_status ace_server_get_stats(ace_server srv, ace_server_stats* out) {
    if (!srv || !out) return ACE_E_INVALID;
    std::lock_guard<std::mutex> lk(srv->mu);
    ace_server_stats s{};
    std::vector<double> all, ins, sco;
    for (size_t i = 0; i < srv->latency_ms.size(); ++i) {
        const double v = srv->latency_ms[i];
        if (v < 0) continue;
        all.push_back(v);
        (srv->kind_of[i] == ACE_REQ_INSERT ? ins : sco).push_back(v);
        s.rows += srv->rows_of[i];
        if (srv->kind_of[i] == ACE_REQ_INSERT) s.insert_rows += srv->rows_of[i];
    }
    s.requests = (int64_t)all.size();
    s.inserts = (int64_t)ins.size();
    s.scores = (int64_t)sco.size();
    double sum = 0, mx = 0;
    for (double v : all) {
        sum += v;
        mx = std::max(mx, v);
    }
    s.mean_ms = all.empty() ? 0.0 : sum / (double)all.size();
    s.max_ms = mx;
    s.p50_ms = percentile(all, 50.0);
    s.p99_ms = percentile(all, 99.0);
    s.p99_insert_ms = percentile(ins, 99.0);
    s.p99_score_ms = percentile(sco, 99.0);
    s.wall_ms = srv->have_first ? ms_between(srv->t_first, srv->t_last) : 0.0;
    *out = s;
    return ACE_OK;
}

ace_status ace_server_reset_stats(ace_server srv) {
    if (!srv) return ACE_E_INVALID;
    std::lock_guard<std::mutex> sub(srv->submit_mu);
    std::unique_lock<std::mutex> lk(srv->mu);
    srv->cv.wait(lk, [&] { return srv->inflight == 0; });
    srv->ticket_base = srv->next_ticket;
    srv->latency_ms.clear();
    srv->kind_of.clear();
    srv->rows_of.clear();
    srv->have_first = false;
    return ACE_OK;
}

ace_status ace_server_destroy(ace_server srv) {
    if (!srv) return ACE_E_INVALID;
    (void)ace_server_drain(srv);
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
    }
    srv->cv.notify_all();
    srv->completer.join();
    DevGuard g(srv->c->cfg.device);
    for (auto& sl : srv->slots) {
        (void)hipStreamSynchronize(sl.s);
        free_slot(srv->c, sl);
    }
    srv->c->bytes -= srv->bytes;
    srv->c->server_attached = 0;
    delete srv;
    return ACE_OK;
}

}  // extern "C"
