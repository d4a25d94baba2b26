// Serving loop: a request queue in front of one ACE context.
//
// A request is a block of rows to insert (counting phase of Alg. 1), to score (query
// phase) or to delete (rows inserted earlier leaving a sliding window: Sec. 3.4.1,
// Eq. dynsub).  Submission appends it to a FIFO queue.  A dispatcher thread does continuous
// batching: whenever one of S slots is free it takes the longest prefix of the queue that
// fits batch_rows rows (at least one request), inserts, scores and deletes mixed, as one batch.  Each slot owns a
// HIP stream, the hash workspace, device buffers for a batch and pinned host staging.  On
// its stream a batch runs host-to-device copies -> one hash of all its rows -> the count
// phase: one count-update (increment or decrement) or score launch per run of consecutive
// same-kind requests, in admission order -> device-to-host copy of s and T.  A completion thread polls the
// events of busy slots, copies each request's outputs to the caller, records its latency
// and frees the slot.  With use_graphs, the hash part of a batch is one hipGraph launch:
// the pipeline (list reset, conversion, projection, FP64 pass) is captured once per slot and
// row bucket (multiples of 256 rows up to 8192, then powers of two), and the kernels read the
// batch's real row count from
// a device word that a small copy sets before each launch.
//
// Ordering.  Hashing reads only the rows and W, so hashes of different batches overlap
// freely.  The count phase of a batch waits (hipStreamWaitEvent) on the count phase of the
// batch dispatched before it, so count phases run in admission order and a score sees
// exactly the inserts and deletes admitted before it, whatever S is: the results equal those of
// running the requests one at a time in admission order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "ace_context.h"

using namespace ace;

namespace {

using Clock = std::chrono::steady_clock;

// Rows of one request, or part of it, that the gather kernel copies: src is a device-mapped
// address of pinned host memory.
struct GatherTask {
    const float* src;
    int32_t dst_row;
    int32_t nrows;
};
constexpr int kGatherRows = 32;   // rows per task

// One workgroup per task: copy nrows * d contiguous floats from pinned host memory (read
// over the host link) into the batch's device rows.  16-byte loads when both ends allow.
__global__ __launch_bounds__(256) void gather_rows_kernel(const GatherTask* __restrict__ tasks, float* __restrict__ dst,
                                                          int d) {
    const GatherTask t = tasks[blockIdx.x];
    const int64_t count = (int64_t)t.nrows * d;
    float* o = dst + (int64_t)t.dst_row * d;
    if ((d & 3) == 0 && ((reinterpret_cast<uintptr_t>(t.src) & 15u) == 0)) {
        const float4* s4 = reinterpret_cast<const float4*>(t.src);
        float4* o4 = reinterpret_cast<float4*>(o);
        const int64_t c4 = count >> 2;
        int64_t i = threadIdx.x;
        for (; i + 3 * 256 < c4; i += 4 * 256) {
            const float4 a = s4[i], b = s4[i + 256], c = s4[i + 512], e = s4[i + 768];
            o4[i] = a;
            o4[i + 256] = b;
            o4[i + 512] = c;
            o4[i + 768] = e;
        }
        for (; i < c4; i += 256) o4[i] = s4[i];
    } else {
        for (int64_t i = threadIdx.x; i < count; i += 256) o[i] = t.src[i];
    }
}

constexpr size_t kMaxPending = 1 << 16;   // admitted but not completed requests

struct Req {
    int kind = 0;
    int64_t n = 0;
    const float* X = nullptr;
    float* s_user = nullptr;
    uint32_t* T_user = nullptr;
    bool pinned = false;          // copy from X directly (no staging)
    bool gather = false;          // X lies in device-mapped pinned memory: the gather kernel reads it
    uint64_t ticket = 0;
    int64_t off = 0;              // first row of the request inside its batch
    Clock::time_point t_arrive;
};

enum SlotState { SLOT_FREE = 0, SLOT_DISPATCHING = 1, SLOT_BUSY = 2 };

struct Slot {
    hipStream_t s = nullptr;
    hipEvent_t done = nullptr;     // the whole batch (outputs copied back)
    hipEvent_t cnt = nullptr;      // the batch's count phase (updates and scores)
    Workspace ws;
    float* Xd = nullptr;       // [max_rows][d] device rows of the batch
    float* sd = nullptr;       // [max_rows] device scores
    uint32_t* Td = nullptr;    // [max_rows] device totals
    float* Xh = nullptr;       // pinned staging of pageable rows
    float* sh = nullptr;       // pinned staging of the outputs
    uint32_t* Th = nullptr;
    GatherTask* tasks_h = nullptr;   // pinned: gather tasks of the batch
    GatherTask* tasks_d = nullptr;   // device copy read by the gather kernel
    int64_t task_cap = 0;
    int64_t* n_dev = nullptr;        // real rows of the batch (read by the captured hash)
    int64_t* n_host = nullptr;       // pinned source of n_dev
    std::vector<std::pair<int64_t, hipGraphExec_t>> graphs;   // hash pipeline per row bucket
    int state = SLOT_FREE;
    bool has_score = false;
    std::vector<Req> reqs;     // the batch in flight
};

double ms_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

}  // namespace

struct ace_server_s {
    ace_ctx c = nullptr;
    ace_server_config cfg{};
    std::vector<Slot> slots;
    std::mutex mu;                   // guards everything below
    std::condition_variable cv;      // queue, slot or completion state changed
    std::mutex submit_mu;            // one submitter at a time
    std::thread dispatcher, completer;
    bool stop = false;
    bool hold = false;               // test hook: no new batch while set (ace_server_debug_hold)
    ace_status err = ACE_OK;         // first device error (sticky)
    size_t bytes = 0;                // device bytes the slots hold (returned to the budget on destroy)
    std::deque<Req> queue;           // admitted, not yet dispatched
    int64_t pending = 0;             // admitted, not yet completed
    int64_t busy = 0;                // slots in SLOT_BUSY
    uint64_t next_ticket = 0;
    uint64_t ticket_base = 0;        // records start at this ticket
    std::vector<double> latency_ms;  // per ticket since ticket_base (-1 until completed)
    std::vector<double> queue_ms;    // per ticket: arrival to the launch of its batch
    std::vector<uint8_t> done_of;    // 0 pending, 1 completed, 2 withdrawn (ace_server_cancel)
    std::vector<uint8_t> kind_of;
    std::vector<int64_t> rows_of;
    int64_t batches = 0, batched_requests = 0, gathered_requests = 0, graph_launches = 0, graph_captures = 0;
    int64_t cancelled = 0;           // requests withdrawn from the queue since the last reset
    int next_slot = 0;
    int last_slot = -1;              // slot of the most recently dispatched batch
    bool have_first = false;
    Clock::time_point t_first, t_last;
};

namespace {

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

// Mark the requests of a batch complete (called with mu held).
void complete_locked(ace_server srv, std::vector<Req>& reqs, Clock::time_point now, bool ok) {
    for (const Req& q : reqs) {
        if (q.ticket >= srv->ticket_base) {
            const size_t i = q.ticket - srv->ticket_base;
            srv->latency_ms[i] = ok ? ms_between(q.t_arrive, now) : -1.0;
            srv->done_of[i] = 1;
        }
        --srv->pending;
    }
    srv->t_last = now;
    reqs.clear();
}

void completion_loop(ace_server srv) {
    (void)hipSetDevice(srv->c->cfg.device);
    std::vector<int> busy;
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(srv->mu);
            srv->cv.wait(lk, [&] { return srv->stop || srv->busy > 0; });
            if (srv->stop && srv->busy == 0) return;
            busy.clear();
            for (int i = 0; i < (int)srv->slots.size(); ++i)
                if (srv->slots[i].state == SLOT_BUSY) busy.push_back(i);
        }
        bool any = false;
        for (int i : busy) {
            Slot& sl = srv->slots[i];
            hipError_t q = hipEventQuery(sl.done);
            if (q == hipErrorNotReady) continue;
            const bool ok = q == hipSuccess;
            if (!ok) (void)hipGetLastError();
            if (ok && sl.has_score) {
                for (const Req& r : sl.reqs) {
                    if (r.kind != ACE_REQ_SCORE) continue;
                    if (r.s_user) std::memcpy(r.s_user, sl.sh + r.off, sizeof(float) * (size_t)r.n);
                    if (r.T_user) std::memcpy(r.T_user, sl.Th + r.off, sizeof(uint32_t) * (size_t)r.n);
                }
            }
            const Clock::time_point now = Clock::now();
            {
                std::lock_guard<std::mutex> lk(srv->mu);
                if (!ok && srv->err == ACE_OK) srv->err = ACE_E_DEVICE;
                complete_locked(srv, sl.reqs, now, ok);
                sl.state = SLOT_FREE;
                --srv->busy;
            }
            any = true;
        }
        if (any) srv->cv.notify_all();
        else std::this_thread::yield();
    }
}

// Capture the hash pipeline of a B-row bucket on the slot's stream (thread-local capture:
// the completion thread's event queries go on) and instantiate it.  The list reset inside
// is a fill kernel, not a memset.
ace_status capture_hash(ace_server srv, Slot& sl, int64_t B, hipGraphExec_t* out) {
    ace_ctx c = srv->c;
    const int prof = c->profiling;
    c->profiling = 0;   // no event records inside the graph
    ace_status st = check(c, hipStreamBeginCapture(sl.s, hipStreamCaptureModeThreadLocal));
    if (st) {
        c->profiling = prof;
        return st;
    }
    const ace_status hs = hash_chunk(c, &sl.ws, sl.Xd, B, false, sl.s, sl.n_dev, false);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(sl.s, &g);
    c->profiling = prof;
    st = hs ? hs : check(c, e);
    if (!st) st = check(c, hipGraphInstantiate(out, g, nullptr, nullptr, 0));
    if (g) (void)hipGraphDestroy(g);
    return st;
}

// Enqueue one batch on its slot's stream (dispatcher thread, no lock held).
ace_status enqueue_batch(ace_server srv, Slot& sl, int64_t rows, hipEvent_t wait_cnt) {
    ace_ctx c = srv->c;
    const size_t d = (size_t)c->cfg.d;
    ace_status st = ACE_OK;
    // Host-to-device copies of the rows; adjacent sources are merged into one copy.
    const float* run_src = nullptr;
    int64_t run_off = 0, run_n = 0;
    auto flush = [&] {
        if (run_n > 0 && !st)
            st = check(c, hipMemcpyAsync(sl.Xd + (size_t)run_off * d, run_src, sizeof(float) * d * (size_t)run_n,
                                         hipMemcpyHostToDevice, sl.s));
        run_n = 0;
    };
    int64_t ntask = 0;
    for (const Req& q : sl.reqs) {
        if (q.gather) {
            for (int64_t r = 0; r < q.n; r += kGatherRows)
                sl.tasks_h[ntask++] = GatherTask{q.X + (size_t)r * d, (int32_t)(q.off + r),
                                                 (int32_t)(q.n - r < kGatherRows ? q.n - r : kGatherRows)};
            continue;
        }
        const float* src = q.X;
        if (!q.pinned) {
            std::memcpy(sl.Xh + (size_t)q.off * d, q.X, sizeof(float) * d * (size_t)q.n);
            src = sl.Xh + (size_t)q.off * d;
        }
        if (run_n > 0 && src == run_src + (size_t)run_n * d) {
            run_n += q.n;
        } else {
            flush();
            run_src = src;
            run_off = q.off;
            run_n = q.n;
        }
    }
    flush();
    if (ntask > 0) {
        st = st ? st : check(c, hipMemcpyAsync(sl.tasks_d, sl.tasks_h, sizeof(GatherTask) * (size_t)ntask,
                                               hipMemcpyHostToDevice, sl.s));
        if (!st) {
            hipLaunchKernelGGL(gather_rows_kernel, dim3((unsigned)ntask), dim3(256), 0, sl.s, sl.tasks_d, sl.Xd,
                               (int)d);
            st = check(c, hipGetLastError());
        }
    }
    // Hashing does not read the counts: it overlaps with the batches in flight.
    int64_t ldc = rows;
    if (srv->cfg.use_graphs) {
        // One graph launch: the hash pipeline captured once per slot for a bucket of B rows
        // (multiples of 256 up to 8192, then powers of two; at most max_rows), so at most 255
        // padded rows per small batch; the batch's row count goes to n_dev.
        int64_t B = (rows + 255) / 256 * 256;
        if (B > 8192) {
            B = 16384;
            while (B < rows) B *= 2;
        }
        if (B > srv->cfg.max_rows) B = srv->cfg.max_rows;
        hipGraphExec_t ex = nullptr;
        for (auto& g : sl.graphs)
            if (g.first == B) ex = g.second;
        if (!st && !ex) {
            st = capture_hash(srv, sl, B, &ex);
            if (!st) {
                sl.graphs.push_back({B, ex});
                ++srv->graph_captures;
            }
        }
        if (!st) {
            *sl.n_host = rows;
            st = check(c, hipMemcpyAsync(sl.n_dev, sl.n_host, sizeof(int64_t), hipMemcpyHostToDevice, sl.s));
        }
        if (!st) {
            st = check(c, hipGraphLaunch(ex, sl.s));
            c->bits_hashed += (u64)rows * (u64)c->cfg.K * (u64)c->cfg.L;
            ++srv->graph_launches;
        }
        ldc = B;
    } else {
        st = st ? st : hash_chunk(c, &sl.ws, sl.Xd, rows, false, sl.s);
    }
    // Count phase, after the previous batch's count phase: one launch per run of
    // consecutive requests of one kind, in admission order.
    if (wait_cnt) st = st ? st : check(c, hipStreamWaitEvent(sl.s, wait_cnt, 0));
    size_t i = 0;
    while (!st && i < sl.reqs.size()) {
        const int kind = sl.reqs[i].kind;
        const int64_t off = sl.reqs[i].off;
        int64_t len = 0;
        for (; i < sl.reqs.size() && sl.reqs[i].kind == kind; ++i) len += sl.reqs[i].n;
        const uint16_t* codes = sl.ws.codes + off;   // table j of row r at codes[j * ldc + r]
        if (kind == ACE_REQ_INSERT || kind == ACE_REQ_DELETE)
            st = check(c, launch_count_update(codes, ldc, len, c->cfg.K, c->cfg.L, kind == ACE_REQ_INSERT ? +1 : -1,
                                              c->counts, c->cbits, c->S2, c->S3, c->err, c->rcnt + 3, sl.s));
        else
            st = check(c, launch_score(codes, ldc, len, c->cfg.K, c->cfg.L, c->counts, c->cbits, sl.sd + off,
                                       sl.Td + off,
                                       c->mom, sl.s));
    }
    st = st ? st : check(c, hipEventRecord(sl.cnt, sl.s));
    if (sl.has_score) {
        st = st ? st : check(c, hipMemcpyAsync(sl.sh, sl.sd, sizeof(float) * rows, hipMemcpyDeviceToHost, sl.s));
        st = st ? st : check(c, hipMemcpyAsync(sl.Th, sl.Td, sizeof(uint32_t) * rows, hipMemcpyDeviceToHost, sl.s));
    }
    return st ? st : check(c, hipEventRecord(sl.done, sl.s));
}

// Continuous batching: whenever a slot is free, the longest prefix of the queue that fits
// batch_rows rows (at least one request, each <= max_rows) becomes one batch.
void dispatch_loop(ace_server srv) {
    (void)hipSetDevice(srv->c->cfg.device);
    const int S = (int)srv->slots.size();
    for (;;) {
        hipEvent_t wait_cnt = nullptr;
        int idx = -1;
        int64_t rows = 0;
        ace_status prior = ACE_OK;
        {
            std::unique_lock<std::mutex> lk(srv->mu);
            srv->cv.wait(lk, [&] {
                if (srv->stop && srv->queue.empty()) return true;
                if (srv->queue.empty() || (srv->hold && !srv->stop)) return false;
                for (int k = 0; k < S; ++k)
                    if (srv->slots[(srv->next_slot + k) % S].state == SLOT_FREE) return true;
                return false;
            });
            if (srv->queue.empty()) return;   // stop requested and nothing left
            for (int k = 0; k < S && idx < 0; ++k)
                if (srv->slots[(srv->next_slot + k) % S].state == SLOT_FREE) idx = (srv->next_slot + k) % S;
            srv->next_slot = (idx + 1) % S;
            Slot& sl = srv->slots[idx];
            sl.state = SLOT_DISPATCHING;
            sl.reqs.clear();
            sl.has_score = false;
            while (!srv->queue.empty() && (rows == 0 || rows + srv->queue.front().n <= srv->cfg.batch_rows)) {
                Req q = srv->queue.front();
                srv->queue.pop_front();
                q.off = rows;
                rows += q.n;
                sl.has_score |= q.kind == ACE_REQ_SCORE;
                sl.reqs.push_back(q);
            }
            // The previous batch's slot cannot be dispatched again before this batch, so its
            // count event still marks that batch (complete already if the slot is free).
            if (srv->last_slot >= 0 && srv->last_slot != idx) wait_cnt = srv->slots[srv->last_slot].cnt;
            srv->last_slot = idx;
            prior = srv->err;
        }
        Slot& sl = srv->slots[idx];
        // After a device error every later batch completes unlaunched, with the error.
        ace_status st = prior != ACE_OK ? prior : enqueue_batch(srv, sl, rows, wait_cnt);
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            if (st != ACE_OK) {
                if (srv->err == ACE_OK) srv->err = st;
                complete_locked(srv, sl.reqs, Clock::now(), false);
                sl.state = SLOT_FREE;
            } else {
                const Clock::time_point now = Clock::now();
                for (const Req& q : sl.reqs)
                    if (q.ticket >= srv->ticket_base) srv->queue_ms[q.ticket - srv->ticket_base] = ms_between(q.t_arrive, now);
                sl.state = SLOT_BUSY;
                ++srv->busy;
                ++srv->batches;
                srv->batched_requests += (int64_t)sl.reqs.size();
                for (const Req& q : sl.reqs) srv->gathered_requests += q.gather ? 1 : 0;
            }
        }
        srv->cv.notify_all();
    }
}

void free_slot(Slot& sl) {
    for (auto& g : sl.graphs) (void)hipGraphExecDestroy(g.second);
    sl.graphs.clear();
    ws_free(&sl.ws);
    void* dev[] = {sl.Xd, sl.sd, sl.Td, sl.tasks_d, sl.n_dev};
    for (void* p : dev)
        if (p) (void)hipFree(p);
    void* host[] = {sl.Xh, sl.sh, sl.Th, sl.tasks_h, sl.n_host};
    for (void* p : host)
        if (p) (void)hipHostFree(p);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.cnt) (void)hipEventDestroy(sl.cnt);
    if (sl.s) (void)hipStreamDestroy(sl.s);
    sl = Slot();
}

ace_status alloc_slot(ace_ctx c, Slot& sl, int64_t rows) {
    const size_t d = (size_t)c->cfg.d;
    if (hipStreamCreateWithFlags(&sl.s, hipStreamNonBlocking) != hipSuccess) return ACE_E_DEVICE;
    if (hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess) return ACE_E_DEVICE;
    if (hipEventCreateWithFlags(&sl.cnt, hipEventDisableTiming) != hipSuccess) return ACE_E_DEVICE;
    ace_status st = ws_alloc(c, &sl.ws, rows);
    st = st ? st : dev_alloc(c, (void**)&sl.Xd, sizeof(float) * d * (size_t)rows);
    st = st ? st : dev_alloc(c, (void**)&sl.sd, sizeof(float) * (size_t)rows);
    st = st ? st : dev_alloc(c, (void**)&sl.Td, sizeof(uint32_t) * (size_t)rows);
    // A batch of `rows` rows made of requests of >= 1 row needs at most
    // rows / kGatherRows + (number of requests) <= rows / kGatherRows + rows tasks.
    sl.task_cap = rows / kGatherRows + rows + 1;
    st = st ? st : dev_alloc(c, (void**)&sl.tasks_d, sizeof(GatherTask) * (size_t)sl.task_cap);
    st = st ? st : dev_alloc(c, (void**)&sl.n_dev, sizeof(int64_t));
    if (st) return st;
    if (hipHostMalloc((void**)&sl.Xh, sizeof(float) * d * (size_t)rows, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&sl.sh, sizeof(float) * (size_t)rows, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&sl.Th, sizeof(uint32_t) * (size_t)rows, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&sl.tasks_h, sizeof(GatherTask) * (size_t)sl.task_cap, hipHostMallocDefault) !=
            hipSuccess ||
        hipHostMalloc((void**)&sl.n_host, sizeof(int64_t), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return ACE_E_NOMEM;
    }
    return ACE_OK;
}

// True iff [X, X + bytes) lies inside one pinned host allocation that the device reads at
// the same address, as the runtime reports it.  Only such rows go to the gather kernel;
// anything else is copied by the runtime's DMA, which checks its own source.
bool device_mapped_pinned(const float* X, size_t bytes) {
    hipPointerAttribute_t a{};
    if (hipPointerGetAttributes(&a, X) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    if (a.type != hipMemoryTypeHost || a.devicePointer != (const void*)X) return false;
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    if (hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)X) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    const uintptr_t b = reinterpret_cast<uintptr_t>(base), x = reinterpret_cast<uintptr_t>(X);
    return x >= b && bytes <= size && x - b <= size - bytes;
}

// gather: -1 = decide here (size, pinned flag and runtime check); 0 = never; 1 = the caller
// checked the rows (only the size is checked here).
ace_status submit_at(ace_server srv, int32_t kind, const float* X, int64_t n, float* s_host, uint32_t* T_host,
                     int32_t flags, Clock::time_point t_arrive, uint64_t* ticket, int gather = -1) {
    ace_ctx c = srv->c;
    if (kind != ACE_REQ_INSERT && kind != ACE_REQ_SCORE && kind != ACE_REQ_DELETE) return ACE_E_INVALID;
    if (n < 1 || n > srv->cfg.max_rows || !X) return ACE_E_INVALID;
    if (flags & ~ACE_SUBMIT_PINNED) return ACE_E_INVALID;
    std::lock_guard<std::mutex> sub(srv->submit_mu);
    std::unique_lock<std::mutex> lk(srv->mu);
    if (srv->err != ACE_OK) return srv->err;
    // n_total counts every admitted insert less every admitted delete, so the guards hold
    // for any interleaving.
    if (kind == ACE_REQ_INSERT && c->n_total + n > c->cap) return ACE_E_OVERFLOW;
    if (kind == ACE_REQ_DELETE && n > c->n_total) return ACE_E_STATE;
    if (kind == ACE_REQ_SCORE && c->cbits == 32 && (u64)c->cfg.L * (u64)c->n_total > 0xFFFFFFFFull)
        return ACE_E_OVERFLOW;
    if (c->fail_next) {
        c->fail_next = 0;
        srv->err = ACE_E_DEVICE;
        return ACE_E_DEVICE;
    }
    srv->cv.wait(lk, [&] { return srv->pending < (int64_t)kMaxPending || srv->err != ACE_OK; });
    if (srv->err != ACE_OK) return srv->err;
    const size_t bytes = sizeof(float) * (size_t)c->cfg.d * (size_t)n;
    if ((int64_t)bytes > srv->cfg.gather_max_bytes) {
        gather = 0;   // a copy moves large requests faster than the gather kernel
    } else if (gather < 0) {
        gather = 0;
        if (flags & ACE_SUBMIT_PINNED) {
            DevGuard g(c->cfg.device);
            gather = device_mapped_pinned(X, bytes) ? 1 : 0;
        }
    }
    Req q;
    q.gather = gather == 1;
    q.kind = kind;
    q.n = n;
    q.X = X;
    q.s_user = s_host;
    q.T_user = T_host;
    q.pinned = (flags & ACE_SUBMIT_PINNED) != 0;
    q.t_arrive = t_arrive;
    q.ticket = srv->next_ticket++;
    if (kind == ACE_REQ_INSERT) c->n_total += n;
    if (kind == ACE_REQ_DELETE) c->n_total -= n;
    srv->latency_ms.push_back(-1.0);
    srv->queue_ms.push_back(-1.0);
    srv->done_of.push_back(0);
    srv->kind_of.push_back((uint8_t)kind);
    srv->rows_of.push_back(n);
    if (!srv->have_first) {
        srv->have_first = true;
        srv->t_first = t_arrive;
    }
    ++srv->pending;
    srv->queue.push_back(q);
    if (ticket) *ticket = q.ticket;
    lk.unlock();
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

ace_status drain_locked(ace_server srv, std::unique_lock<std::mutex>& lk) {
    srv->cv.wait(lk, [&] { return srv->pending == 0; });
    return srv->err;
}

}  // namespace

extern "C" {

ace_status ace_server_create(ace_ctx c, const ace_server_config* cfg, ace_server* out) {
    if (!c || !cfg || !out) return ACE_E_INVALID;
    if (c->sticky != ACE_OK) return c->sticky;
    if (cfg->slots < 1 || cfg->slots > 64 || cfg->max_rows < 1 || cfg->max_rows > ((int64_t)1 << 24)) return ACE_E_INVALID;
    if (cfg->batch_rows < 0 || cfg->gather_max_bytes < -1) return ACE_E_INVALID;
    if ((cfg->use_graphs != 0 && cfg->use_graphs != 1) || cfg->reserved != 0) return ACE_E_INVALID;
    if (c->server_attached) return ACE_E_STATE;
    DevGuard g(c->cfg.device);
    ace_server srv = new ace_server_s();
    srv->c = c;
    srv->cfg = *cfg;
    if (srv->cfg.gather_max_bytes == 0) srv->cfg.gather_max_bytes = 64 * 1024;
    if (srv->cfg.batch_rows == 0 || srv->cfg.batch_rows > srv->cfg.max_rows) srv->cfg.batch_rows = (int32_t)srv->cfg.max_rows;
    srv->slots.resize(cfg->slots);
    const size_t bytes0 = c->bytes;
    ace_status st = ACE_OK;
    int got = 0;
    for (; got < cfg->slots; ++got) {
        const size_t before = c->bytes;
        st = alloc_slot(c, srv->slots[got], cfg->max_rows);
        if (st) {
            // give back what the failed slot took; keep the slots that fit
            free_slot(srv->slots[got]);
            c->bytes = before;
            break;
        }
    }
    srv->bytes = c->bytes - bytes0;
    if (got == 0 || (st && st != ACE_E_NOMEM)) {
        for (auto& sl : srv->slots) free_slot(sl);
        c->bytes = bytes0;
        delete srv;
        return st ? st : ACE_E_NOMEM;
    }
    srv->slots.resize(got);
    c->server_attached = 1;
    srv->completer = std::thread(completion_loop, srv);
    srv->dispatcher = std::thread(dispatch_loop, srv);
    *out = srv;
    return ACE_OK;
}

ace_status ace_server_submit(ace_server srv, int32_t kind, const float* X_host, int64_t n, float* s_host,
                             uint32_t* T_host, int32_t flags, uint64_t* ticket) {
    if (!srv) return ACE_E_INVALID;
    return submit_at(srv, kind, X_host, n, s_host, T_host, flags, Clock::now(), ticket);
}

ace_status ace_server_wait_for(ace_server srv, uint64_t ticket, double timeout_ms, double* latency_ms) {
    if (!srv || !(timeout_ms >= 0.0)) return ACE_E_INVALID;
    std::unique_lock<std::mutex> lk(srv->mu);
    if (ticket >= srv->next_ticket) return ACE_E_INVALID;
    auto ready = [&] { return ticket < srv->ticket_base || srv->done_of[ticket - srv->ticket_base]; };
    if (std::isinf(timeout_ms)) {
        srv->cv.wait(lk, ready);
    } else {
        const auto limit = Clock::now() + std::chrono::duration_cast<Clock::duration>(
                                              std::chrono::duration<double, std::milli>(timeout_ms));
        if (!srv->cv.wait_until(lk, limit, ready)) return ACE_E_TIMEOUT;
    }
    const bool known = ticket >= srv->ticket_base;
    if (latency_ms) *latency_ms = known ? srv->latency_ms[ticket - srv->ticket_base] : -1.0;
    if (known && srv->done_of[ticket - srv->ticket_base] == 2) return ACE_E_STATE;
    return srv->err;
}

ace_status ace_server_wait(ace_server srv, uint64_t ticket, double* latency_ms) {
    return ace_server_wait_for(srv, ticket, HUGE_VAL, latency_ms);
}

ace_status ace_server_debug_hold(ace_server srv, int32_t hold) {
    if (!srv || (hold != 0 && hold != 1)) return ACE_E_INVALID;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->hold = hold != 0;
    }
    srv->cv.notify_all();
    return ACE_OK;
}

ace_status ace_server_cancel(ace_server srv, uint64_t ticket) {
    if (!srv) return ACE_E_INVALID;
    ace_status st = ACE_E_STATE;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (ticket >= srv->next_ticket) return ACE_E_INVALID;
        for (auto it = srv->queue.begin(); it != srv->queue.end(); ++it) {
            if (it->ticket != ticket) continue;
            // Withdrawing an insert must not leave fewer points than the deletes admitted
            // since; withdrawing a delete gives its rows back (within the insert cap).
            if (it->kind == ACE_REQ_INSERT && srv->c->n_total < it->n) break;
            if (it->kind == ACE_REQ_DELETE && srv->c->n_total + it->n > srv->c->cap) break;
            if (it->kind == ACE_REQ_INSERT) srv->c->n_total -= it->n;
            if (it->kind == ACE_REQ_DELETE) srv->c->n_total += it->n;
            if (ticket >= srv->ticket_base) {
                const size_t i = ticket - srv->ticket_base;
                srv->done_of[i] = 2;
                srv->latency_ms[i] = -1.0;
            }
            srv->queue.erase(it);
            --srv->pending;
            ++srv->cancelled;
            st = ACE_OK;
            break;
        }
    }
    if (st == ACE_OK) srv->cv.notify_all();
    return st;
}

ace_status ace_server_drain(ace_server srv) {
    if (!srv) return ACE_E_INVALID;
    std::lock_guard<std::mutex> sub(srv->submit_mu);
    std::unique_lock<std::mutex> lk(srv->mu);
    return drain_locked(srv, lk);
}

ace_status ace_server_replay(ace_server srv, const ace_request* reqs, int64_t nreq, const float* pool,
                             int64_t pool_rows, int32_t flags, float* s_out, uint32_t* T_out, double* latency_ms) {
    if (!srv || nreq < 0 || (nreq > 0 && (!reqs || !pool))) return ACE_E_INVALID;
    if (pool_rows < 0 || (flags & ~ACE_SUBMIT_PINNED)) return ACE_E_INVALID;
    for (int64_t r = 0; r < nreq; ++r) {
        const ace_request& q = reqs[r];
        if (q.kind != ACE_REQ_INSERT && q.kind != ACE_REQ_SCORE && q.kind != ACE_REQ_DELETE) return ACE_E_INVALID;
        if (q.n < 1 || q.n > srv->cfg.max_rows || q.row0 < 0 || q.row0 > pool_rows - q.n) return ACE_E_INVALID;
        if (!(q.t_arrival_s >= 0)) return ACE_E_INVALID;
        if (q.kind == ACE_REQ_SCORE && (s_out || T_out) && q.out0 < 0) return ACE_E_INVALID;
    }
    const size_t d = (size_t)srv->c->cfg.d;
    int gather = 0;
    if ((flags & ACE_SUBMIT_PINNED) && nreq > 0) {
        DevGuard g(srv->c->cfg.device);
        gather = device_mapped_pinned(pool, sizeof(float) * d * (size_t)pool_rows) ? 1 : 0;
    }
    std::vector<uint64_t> tickets((size_t)nreq);
    const Clock::time_point t0 = Clock::now();
    ace_status st = ACE_OK;
    for (int64_t r = 0; r < nreq && !st; ++r) {
        const ace_request& q = reqs[r];
        Clock::time_point ta = Clock::now();
        if (q.t_arrival_s > 0) {
            ta = t0 + std::chrono::duration_cast<Clock::duration>(std::chrono::duration<double>(q.t_arrival_s));
            while (Clock::now() < ta) std::this_thread::yield();
        }
        float* so = (q.kind == ACE_REQ_SCORE && s_out) ? s_out + q.out0 : nullptr;
        uint32_t* To = (q.kind == ACE_REQ_SCORE && T_out) ? T_out + q.out0 : nullptr;
        st = submit_at(srv, q.kind, pool + (size_t)q.row0 * d, q.n, so, To, flags, ta, &tickets[r], gather);
    }
    const ace_status st2 = ace_server_drain(srv);
    if (latency_ms) {
        std::lock_guard<std::mutex> lk(srv->mu);
        for (int64_t r = 0; r < nreq; ++r)
            latency_ms[r] = tickets[r] >= srv->ticket_base && tickets[r] < srv->next_ticket
                                ? srv->latency_ms[tickets[r] - srv->ticket_base]
                                : -1.0;
    }
    return st ? st : st2;
}

ace_status ace_server_get_stats(ace_server srv, ace_server_stats* out) {
    if (!srv || !out) return ACE_E_INVALID;
    std::lock_guard<std::mutex> lk(srv->mu);
    ace_server_stats s{};
    std::vector<double> all, ins, sco, del, qw;
    for (size_t i = 0; i < srv->latency_ms.size(); ++i) {
        if (!srv->done_of[i] || srv->latency_ms[i] < 0) continue;
        const double v = srv->latency_ms[i];
        all.push_back(v);
        qw.push_back(srv->queue_ms[i]);
        const int k = srv->kind_of[i];
        (k == ACE_REQ_INSERT ? ins : k == ACE_REQ_DELETE ? del : sco).push_back(v);
        s.rows += srv->rows_of[i];
        if (k == ACE_REQ_INSERT) s.insert_rows += srv->rows_of[i];
        if (k == ACE_REQ_DELETE) s.delete_rows += srv->rows_of[i];
    }
    s.requests = (int64_t)all.size();
    s.inserts = (int64_t)ins.size();
    s.scores = (int64_t)sco.size();
    s.deletes = (int64_t)del.size();
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
    s.p99_delete_ms = percentile(del, 99.0);
    s.wall_ms = srv->have_first ? ms_between(srv->t_first, srv->t_last) : 0.0;
    s.batches = srv->batches;
    s.mean_batch_requests = srv->batches ? (double)srv->batched_requests / (double)srv->batches : 0.0;
    s.gathered_requests = srv->gathered_requests;
    s.graph_launches = srv->graph_launches;
    s.graph_captures = srv->graph_captures;
    s.slots = (int64_t)srv->slots.size();
    s.cancelled = srv->cancelled;
    s.p50_queue_ms = percentile(qw, 50.0);
    s.p99_queue_ms = percentile(qw, 99.0);
    *out = s;
    return ACE_OK;
}

ace_status ace_server_reset_stats(ace_server srv) {
    if (!srv) return ACE_E_INVALID;
    std::lock_guard<std::mutex> sub(srv->submit_mu);
    std::unique_lock<std::mutex> lk(srv->mu);
    (void)drain_locked(srv, lk);
    srv->ticket_base = srv->next_ticket;
    srv->latency_ms.clear();
    srv->queue_ms.clear();
    srv->done_of.clear();
    srv->kind_of.clear();
    srv->rows_of.clear();
    srv->batches = srv->batched_requests = srv->gathered_requests = srv->graph_launches = srv->cancelled = 0;
    srv->have_first = false;
    return ACE_OK;
}

ace_status ace_server_destroy(ace_server srv) {
    if (!srv) return ACE_E_INVALID;
    (void)ace_server_debug_hold(srv, 0);
    (void)ace_server_drain(srv);
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
    }
    srv->cv.notify_all();
    srv->dispatcher.join();
    srv->completer.join();
    DevGuard g(srv->c->cfg.device);
    for (auto& sl : srv->slots) {
        (void)hipStreamSynchronize(sl.s);
        free_slot(sl);
    }
    srv->c->bytes -= srv->bytes;
    srv->c->server_attached = 0;
    delete srv;
    return ACE_OK;
}

}  // extern "C"
