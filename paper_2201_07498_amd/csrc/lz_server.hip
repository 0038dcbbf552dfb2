// Serving runtime: continuous batching of Top-K solves on one GPU.
//
// One worker thread per slot.  Requests wait in a FIFO queue; a request
// is admitted when one of max_slots slots is free and its footprint (CSR,
// solver workspace, outputs) can be carved out of a fixed HBM arena
// (first-fit, coalescing free list), so no device allocation happens while
// serving.  The first few queued requests may be admitted out of order when
// the head does not fit (bounded backfill; a head bypassed too often blocks
// backfill until it is admitted).  Each slot has its own HIP stream; an
// admitted request's copies and kernels are enqueued there, so requests of
// different sizes and precisions run concurrently on the device.  The Lanczos
// iterations of a request can be captured in a hipGraph and replayed.  A
// slot's thread advances it through a small state machine, waiting on events:
//   ADMIT:   H2D of the CSR, setup, start vector, m iterations, D2H of state
//   LANCZOS: restart check (more iterations if breakdowns consumed some),
//            then Jacobi, selection, Ritz vectors, report, D2H of results
//   FINISH:  results to the caller, arena block and slot released.
// Launch shapes depend only on the request, so a request's results are the
// same alone and in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <exception>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/lanczos_topk.h"
#include "lz_internal.h"

namespace lz {
namespace {

constexpr size_t ALIGN = 256;
constexpr int BACKFILL = 8;          // queued requests considered per admission
constexpr int MAX_BYPASS = 32;       // then the head is admitted first
constexpr int MAX_RESTART_ROUNDS = 2 * MMAX + 2;

size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

// First-fit allocator over one device allocation.
class Arena {
   public:
    bool init(size_t bytes) {
        bytes = align_up(bytes);
        if (hipMalloc(&base_, bytes) != hipSuccess) return false;
        size_ = bytes;
        free_[0] = bytes;
        return true;
    }
    void destroy() {
        if (base_) (void)hipFree(base_);
        base_ = nullptr;
    }
    bool alloc(size_t bytes, size_t* off) {
        bytes = align_up(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const size_t o = it->first, rem = it->second - bytes;
            free_.erase(it);
            if (rem) free_[o + bytes] = rem;
            *off = o;
            in_use_ += bytes;
            peak_ = std::max(peak_, in_use_);
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = align_up(bytes);
        in_use_ -= bytes;
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
    char* base() const { return (char*)base_; }
    size_t size() const { return size_; }
    size_t in_use() const { return in_use_; }
    size_t peak() const { return peak_; }

   private:
    void* base_ = nullptr;
    size_t size_ = 0, in_use_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;
};

// Placement of one request inside its arena block.
struct Layout {
    size_t rowptr = 0, col = 0, val = 0, ws = 0, vals = 0, vecs = 0, total = 0;
};

Layout layout_of(const Plan& p) {
    Layout l;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    l.rowptr = take((size_t)(p.n + 1) * 8);
    l.col = take((size_t)p.nnz * 4);
    l.val = take((size_t)p.nnz * storage_bytes(p.prec));
    l.ws = take(p.bytes);
    l.vals = take((size_t)p.K * 8);
    l.vecs = take((size_t)p.n * p.K * 8);
    l.total = o;
    return l;
}

struct Req {
    uint64_t ticket = 0;
    lz_request r{};
    Plan plan;
    Layout lay;
    int status = LZ_PENDING;
    lz_result res{};
    int bypassed = 0;
};

enum Phase { IDLE = 0, LANCZOS = 1, FINISH = 2 };

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t ev_start = nullptr, ev_phase = nullptr;
    State* hstate = nullptr;      // pinned copy of the device state
    double* hvals = nullptr;      // pinned eigenvalues
    Req* req = nullptr;
    Phase phase = IDLE;
    size_t off = 0;
    Bufs bufs{};
    Csr csr{};
    double* dvals = nullptr;
    double* dvecs = nullptr;
    hipGraphExec_t gexec = nullptr;
    int rounds = 0;
};

}  // namespace

struct Server {
    int device = 0;
    bool use_graphs = false;
    Arena arena;
    std::vector<Slot> slots;
    std::mutex mu;
    std::condition_variable cv, done_cv;
    std::deque<Req*> queue;
    std::unordered_map<uint64_t, std::unique_ptr<Req>> reqs;
    std::vector<std::thread> workers;
    bool stop = false;
    uint64_t next_ticket = 1;
    uint64_t submitted = 0, completed = 0, rejected = 0;
    int active = 0;
    double enqueue_ms = 0.0;     // worker threads' time in admit / advance (read under mu)
    std::chrono::steady_clock::time_point t0;

    double now_ms() const {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    void add_enqueue_time(std::chrono::steady_clock::time_point since) {
        const double ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - since).count();
        std::lock_guard<std::mutex> lk(mu);
        enqueue_ms += ms;
    }
    void run_slot(Slot& s);
    Req* pick(Slot& s);
    bool admit(Slot& s, Req* q);
    void advance(Slot& s);
    void complete(Slot& s, int status);
    hipError_t launch_lanczos(Slot& s);
};

hipError_t Server::launch_lanczos(Slot& s) {
    const Plan& p = s.req->plan;
    const lz_request& r = s.req->r;
    auto body = [&]() -> hipError_t {
        hipError_t e = launch_setup(p, s.bufs, s.csr, r.seed, r.reorth, LZ_REORDER_AUTO, s.stream);
        if (e == hipSuccess) e = launch_init(p, s.bufs, s.stream);
        for (int t = 0; t < p.m && e == hipSuccess; ++t)
            e = launch_iteration(p, s.bufs, s.csr, t + 1, r.reorth, s.stream);
        return e;
    };
    if (!use_graphs) return body();
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(s.stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    const hipError_t eb = body();
    e = hipStreamEndCapture(s.stream, &g);
    if (eb != hipSuccess) e = eb;
    if (e == hipSuccess) e = hipGraphInstantiate(&s.gexec, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (e == hipSuccess) e = hipGraphLaunch(s.gexec, s.stream);
    return e;
}

bool Server::admit(Slot& s, Req* q) {
    s.req = q;
    s.rounds = 0;
    char* base = arena.base() + s.off;
    const Layout& l = q->lay;
    const lz_request& r = q->r;
    const size_t vb = storage_bytes(r.precision);
    s.csr = Csr{(const int64_t*)(base + l.rowptr), (const int32_t*)(base + l.col), base + l.val, r.n, r.nnz};
    s.bufs = resolve(q->plan, base + l.ws);
    s.dvals = (double*)(base + l.vals);
    s.dvecs = (double*)(base + l.vecs);
    q->res.t_admit_ms = now_ms();
    hipError_t e = hipEventRecord(s.ev_start, s.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(base + l.rowptr, r.rowptr, (size_t)(r.n + 1) * 8, hipMemcpyHostToDevice, s.stream);
    if (e == hipSuccess && r.nnz > 0) e = hipMemcpyAsync(base + l.col, r.col, (size_t)r.nnz * 4, hipMemcpyHostToDevice, s.stream);
    if (e == hipSuccess && r.nnz > 0) e = hipMemcpyAsync(base + l.val, r.val, (size_t)r.nnz * vb, hipMemcpyHostToDevice, s.stream);
    if (e == hipSuccess) e = launch_lanczos(s);
    if (e == hipSuccess) e = hipMemcpyAsync(s.hstate, s.bufs.st, STATE_REPORT_BYTES, hipMemcpyDeviceToHost, s.stream);
    if (e == hipSuccess) e = hipEventRecord(s.ev_phase, s.stream);
    s.phase = LANCZOS;
    return e == hipSuccess;
}

void Server::complete(Slot& s, int status) {
    Req* q = s.req;
    (void)hipStreamSynchronize(s.stream);
    float ms = 0.f;
    if (status == LZ_OK && hipEventElapsedTime(&ms, s.ev_start, s.ev_phase) == hipSuccess) q->res.device_ms = ms;
    if (s.gexec) {
        (void)hipGraphExecDestroy(s.gexec);
        s.gexec = nullptr;
    }
    if (status == LZ_OK) {
        const State* st = s.hstate;
        std::memcpy(q->r.out_vals, s.hvals, sizeof(double) * q->r.K);
        q->res.m_eff = std::min(st->j, q->r.m);
        q->res.restarts = st->restarts;
        double rm = 0.0;
        for (int k = 0; k < q->r.K; ++k) rm = std::max(rm, st->resid[k]);
        if (q->r.out_resid) std::memcpy(q->r.out_resid, st->resid, sizeof(double) * q->r.K);
        q->res.resid_max = rm;
        q->res.ortho_loss = st->ortho_loss;
    }
    q->res.status = status;
    q->res.t_done_ms = now_ms();
    {
        std::lock_guard<std::mutex> lk(mu);
        arena.release(s.off, q->lay.total);
        q->status = status;
        ++completed;
        --active;
    }
    s.req = nullptr;
    s.phase = IDLE;
    done_cv.notify_all();
    cv.notify_all();                  // the freed arena block may let a waiting request in
}

void Server::advance(Slot& s) {
    Req* q = s.req;
    const Plan& p = q->plan;
    const State* st = s.hstate;
    if (s.phase == LANCZOS) {
        if (st->status != 0) return complete(s, st->status);
        if (st->j < p.m) {              // breakdowns consumed iterations: run more
            if (++s.rounds > MAX_RESTART_ROUNDS) return complete(s, LZ_ERR_BREAKDOWN);
            hipError_t e = hipSuccess;
            for (int t = st->j; t < p.m && e == hipSuccess; ++t)
                e = launch_iteration(p, s.bufs, s.csr, p.m, q->r.reorth, s.stream);
            if (e == hipSuccess) e = hipMemcpyAsync(s.hstate, s.bufs.st, STATE_REPORT_BYTES, hipMemcpyDeviceToHost, s.stream);
            if (e == hipSuccess) e = hipEventRecord(s.ev_phase, s.stream);
            if (e != hipSuccess) complete(s, LZ_ERR_HIP);
            return;
        }
        hipError_t e = launch_finish(p, s.bufs, s.csr, s.dvals, s.dvecs, 1, s.stream);
        if (e == hipSuccess) e = hipMemcpyAsync(s.hvals, s.dvals, sizeof(double) * p.K, hipMemcpyDeviceToHost, s.stream);
        if (e == hipSuccess && q->r.out_vecs)
            e = hipMemcpyAsync(q->r.out_vecs, s.dvecs, sizeof(double) * p.n * p.K, hipMemcpyDeviceToHost, s.stream);
        if (e == hipSuccess) e = hipMemcpyAsync(s.hstate, s.bufs.st, STATE_REPORT_BYTES, hipMemcpyDeviceToHost, s.stream);
        if (e == hipSuccess) e = hipEventRecord(s.ev_phase, s.stream);
        if (e != hipSuccess) return complete(s, LZ_ERR_HIP);
        s.phase = FINISH;
        return;
    }
    if (s.phase == FINISH) complete(s, st->status);
}

// The first queued request (within the backfill window) whose footprint
// fits the arena, taken off the queue; null if none.  Called under mu.
Req* Server::pick(Slot& s) {
    const int look = std::min<int>(BACKFILL, (int)queue.size());
    for (int i = 0; i < look; ++i) {
        if (i > 0 && queue.front()->bypassed >= MAX_BYPASS) break;
        Req* q = queue[i];
        size_t off = 0;
        if (!arena.alloc(q->lay.total, &off)) continue;
        s.off = off;
        for (int k = 0; k < i; ++k) queue[k]->bypassed++;
        queue.erase(queue.begin() + i);
        ++active;
        return q;
    }
    return nullptr;
}

// One worker thread per slot: it admits a request when its slot is free,
// sleeps on the slot's phase event (created with blocking sync) while the
// device works, and advances the slot when the event has completed.  The
// queue, the arena and the counters are shared under mu; every thread
// enqueues its own slot's copies and launches, so the host-side cost of
// capture and launch is spread over the threads.
void Server::run_slot(Slot& s) {
    (void)hipSetDevice(device);
    for (;;) {
        if (s.phase == IDLE) {
            Req* q = nullptr;
            {
                std::unique_lock<std::mutex> lk(mu);
                for (;;) {
                    q = pick(s);
                    if (q || (stop && queue.empty())) break;
                    cv.wait(lk);
                }
            }
            if (!q) return;
            q->res.slot = (int)(&s - slots.data());
            const auto t0 = std::chrono::steady_clock::now();
            if (!admit(s, q)) complete(s, LZ_ERR_HIP);
            add_enqueue_time(t0);
            continue;
        }
        const hipError_t e = hipEventSynchronize(s.ev_phase);
        const auto t0 = std::chrono::steady_clock::now();
        if (e != hipSuccess)
            complete(s, LZ_ERR_HIP);
        else
            advance(s);
        add_enqueue_time(t0);
    }
}

}  // namespace lz

using namespace lz;

static int check_request(const lz_request* r) {
    if (!r || !r->rowptr || !r->out_vals) return LZ_ERR_INVALID_ARG;
    if (r->nnz > 0 && (!r->col || !r->val)) return LZ_ERR_INVALID_ARG;
    if (r->n < 1 || r->n >= (int64_t(1) << 31) || r->nnz < 0 || r->nnz >= (int64_t(1) << 40)) return LZ_ERR_INVALID_ARG;
    if (r->precision < LZ_FP64 || r->precision > LZ_BF16) return LZ_ERR_INVALID_ARG;
    if (r->K < 1 || r->m < r->K || r->m > LZ_MAX_STEPS || (int64_t)r->m > r->n) return LZ_ERR_INVALID_ARG;
    if (r->reorth < LZ_REORTH_NONE || r->reorth > LZ_REORTH_SELECTIVE) return LZ_ERR_INVALID_ARG;
    return LZ_OK;
}

extern "C" {

size_t lz_request_footprint(int64_t n, int64_t nnz, int32_t K, int32_t m, int32_t precision) {
    if (n < 1 || nnz < 0 || K < 1 || m < K || m > LZ_MAX_STEPS || precision < 0 || precision > 2) return 0;
    return layout_of(make_plan(n, nnz, K, m, precision)).total;
}

int lz_server_create(int device, size_t hbm_budget_bytes, int32_t max_slots, int32_t use_graphs, lz_server** out) {
    if (!out || max_slots < 1 || max_slots > 64 || hbm_budget_bytes < ALIGN) return LZ_ERR_INVALID_ARG;
    *out = nullptr;
    if (hipSetDevice(device) != hipSuccess) return LZ_ERR_HIP;
    auto* s = new Server;
    s->device = device;
    s->use_graphs = use_graphs != 0;
    s->t0 = std::chrono::steady_clock::now();
    if (!s->arena.init(hbm_budget_bytes)) {
        delete s;
        return LZ_ERR_OUT_OF_MEMORY;
    }
    s->slots.resize(max_slots);
    for (Slot& sl : s->slots) {
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreate(&sl.ev_start) != hipSuccess ||
            hipEventCreateWithFlags(&sl.ev_phase, hipEventBlockingSync) != hipSuccess ||
            hipHostMalloc((void**)&sl.hstate, sizeof(State), hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void**)&sl.hvals, sizeof(double) * MMAX, hipHostMallocDefault) != hipSuccess) {
            lz_server_destroy((lz_server*)s);
            return LZ_ERR_HIP;
        }
    }
    // One thread per slot.  If the system refuses a thread, the ones already
    // started find the queue empty and stopped, and return.
    try {
        s->workers.reserve(s->slots.size());
        for (Slot& sl : s->slots) s->workers.emplace_back([s, &sl] { s->run_slot(sl); });
    } catch (const std::exception&) {
        lz_server_destroy((lz_server*)s);
        return LZ_ERR_OUT_OF_MEMORY;
    }
    *out = (lz_server*)s;
    return LZ_OK;
}

int lz_server_submit(lz_server* srv, const lz_request* req, uint64_t* ticket) {
    auto* s = (Server*)srv;
    if (!s || !ticket) return LZ_ERR_INVALID_ARG;
    const int rc = check_request(req);
    if (rc != LZ_OK) return rc;
    auto q = std::make_unique<Req>();
    q->r = *req;
    q->plan = make_plan(req->n, req->nnz, req->K, req->m, req->precision);
    // The SpMV variant is fixed when the graph is captured: take the device's
    // relabelling decision on the host, from the caller's row pointer.
    if (!q->plan.sweep && want_xcache(q->plan, true))
        q->plan.xcache = want_xcache(q->plan, host_relabel_decision(req->rowptr, req->n, req->nnz, LZ_REORDER_AUTO));
    q->lay = layout_of(q->plan);
    std::lock_guard<std::mutex> lk(s->mu);
    if (q->lay.total > s->arena.size()) {
        ++s->rejected;
        return LZ_ERR_TOO_LARGE;
    }
    q->ticket = s->next_ticket++;
    q->res.t_submit_ms = s->now_ms();
    q->res.status = LZ_PENDING;
    q->res.slot = -1;
    *ticket = q->ticket;
    s->queue.push_back(q.get());
    s->reqs.emplace(q->ticket, std::move(q));
    ++s->submitted;
    s->cv.notify_one();
    return LZ_OK;
}

int lz_server_poll(lz_server* srv, uint64_t ticket, lz_result* res) {
    auto* s = (Server*)srv;
    if (!s) return LZ_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return LZ_ERR_INVALID_ARG;
    if (it->second->status == LZ_PENDING) return LZ_PENDING;
    if (res) *res = it->second->res;
    return it->second->status;
}

int lz_server_wait(lz_server* srv, uint64_t ticket, lz_result* res) {
    auto* s = (Server*)srv;
    if (!s) return LZ_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return LZ_ERR_INVALID_ARG;
    Req* q = it->second.get();
    s->done_cv.wait(lk, [q] { return q->status != LZ_PENDING; });
    if (res) *res = q->res;
    return q->status;
}

int lz_server_get_stats(lz_server* srv, lz_server_stats* out) {
    auto* s = (Server*)srv;
    if (!s || !out) return LZ_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    out->submitted = s->submitted;
    out->completed = s->completed;
    out->rejected = s->rejected;
    out->active = (uint64_t)s->active;
    out->queued = s->queue.size();
    out->arena_bytes = s->arena.size();
    out->arena_in_use = s->arena.in_use();
    out->arena_peak = s->arena.peak();
    out->worker_enqueue_ms = s->enqueue_ms;
    return LZ_OK;
}

int lz_server_destroy(lz_server* srv) {
    auto* s = (Server*)srv;
    if (!s) return LZ_ERR_INVALID_ARG;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    for (std::thread& w : s->workers)
        if (w.joinable()) w.join();
    for (Slot& sl : s->slots) {
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.ev_start) (void)hipEventDestroy(sl.ev_start);
        if (sl.ev_phase) (void)hipEventDestroy(sl.ev_phase);
        if (sl.hstate) (void)hipHostFree(sl.hstate);
        if (sl.hvals) (void)hipHostFree(sl.hvals);
    }
    s->arena.destroy();
    delete s;
    return LZ_OK;
}

}  // extern "C"
