// Serving scheduler: a stream of independent compression and decompression
// requests (the in-situ setting of Sec. 1-2, where a running simulation hands
// each quantity to the compressor as it is produced) served by continuous
// batching with admission against a device-memory budget.
//
// A worker thread owns SLOTS launch slots.  Whenever a slot is free it takes
// requests from the head of the arrival FIFO, in order, while the number of
// admitted-but-unfinished requests stays within max_inflight and their device
// footprint within the budget, and launches them as one batch: requests are
// grouped by kernel class exactly as cz_compress_batch does, compressions and
// decompressions on two streams of the slot.  Requests that arrive while
// batches run wait for the next free slot, so the batch size follows the load.
// A request is complete when its slot's batch has finished; its status comes
// from its own per-field status word.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "cz_host.h"

namespace {

using Clock = std::chrono::steady_clock;
constexpr int SLOTS = 4;
constexpr int MAX_BATCH = 1024;

struct Req {
    cz_request r{};
    uint64_t foot = 0;  // device bytes the request reads and writes
    double t_arrive = 0, t_admit = -1, t_done = -1;
    int status = CZ_OK;
    size_t out_bytes = 0;
    bool done = false;
};

// One direction of a launch: its requests in field order and the arrays the
// batch machinery takes.
struct Part {
    std::vector<uint64_t> ids;
    std::vector<cz_params> ps;
    std::vector<const void *> srcs;
    std::vector<size_t> src_bytes;
    std::vector<void *> dsts;
    std::vector<size_t> caps;
    czh::Layout layout;
    void clear()
    {
        ids.clear();
        ps.clear();
        srcs.clear();
        src_bytes.clear();
        dsts.clear();
        caps.clear();
        layout = czh::Layout();
    }
};

struct Slot {
    hipStream_t st[2] = {};
    hipEvent_t ev[2] = {};
    czh::BatchWork work[2];
    Part part[2];
    bool busy = false;
};

}  // namespace

struct cz_server {
    cz_ctx *ctx = nullptr;
    size_t budget = 0;
    int max_inflight = 1;
    Clock::time_point t0;
    std::mutex m;
    std::condition_variable cv;
    std::deque<Req> reqs;        // by ticket (deque: references stay valid as it grows)
    std::deque<uint64_t> fifo;   // submitted, not yet admitted
    size_t inflight_bytes = 0;
    int inflight = 0;
    bool stopping = false;
    int fatal = CZ_OK;
    Slot slots[SLOTS];
    std::thread worker;

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

namespace {

uint64_t raw_bytes(const cz_params &p) { return (uint64_t)p.nx * p.ny * p.nz * p.elem_bytes; }

// Validate a request; on success its footprint.
int check_request(const cz_request *r, uint64_t *foot)
{
    if (!r || (r->op != 0 && r->op != 1))
        return CZ_ERR_ARG;
    uint64_t nb = 0;
    int rc = czh::check_params(&r->p, &nb);
    if (rc != CZ_OK)
        return rc;
    const uint64_t raw = raw_bytes(r->p);
    if (r->op == 0) {
        const uint64_t bound = czh::bound_of(r->p, nb);
        if (r->dst_cap < bound)
            return CZ_ERR_CAPACITY;
        if (!r->d_dst || (nb && !r->d_src))
            return CZ_ERR_ARG;
        *foot = raw + bound;
    } else {
        if (!r->d_src || r->src_bytes < czh::payload_start(nb))
            return CZ_ERR_FORMAT;
        if (r->dst_cap < raw)
            return CZ_ERR_CAPACITY;
        if (nb && !r->d_dst)
            return CZ_ERR_ARG;
        *foot = r->src_bytes + raw;
    }
    return CZ_OK;
}

// Launch the gathered parts of a slot.  Returns a CZ_* code.
int launch_slot(cz_server *s, Slot &sl)
{
    for (int d = 0; d < 2; ++d) {
        Part &pt = sl.part[d];
        if (!pt.ids.empty()) {
            const int n = (int)pt.ids.size();
            int rc = czh::layout_batch(s->ctx, d == 0, n, pt.ps.data(), &pt.layout);
            if (rc == CZ_OK)
                rc = czh::size_work(sl.work[d], pt.layout);
            if (rc != CZ_OK)
                return rc;
            czh::stage_batch(sl.work[d], pt.layout, pt.ps.data(), pt.srcs.data(), pt.src_bytes.data(),
                             pt.dsts.data());
            // (the enqueue also copies stream sizes and per-field status to pinned memory)
            if ((rc = czh::enqueue_batch(sl.work[d], pt.layout, nullptr, true, sl.st[d])) != CZ_OK)
                return rc;
        }
        if (hipEventRecord(sl.ev[d], sl.st[d]) != hipSuccess)
            return CZ_ERR_HIP;
    }
    return CZ_OK;
}

// Mark the requests of a finished (or failed) slot done.  Caller holds s->m.
void finish_slot(cz_server *s, Slot &sl, int err)
{
    const double t = s->now();
    for (int d = 0; d < 2; ++d) {
        Part &pt = sl.part[d];
        const czh::Layout &L = pt.layout;
        for (size_t pos = 0; pos < pt.ids.size(); ++pos) {
            // per-field status words are in class order; map back to the field
            const int i = err == CZ_OK ? L.order[pos] : (int)pos;
            Req &q = s->reqs[pt.ids[i]];
            q.status = err != CZ_OK ? err : czh::status_to_error(sl.work[d].fstat_host[pos]);
            q.out_bytes = (d == 0 && err == CZ_OK) ? (size_t)sl.work[d].totals_host[i] : 0;
            q.t_done = t;
            q.done = true;
            s->inflight_bytes -= q.foot;
            s->inflight -= 1;
        }
        pt.clear();
    }
    sl.busy = false;
}

void worker_main(cz_server *s)
{
    (void)hipSetDevice(s->ctx->device);
    while (true) {
        bool progressed = false;
        // completions
        for (Slot &sl : s->slots) {
            if (!sl.busy)
                continue;
            const hipError_t e0 = hipEventQuery(sl.ev[0]);
            const hipError_t e1 = hipEventQuery(sl.ev[1]);
            if (e0 == hipErrorNotReady || e1 == hipErrorNotReady)
                continue;
            std::lock_guard<std::mutex> lk(s->m);
            const int err = (e0 == hipSuccess && e1 == hipSuccess) ? CZ_OK : CZ_ERR_HIP;
            if (err != CZ_OK)
                s->fatal = err;
            finish_slot(s, sl, err);
            progressed = true;
        }
        if (progressed)
            s->cv.notify_all();
        // admissions: strict FIFO, one batch per free slot
        for (Slot &sl : s->slots) {
            if (sl.busy)
                continue;
            {
                std::lock_guard<std::mutex> lk(s->m);
                int taken = 0;
                const double t = s->now();
                while (!s->fifo.empty() && taken < MAX_BATCH && s->inflight < s->max_inflight &&
                       s->fatal == CZ_OK) {
                    Req &q = s->reqs[s->fifo.front()];
                    if (s->inflight_bytes + q.foot > s->budget)
                        break;
                    Part &pt = sl.part[q.r.op];
                    pt.ids.push_back(s->fifo.front());
                    pt.ps.push_back(q.r.p);
                    pt.srcs.push_back(q.r.d_src);
                    pt.src_bytes.push_back(q.r.src_bytes);
                    pt.dsts.push_back(q.r.d_dst);
                    pt.caps.push_back(q.r.dst_cap);
                    q.t_admit = t;
                    s->inflight += 1;
                    s->inflight_bytes += q.foot;
                    s->fifo.pop_front();
                    ++taken;
                }
                if (!taken)
                    break;
                sl.busy = true;
            }
            const int rc = launch_slot(s, sl);
            if (rc != CZ_OK) {
                (void)hipStreamSynchronize(sl.st[0]);
                (void)hipStreamSynchronize(sl.st[1]);
                std::lock_guard<std::mutex> lk(s->m);
                if (rc == CZ_ERR_HIP)
                    s->fatal = rc;
                finish_slot(s, sl, rc);
                s->cv.notify_all();
            }
            progressed = true;
        }
        std::unique_lock<std::mutex> lk(s->m);
        bool busy = false;
        for (Slot &sl : s->slots)
            busy |= sl.busy;
        if (s->stopping && s->fifo.empty() && !busy)
            break;
        if (!progressed) {
            if (!busy) {
                // nothing on the device: sleep until a request arrives or stop
                s->cv.wait(lk, [s] { return s->stopping || !s->fifo.empty(); });
                if (s->fatal != CZ_OK) {
                    // the device failed: fail whatever is still queued
                    while (!s->fifo.empty()) {
                        Req &q = s->reqs[s->fifo.front()];
                        q.status = s->fatal;
                        q.t_done = s->now();
                        q.done = true;
                        s->fifo.pop_front();
                    }
                    s->cv.notify_all();
                }
            } else {
                lk.unlock();
                std::this_thread::yield();  // batches in flight: poll their events
            }
        }
    }
}

void destroy_slots(cz_server *s)
{
    for (Slot &sl : s->slots) {
        for (int d = 0; d < 2; ++d) {
            if (sl.st[d])
                (void)hipStreamSynchronize(sl.st[d]);
            sl.work[d].release();
            if (sl.ev[d])
                (void)hipEventDestroy(sl.ev[d]);
            if (sl.st[d])
                (void)hipStreamDestroy(sl.st[d]);
        }
    }
}

}  // namespace

extern "C" {

int cz_server_start(cz_ctx *ctx, size_t hbm_budget_bytes, int max_inflight, cz_server **out)
{
    if (!ctx || !out || max_inflight < 1 || hbm_budget_bytes == 0)
        return CZ_ERR_ARG;
    *out = nullptr;
    czh::DeviceGuard guard(ctx->device);
    cz_server *s = new (std::nothrow) cz_server();
    if (!s)
        return CZ_ERR_ARG;
    s->ctx = ctx;
    s->budget = hbm_budget_bytes;
    s->max_inflight = max_inflight;
    s->t0 = Clock::now();
    bool ok = true;
    for (Slot &sl : s->slots)
        for (int d = 0; d < 2 && ok; ++d)
            ok = hipStreamCreateWithFlags(&sl.st[d], hipStreamNonBlocking) == hipSuccess &&
                 hipEventCreateWithFlags(&sl.ev[d], hipEventDisableTiming) == hipSuccess &&
                 sl.work[d].init() == CZ_OK;
    if (!ok) {
        destroy_slots(s);
        delete s;
        return CZ_ERR_HIP;
    }
    try {
        s->worker = std::thread(worker_main, s);
    } catch (...) {
        destroy_slots(s);
        delete s;
        return CZ_ERR_ARG;
    }
    *out = s;
    return CZ_OK;
}

double cz_server_time(cz_server *s) { return s ? s->now() : -1.0; }

int cz_submit(cz_server *s, const cz_request *r, uint64_t *ticket)
{
    if (!s || !ticket)
        return CZ_ERR_ARG;
    uint64_t foot = 0;
    int rc = check_request(r, &foot);
    if (rc != CZ_OK)
        return rc;
    if (foot > s->budget)
        return CZ_ERR_BUDGET;
    {
        std::lock_guard<std::mutex> lk(s->m);
        if (s->stopping)
            return CZ_ERR_ARG;
        if (s->fatal != CZ_OK)
            return s->fatal;
        Req q;
        q.r = *r;
        q.foot = foot;
        q.t_arrive = s->now();
        *ticket = s->reqs.size();
        s->reqs.push_back(q);
        s->fifo.push_back(*ticket);
    }
    s->cv.notify_all();
    return CZ_OK;
}

int cz_poll(cz_server *s, uint64_t ticket, int *done, int *status, size_t *out_bytes, double *t_arrive,
            double *t_admit, double *t_done)
{
    if (!s || !done)
        return CZ_ERR_ARG;
    std::lock_guard<std::mutex> lk(s->m);
    if (ticket >= s->reqs.size())
        return CZ_ERR_ARG;
    const Req &q = s->reqs[ticket];
    *done = q.done ? 1 : 0;
    if (status)
        *status = q.status;
    if (out_bytes)
        *out_bytes = q.out_bytes;
    if (t_arrive)
        *t_arrive = q.t_arrive;
    if (t_admit)
        *t_admit = q.t_admit;
    if (t_done)
        *t_done = q.t_done;
    return CZ_OK;
}

int cz_wait(cz_server *s, uint64_t ticket)
{
    if (!s)
        return CZ_ERR_ARG;
    std::unique_lock<std::mutex> lk(s->m);
    if (ticket >= s->reqs.size())
        return CZ_ERR_ARG;
    s->cv.wait(lk, [s, ticket] { return s->reqs[ticket].done; });
    return s->reqs[ticket].status;
}

int cz_server_stop(cz_server *s)
{
    if (!s)
        return CZ_ERR_ARG;
    {
        std::lock_guard<std::mutex> lk(s->m);
        s->stopping = true;
    }
    s->cv.notify_all();
    if (s->worker.joinable())
        s->worker.join();
    const int rc = s->fatal;
    {
        czh::DeviceGuard guard(s->ctx->device);
        destroy_slots(s);
    }
    delete s;
    return rc;
}

}  // extern "C"
