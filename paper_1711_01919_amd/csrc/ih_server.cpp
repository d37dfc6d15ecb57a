// Serving loop: frame + region-query requests from many video streams,
// admitted FIFO under an HBM budget, batched continuously onto several HIP
// streams, with integral histograms kept resident on the device.
//
// Threads: callers submit, poll and query from any thread; one scheduler
// thread owns every HIP call of the server and all of its device memory.  A
// request moves pending -> admitted (device memory reserved, part of a
// dispatched batch) -> done (results in pinned host memory) -> collected by
// ih_poll.  Queries on a stream's latest resident histogram
// (ih_server_query_latest) go through the scheduler too, ahead of frame
// admissions, and their caller waits for them.
#include "ih.h"
#include "ih_admission.h"
#include "ih_internal.h"
#include "ih_launch.h"
#include "ih_util.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <thread>
#include <unordered_map>
#include <string>
#include <vector>

namespace {

using ih::fail;
using ih::hip_fail;

uint64_t now_ns()
{
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch()).count();
}

constexpr size_t kAlign = 256;

// Pinned host staging: one block allocated on first use and carved by an
// Arena; requests that do not fit it fall back to recycled size-class
// buffers, pinned when the runtime can pin them and ordinary (pageable,
// copied through the runtime's staging) when it cannot.
class PinnedPool {
public:
    explicit PinnedPool(size_t arena_bytes = 0) : arena_bytes_(arena_bytes) {}
    ~PinnedPool()
    {
        for (auto& kv : free_)
            for (void* p : kv.second) release_buffer(p);
        if (base_) (void)hipHostFree(base_);
    }
    void set_arena_bytes(size_t b) { arena_bytes_ = b; }
    // cap == 0 marks an arena block (its offset is p - base_).
    void* get(size_t bytes, size_t* cap)
    {
        std::lock_guard<std::mutex> lock(mu_);
        if (!tried_ && arena_bytes_) {
            tried_ = true;
            if (hipHostMalloc(&base_, arena_bytes_, hipHostMallocDefault) == hipSuccess) {
                arena_.reset(arena_bytes_);
            } else {
                (void)hipGetLastError();
                base_ = nullptr;
            }
        }
        size_t off = 0;
        if (base_ && arena_.alloc(bytes, &off)) {
            *cap = 0;
            sizes_[off] = bytes;
            return static_cast<char*>(base_) + off;
        }
        size_t c = 4096;
        while (c < bytes) c <<= 1;
        *cap = c;
        auto& v = free_[c];
        if (!v.empty()) {
            void* p = v.back();
            v.pop_back();
            return p;
        }
        void* p = nullptr;
        if (hipHostMalloc(&p, c, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            p = std::malloc(c);
            if (p) pageable_.insert(p);
        }
        return p;
    }
    void put(void* p, size_t cap)
    {
        if (!p) return;
        std::lock_guard<std::mutex> lock(mu_);
        if (cap == 0) {
            const size_t off = static_cast<size_t>(static_cast<char*>(p) - static_cast<char*>(base_));
            auto it = sizes_.find(off);
            if (it != sizes_.end()) {
                arena_.release(off, it->second);
                sizes_.erase(it);
            }
            return;
        }
        free_[cap].push_back(p);
    }

private:
    void release_buffer(void* p)
    {
        auto it = pageable_.find(p);
        if (it == pageable_.end()) {
            (void)hipHostFree(p);
        } else {
            std::free(p);
            pageable_.erase(it);
        }
    }
    std::mutex mu_;
    std::set<void*> pageable_;                 // size-class buffers the runtime could not pin
    size_t arena_bytes_ = 0;
    bool tried_ = false;
    void* base_ = nullptr;
    ih::Arena arena_;
    std::map<size_t, size_t> sizes_;
    std::map<size_t, std::vector<void*>> free_;
};

struct Request {
    uint64_t ticket = 0;
    int32_t stream_id = 0, H = 0, W = 0, B = 0;
    size_t nq = 0;
    void* frame_h = nullptr; size_t frame_cap = 0;
    void* rects_h = nullptr; size_t rects_cap = 0;
    void* hists_h = nullptr; size_t hists_cap = 0;
    // device blocks (arena offsets): the integral histogram, and the rest
    size_t ih_off = 0, ih_bytes = 0, work_off = 0, work_bytes = 0;
    ih::Geom geom{};
    bool has_lut = false;    // bins from `lut` (copied at submit) instead of Q(v)
    uint8_t lut[256] = {};
    // a query on the stream's latest resident histogram (ih_server_query_latest)
    bool latest_query = false;
    uint64_t frame_ticket = 0;   // the histogram it read
    ih_timing t{0, 0, 0};
    ih_status status = IH_OK;
    std::string detail;      // error text recorded on the scheduler thread
    bool done = false;
};

// Device and pinned buffers for one batch's launch image (frame table and
// job tables), two per HIP stream (a stream runs at most two batches).
struct ImageSlot {
    void* d = nullptr;
    void* h = nullptr;
    bool busy = false;
};

struct Batch {
    std::vector<std::shared_ptr<Request>> reqs;
    hipEvent_t done = nullptr;
    int stream = 0, slot = -1;
};

}  // namespace

struct ih_server {
    ih_server_config cfg{};
    int device = 0;
    // shared state (mu)
    std::mutex mu;
    std::condition_variable cv;                            // wakes the scheduler
    std::condition_variable cv_done;                       // wakes callers waiting for a latest-query
    bool stop = false;
    bool hold = false;                                     // queue requests without admitting them
    uint64_t budget_blocked = 0;                           // admissions deferred for device memory
    uint64_t next_ticket = 1;
    std::deque<std::shared_ptr<Request>> pending;
    std::deque<std::shared_ptr<Request>> queries;          // latest-queries, served before admissions
    std::unordered_map<uint64_t, std::shared_ptr<Request>> by_ticket;
    size_t admitted = 0;                                   // requests reserved, not yet done
    int64_t retained = 0;                                  // resident histograms kept (copy for stats)
    std::map<int32_t, uint64_t> retained_tickets;          // stream -> ticket of its resident histogram (copy)
    // scheduler-thread state
    std::thread worker;
    bool hip_ready = false;
    ih_status hip_status = IH_OK;
    char* d_arena = nullptr;
    ih::Residency res;                                     // arena + retained histograms
    size_t image_bytes = 0;                                // one image slot
    std::vector<hipStream_t> streams;
    std::vector<int> inflight_per_stream;
    std::vector<std::array<ImageSlot, 2>> slots;           // per stream
    std::list<Batch> inflight;
    std::vector<hipEvent_t> event_pool;
    PinnedPool pinned;
};

namespace {

size_t ih_bytes_of(int32_t H, int32_t W, int32_t B) { return (size_t)H * W * B * 4; }

// Device bytes of everything except the integral histogram: frame,
// rectangles, results, carries and, for table bins, the table.
size_t work_bytes_of(const ih::Geom& g, size_t nq, bool lut)
{
    return ih::align_up((size_t)g.H * g.W, kAlign) + ih::align_up(nq * sizeof(ih_rect), kAlign) +
           ih::align_up(nq * g.B * 4, kAlign) + ih::align_up(ih::frame_scratch_words(g) * 4, kAlign) +
           (lut ? 256 : 0) + kAlign;
}

void release_pinned(ih_server* s, Request& r)
{
    s->pinned.put(r.frame_h, r.frame_cap);
    s->pinned.put(r.rects_h, r.rects_cap);
    s->pinned.put(r.hists_h, r.hists_cap);
    r.frame_h = r.rects_h = r.hists_h = nullptr;
}

// Scheduler thread: create streams, image slots and the arena on first use.
ih_status init_hip(ih_server* s)
{
    if (s->hip_ready) return s->hip_status;
    s->hip_ready = true;
    hipError_t e = hipSetDevice(s->device);
    // load every kernel's code now, not on its first launch inside a request
    if (e == hipSuccess) e = ih::preload_kernels();
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&s->d_arena), s->cfg.hbm_budget_bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        s->hip_status = hip_fail(e, "server arena");
        return s->hip_status;
    }
    s->res.reset(s->cfg.hbm_budget_bytes);
    s->image_bytes = ih::align_up(ih::batch_image_bound((size_t)s->cfg.max_batch), kAlign);
    for (int k = 0; k < s->cfg.n_hip_streams; ++k) {
        hipStream_t st = nullptr;
        e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e != hipSuccess) {
            s->hip_status = hip_fail(e, "hipStreamCreate");
            return s->hip_status;
        }
        s->streams.push_back(st);
        s->inflight_per_stream.push_back(0);
        s->slots.emplace_back();
        for (ImageSlot& sl : s->slots.back()) {
            e = hipMalloc(&sl.d, s->image_bytes);
            if (e == hipSuccess) e = hipHostMalloc(&sl.h, s->image_bytes, hipHostMallocDefault);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                s->hip_status = hip_fail(e, "batch table buffers");
                return s->hip_status;
            }
        }
    }
    return IH_OK;
}

hipEvent_t get_event(ih_server* s)
{
    if (!s->event_pool.empty()) {
        hipEvent_t e = s->event_pool.back();
        s->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
}

// Device addresses inside a request's work block: frame, rectangles,
// results, carries, bin table.
struct WorkPtrs {
    uint8_t* frame;
    ih_rect* rects;
    uint32_t* hists;
    uint32_t* scratch;
    uint32_t* lut;
};
WorkPtrs work_ptrs(ih_server* s, const Request& r)
{
    WorkPtrs w;
    char* p = s->d_arena + r.work_off;
    w.frame = reinterpret_cast<uint8_t*>(p);
    p += r.latest_query ? 0 : ih::align_up((size_t)r.H * r.W, kAlign);     // a query uploads no frame
    w.rects = reinterpret_cast<ih_rect*>(p);
    p += ih::align_up(r.nq * sizeof(ih_rect), kAlign);
    w.hists = reinterpret_cast<uint32_t*>(p);
    p += ih::align_up(r.nq * r.B * 4, kAlign);
    w.scratch = reinterpret_cast<uint32_t*>(p);
    p += r.latest_query ? 0 : ih::align_up(ih::frame_scratch_words(r.geom) * 4, kAlign);
    w.lut = reinterpret_cast<uint32_t*>(p);
    return w;
}

// Enqueue one batch of frame requests on its stream: uploads, the three
// phases for every frame (one launch per phase for all of them, from the
// batch's image slot), the queries, the result downloads.
hipError_t enqueue_frames(ih_server* s, Batch& bt, hipStream_t st)
{
    std::vector<ih::FrameArgs> frames;
    std::vector<char> nt;
    hipError_t e = hipSuccess;
    for (auto& rp : bt.reqs) {
        Request& r = *rp;
        const WorkPtrs w = work_ptrs(s, r);
        uint32_t* d_out = reinterpret_cast<uint32_t*>(s->d_arena + r.ih_off);
        e = hipMemcpyAsync(w.frame, r.frame_h, (size_t)r.H * r.W, hipMemcpyHostToDevice, st);
        if (e == hipSuccess && r.nq)
            e = hipMemcpyAsync(w.rects, r.rects_h, r.nq * sizeof(ih_rect), hipMemcpyHostToDevice, st);
        if (e == hipSuccess && r.has_lut) e = ih::launch_lut_store(r.lut, w.lut, st);
        if (e == hipSuccess && r.geom.K)             // fused schedule: arrival counters start at zero
            e = hipMemsetAsync(w.scratch, 0, (size_t)ih::kCounterWords * sizeof(uint32_t), st);
        if (e != hipSuccess) return e;
        frames.push_back(ih::frame_args(w.frame, d_out, w.scratch, r.geom,
                                        r.has_lut ? reinterpret_cast<const uint8_t*>(w.lut) : nullptr,
                                        r.has_lut && ih::lut_is_general(r.lut)));
        nt.push_back(0);
    }
    ih::BatchImage img;
    ih::build_batch_image(frames, nt, &img);
    if (img.bytes() > s->image_bytes) return hipErrorInvalidValue;     // cannot happen: the slot holds the bound
    ImageSlot& slot = s->slots[bt.stream][bt.slot];
    std::memcpy(slot.h, img.host.data(), img.bytes());
    e = hipMemcpyAsync(slot.d, slot.h, img.bytes(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = ih::enqueue_batch(img, slot.d, -1, st);
    for (size_t k = 0; e == hipSuccess && k < bt.reqs.size(); ++k) {
        Request& r = *bt.reqs[k];
        if (!r.nq) continue;
        const WorkPtrs w = work_ptrs(s, r);
        e = ih::launch_query(frames[k].out, r.H, r.W, r.B, reinterpret_cast<const int32_t*>(w.rects), (int64_t)r.nq,
                             w.hists, nullptr, false, st);
        if (e == hipSuccess) e = hipMemcpyAsync(r.hists_h, w.hists, r.nq * r.B * 4, hipMemcpyDeviceToHost, st);
    }
    return e;
}

// Enqueue a query on a resident histogram (a batch of one latest-query).
hipError_t enqueue_latest_query(ih_server* s, Batch& bt, hipStream_t st)
{
    Request& r = *bt.reqs[0];
    const WorkPtrs w = work_ptrs(s, r);
    // the scheduler marked the histogram as being read when it admitted the query
    const uint32_t* ihp = reinterpret_cast<const uint32_t*>(s->d_arena + r.ih_off);
    hipError_t e = hipMemcpyAsync(w.rects, r.rects_h, r.nq * sizeof(ih_rect), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = ih::launch_query(ihp, r.H, r.W, r.B, reinterpret_cast<const int32_t*>(w.rects), (int64_t)r.nq, w.hists,
                             nullptr, false, st);
    if (e == hipSuccess) e = hipMemcpyAsync(r.hists_h, w.hists, r.nq * r.B * 4, hipMemcpyDeviceToHost, st);
    return e;
}

// Release what an admitted request holds and mark it finished (caller holds
// s->mu).  keep_ih: its histogram became its stream's latest instead.
void finish_locked(ih_server* s, Request& r, ih_status st, const char* detail, bool keep_ih, uint64_t t)
{
    s->res.release(r.work_off, r.work_bytes);
    if (r.latest_query) s->res.release_reader(r.stream_id, r.frame_ticket);
    else if (!keep_ih) s->res.release(r.ih_off, r.ih_bytes);
    r.t.t_done_ns = t;
    r.status = st;
    if (st != IH_OK) r.detail = detail ? detail : "";
    r.done = true;
    if (!r.latest_query) s->admitted -= 1;
}

// Enqueue one batch on its stream and record its completion event.  The
// HIP calls run with s->mu released (they touch only the batch's requests,
// fixed since admission, and scheduler-thread state); the stream and slot are
// marked busy first.  On a failure after work was enqueued, the stream is
// drained before the batch's memory goes back.  Caller holds `lock` on s->mu.
void dispatch(ih_server* s, Batch bt, std::unique_lock<std::mutex>& lock)
{
    hipStream_t st = s->streams[bt.stream];
    const bool query = bt.reqs[0]->latest_query;
    s->slots[bt.stream][bt.slot].busy = true;
    s->inflight_per_stream[bt.stream] += 1;
    lock.unlock();
    hipError_t e = query ? enqueue_latest_query(s, bt, st) : enqueue_frames(s, bt, st);
    if (e == hipSuccess) {
        bt.done = get_event(s);
        if (!bt.done) e = hipErrorOutOfMemory;
    }
    if (e == hipSuccess) e = hipEventRecord(bt.done, st);
    if (e != hipSuccess) (void)hipStreamSynchronize(st);    // whatever was enqueued has finished
    lock.lock();
    if (e == hipSuccess) {
        s->inflight.push_back(std::move(bt));
        return;
    }
    s->slots[bt.stream][bt.slot].busy = false;
    s->inflight_per_stream[bt.stream] -= 1;
    const ih_status fs = hip_fail(e, "batch enqueue");
    const std::string detail = ih_last_error();
    (void)hipGetLastError();
    if (bt.done) s->event_pool.push_back(bt.done);
    const uint64_t t = now_ns();
    for (auto& rp : bt.reqs) finish_locked(s, *rp, fs, detail.c_str(), false, t);
    s->cv_done.notify_all();
}

// Copies of the retention state that other threads read under s->mu.
void refresh_residency_locked(ih_server* s)
{
    s->retained = (int64_t)s->res.retained_count();
    s->retained_tickets = s->res.tickets();
}

// Complete finished batches: stamp, release device memory (keeping the latest
// histogram of each stream when retention is on).  Returns true if any
// finished.  Caller holds s->mu.
bool reap_locked(ih_server* s)
{
    bool any = false;
    for (auto it = s->inflight.begin(); it != s->inflight.end();) {
        hipError_t q = hipEventQuery(it->done);
        if (q == hipErrorNotReady) { ++it; continue; }
        const ih_status st = q == hipSuccess ? IH_OK : hip_fail(q, "batch execution");
        const std::string detail = st == IH_OK ? std::string() : std::string(ih_last_error());
        const uint64_t t = now_ns();
        s->event_pool.push_back(it->done);
        s->slots[it->stream][it->slot].busy = false;
        s->inflight_per_stream[it->stream] -= 1;
        for (auto& rp : it->reqs) {
            Request& r = *rp;
            const bool keep = s->cfg.retain && st == IH_OK && !r.latest_query;
            if (keep) s->res.retain(r.stream_id, ih::Retained{r.ticket, r.H, r.W, r.B, r.ih_off, r.ih_bytes, 0});
            finish_locked(s, r, st, detail.c_str(), keep, t);
        }
        refresh_residency_locked(s);
        it = s->inflight.erase(it);
        any = true;
    }
    if (any) s->cv_done.notify_all();
    return any;
}

// A stream with room for one more batch, and its free image slot.
bool free_stream(ih_server* s, int* stream, int* slot)
{
    for (size_t k = 0; k < s->streams.size(); ++k) {
        if (s->inflight_per_stream[k] >= 2) continue;
        for (int j = 0; j < 2; ++j)
            if (!s->slots[k][j].busy) {
                *stream = (int)k;
                *slot = j;
                return true;
            }
    }
    return false;
}

void fail_request_locked(ih_server* s, Request& r, ih_status st, const char* detail)
{
    r.status = st;
    r.detail = detail;
    r.done = true;
    r.t.t_done_ns = now_ns();
    (void)s;
}

void fail_pending_locked(ih_server* s, ih_status st)
{
    const std::string detail = ih_last_error();
    for (auto& rp : s->pending) fail_request_locked(s, *rp, st, detail.c_str());
    for (auto& rp : s->queries) fail_request_locked(s, *rp, st, detail.c_str());
    s->pending.clear();
    s->queries.clear();
    s->cv_done.notify_all();
}

// Latest-queries first: each takes a stream and reads its stream's resident
// histogram (marked as being read until it finishes).
bool serve_queries_locked(ih_server* s, std::unique_lock<std::mutex>& lock)
{
    bool progressed = false;
    while (!s->queries.empty()) {
        int k = 0, slot = 0;
        if (!free_stream(s, &k, &slot)) break;
        std::shared_ptr<Request> r = s->queries.front();
        ih::Retained h;
        if (!s->res.acquire(r->stream_id, &h)) {
            s->queries.pop_front();
            fail_request_locked(s, *r, fail(IH_ERR_INVALID_ARG, "stream %d has no resident integral histogram",
                                            r->stream_id), ih_last_error());
            s->cv_done.notify_all();
            progressed = true;
            continue;
        }
        bool bad = false;
        for (size_t q = 0; q < r->nq && !bad; ++q) {
            const ih_rect& x = static_cast<const ih_rect*>(r->rects_h)[q];
            bad = x.x0 < 0 || x.x0 > x.x1 || x.x1 >= h.W || x.y0 < 0 || x.y0 > x.y1 || x.y1 >= h.H;
        }
        const size_t hb = ih::align_up(r->nq * (size_t)h.B * 4, kAlign);
        if (bad) {
            s->res.release_reader(r->stream_id, h.ticket);
            s->queries.pop_front();
            fail_request_locked(s, *r, fail(IH_ERR_INVALID_ARG, "a rectangle is outside the %dx%d frame", h.W, h.H),
                                ih_last_error());
            s->cv_done.notify_all();
            progressed = true;
            continue;
        }
        r->H = h.H; r->W = h.W; r->B = h.B;
        r->ih_off = h.off;
        r->frame_ticket = h.ticket;
        r->work_bytes = ih::align_up(r->nq * sizeof(ih_rect), kAlign) + hb + kAlign;
        size_t off = 0;
        const ih::Admit a = s->res.reserve_one(r->work_bytes, !s->inflight.empty(), r->stream_id, &off);
        if (a == ih::Admit::kWait) {
            s->res.release_reader(r->stream_id, h.ticket);
            s->budget_blocked += 1;
            break;
        }
        s->queries.pop_front();
        if (a == ih::Admit::kNever) {
            s->res.release_reader(r->stream_id, h.ticket);
            fail_request_locked(s, *r, fail(IH_ERR_BUDGET, "query results do not fit the budget"), ih_last_error());
            s->cv_done.notify_all();
            progressed = true;
            continue;
        }
        r->work_off = off;
        r->t.t_admit_ns = now_ns();
        Batch bt;
        bt.stream = k;
        bt.slot = slot;
        bt.reqs.push_back(r);
        dispatch(s, std::move(bt), lock);
        progressed = true;
    }
    return progressed;
}

void scheduler(ih_server* s)
{
    std::unique_lock<std::mutex> lock(s->mu);
    for (;;) {
        bool progressed = false;
        if (!s->inflight.empty()) progressed |= reap_locked(s);
        if (s->stop && s->inflight.empty()) {
            fail_pending_locked(s, fail(IH_ERR_SHUTDOWN, "server is shutting down"));
            return;
        }
        if (!s->stop && (!s->queries.empty() || (!s->hold && !s->pending.empty()))) {
            const ih_status hs = init_hip(s);
            if (hs != IH_OK) {
                fail_pending_locked(s, hs);
                continue;
            }
            progressed |= serve_queries_locked(s, lock);
            refresh_residency_locked(s);
        }
        if (!s->stop && !s->hold && !s->pending.empty() && s->hip_status == IH_OK) {
            // Continuous batching: every stream with room takes the requests at
            // the head of the queue that fit (FIFO, no overtaking).
            int k = 0, slot = 0;
            while (!s->pending.empty() && free_stream(s, &k, &slot)) {
                Batch bt;
                bt.stream = k;
                bt.slot = slot;
                while (!s->pending.empty() && (int)bt.reqs.size() < s->cfg.max_batch &&
                       (int)s->admitted < s->cfg.max_slots) {
                    std::shared_ptr<Request> r = s->pending.front();
                    const bool held = !s->inflight.empty() || !bt.reqs.empty();
                    const ih::Admit a = s->res.reserve(r->ih_bytes, r->work_bytes, held, &r->ih_off, &r->work_off);
                    if (a == ih::Admit::kWait) {
                        s->budget_blocked += 1;
                        break;
                    }
                    s->pending.pop_front();
                    if (a == ih::Admit::kNever) {
                        fail_request_locked(s, *r, fail(IH_ERR_BUDGET, "request does not fit the budget's arena"),
                                            ih_last_error());
                        progressed = true;
                        continue;
                    }
                    r->t.t_admit_ns = now_ns();
                    s->admitted += 1;
                    bt.reqs.push_back(r);
                }
                refresh_residency_locked(s);
                if (bt.reqs.empty()) break;
                dispatch(s, std::move(bt), lock);
                progressed = true;
            }
        }
        if (!progressed) {
            // Wake on submit/query/shutdown, or poll the device again shortly.
            s->cv.wait_for(lock, std::chrono::microseconds(s->inflight.empty() ? 2000 : 20));
        }
    }
}

// Validate and queue one request (ih_submit, ih_submit_lut).  The frame,
// rectangles and bin table are copied before it returns.
ih_status submit_request(ih_server* s, int32_t stream_id, const uint8_t* frame_host, int32_t H, int32_t W,
                         int32_t B, const uint8_t* lut_host, const ih_rect* rects_host, size_t nq,
                         uint64_t* ticket)
{
    const uint64_t t0 = now_ns();
    if (!s || !frame_host || !ticket || (nq && !rects_host))
        return fail(IH_ERR_INVALID_ARG, "server, frame, ticket (and rects when nq > 0) must be non-null");
    if (ih_status st = ih::check_shape(H, W, B)) return st;
    for (size_t r = 0; r < nq; ++r) {
        const ih_rect& q = rects_host[r];
        if (q.x0 < 0 || q.x0 > q.x1 || q.x1 >= W || q.y0 < 0 || q.y0 > q.y1 || q.y1 >= H)
            return fail(IH_ERR_INVALID_ARG, "rectangle %zu is outside the %dx%d frame", r, W, H);
    }
    for (int v = 0; lut_host && v < 256; ++v)
        if ((int32_t)lut_host[v] >= B)
            return fail(IH_ERR_INVALID_ARG, "lut[%d]=%d is not a bin below B=%d", v, lut_host[v], B);
    auto r = std::make_shared<Request>();
    r->stream_id = stream_id;
    r->H = H; r->W = W; r->B = B; r->nq = nq;
    r->geom = ih::make_geom(H, W, B, ih::default_tile(H, W, B));
    r->ih_bytes = ih_bytes_of(H, W, B);
    r->has_lut = lut_host != nullptr;
    if (r->has_lut) std::memcpy(r->lut, lut_host, 256);
    r->work_bytes = work_bytes_of(r->geom, nq, r->has_lut);
    const size_t need = ih::align_up(r->ih_bytes, kAlign) + ih::align_up(r->work_bytes, kAlign) + (64u << 10);
    if (need > s->cfg.hbm_budget_bytes)
        return fail(IH_ERR_BUDGET, "request needs %zu device bytes, budget is %llu", need,
                    (unsigned long long)s->cfg.hbm_budget_bytes);
    r->frame_h = s->pinned.get((size_t)H * W, &r->frame_cap);
    r->rects_h = s->pinned.get(std::max<size_t>(nq, 1) * sizeof(ih_rect), &r->rects_cap);
    r->hists_h = s->pinned.get(std::max<size_t>(nq, 1) * B * 4, &r->hists_cap);
    if (!r->frame_h || !r->rects_h || !r->hists_h) {
        release_pinned(s, *r);
        return fail(IH_ERR_OOM, "pinned host staging");
    }
    std::memcpy(r->frame_h, frame_host, (size_t)H * W);
    if (nq) std::memcpy(r->rects_h, rects_host, nq * sizeof(ih_rect));
    r->t.t_submit_ns = t0;
    {
        std::lock_guard<std::mutex> lock(s->mu);
        if (s->stop) {
            release_pinned(s, *r);
            return fail(IH_ERR_SHUTDOWN, "server is shutting down");
        }
        r->ticket = s->next_ticket++;
        s->by_ticket[r->ticket] = r;
        s->pending.push_back(r);
        *ticket = r->ticket;
    }
    s->cv.notify_one();
    return IH_OK;
}

}  // namespace

extern "C" {

ih_status ih_server_create(const ih_server_config* cfg, ih_server** out)
{
    if (!cfg || !out) return fail(IH_ERR_INVALID_ARG, "cfg and out must be non-null");
    *out = nullptr;
    if (cfg->hbm_budget_bytes < (1u << 20)) return fail(IH_ERR_INVALID_ARG, "budget must be at least 1 MiB");
    if (cfg->max_slots < 1 || cfg->n_hip_streams < 1 || cfg->n_hip_streams > 16 || cfg->max_batch < 1)
        return fail(IH_ERR_INVALID_ARG, "max_slots, max_batch >= 1 and n_hip_streams in [1, 16] required");
    ih_server* s = new ih_server;
    s->cfg = *cfg;
    s->pinned.set_arena_bytes(cfg->pinned_bytes ? cfg->pinned_bytes : (1ull << 30));
    if (hipGetDevice(&s->device) != hipSuccess) {
        (void)hipGetLastError();
        s->device = 0;
    }
    s->worker = std::thread(scheduler, s);
    *out = s;
    return IH_OK;
}

ih_status ih_submit(ih_server* s, int32_t stream_id, const uint8_t* frame_host, int32_t H, int32_t W,
                    int32_t B, const ih_rect* rects_host, size_t nq, uint64_t* ticket)
{
    return submit_request(s, stream_id, frame_host, H, W, B, nullptr, rects_host, nq, ticket);
}

ih_status ih_submit_lut(ih_server* s, int32_t stream_id, const uint8_t* frame_host, int32_t H, int32_t W,
                        int32_t B, const uint8_t* lut_host, const ih_rect* rects_host, size_t nq, uint64_t* ticket)
{
    if (!lut_host) return fail(IH_ERR_INVALID_ARG, "lut must be non-null");
    return submit_request(s, stream_id, frame_host, H, W, B, lut_host, rects_host, nq, ticket);
}

ih_status ih_poll(ih_server* s, uint64_t ticket, uint32_t* hists_host, ih_timing* t)
{
    if (!s) return fail(IH_ERR_INVALID_ARG, "server must be non-null");
    std::shared_ptr<Request> r;
    {
        std::lock_guard<std::mutex> lock(s->mu);
        auto it = s->by_ticket.find(ticket);
        if (it == s->by_ticket.end()) return fail(IH_ERR_UNKNOWN_TICKET, "ticket %llu unknown", (unsigned long long)ticket);
        if (!it->second->done) return IH_NOT_READY;
        r = it->second;
        s->by_ticket.erase(it);
    }
    if (t) *t = r->t;
    const ih_status st = r->status;
    if (st == IH_OK && hists_host && r->nq) std::memcpy(hists_host, r->hists_h, r->nq * r->B * 4);
    release_pinned(s, *r);
    if (st != IH_OK)
        return fail(st, "request %llu failed: %s (%s)", (unsigned long long)ticket, ih_status_str(st),
                    r->detail.c_str());
    return IH_OK;
}

ih_status ih_server_query_latest(ih_server* s, int32_t stream_id, const ih_rect* rects_host, size_t nq,
                                 uint32_t* hists_host, uint64_t* frame_ticket)
{
    if (!s || (nq && (!rects_host || !hists_host))) return fail(IH_ERR_INVALID_ARG, "bad arguments");
    if (nq > ((size_t)1 << 24)) return fail(IH_ERR_RANGE, "too many rectangles (%zu)", nq);
    auto r = std::make_shared<Request>();
    r->latest_query = true;
    r->stream_id = stream_id;
    r->nq = nq;
    r->t.t_submit_ns = now_ns();
    if (nq) {
        // results are at most 256 bins per rectangle; the scheduler checks the
        // rectangles against the resident histogram's shape
        r->rects_h = s->pinned.get(nq * sizeof(ih_rect), &r->rects_cap);
        r->hists_h = s->pinned.get(nq * 256 * 4, &r->hists_cap);
        if (!r->rects_h || !r->hists_h) {
            release_pinned(s, *r);
            return fail(IH_ERR_OOM, "pinned host staging");
        }
        std::memcpy(r->rects_h, rects_host, nq * sizeof(ih_rect));
    }
    std::unique_lock<std::mutex> lock(s->mu);
    if (s->stop) {
        lock.unlock();
        release_pinned(s, *r);
        return fail(IH_ERR_SHUTDOWN, "server is shutting down");
    }
    if (nq == 0) {
        // nothing to compute: the ticket of the resident histogram, if any
        const bool any = s->retained_tickets.count(stream_id) != 0;
        const uint64_t tk = any ? s->retained_tickets[stream_id] : 0;
        lock.unlock();
        if (!any) return fail(IH_ERR_INVALID_ARG, "stream %d has no resident integral histogram", stream_id);
        if (frame_ticket) *frame_ticket = tk;
        return IH_OK;
    }
    s->queries.push_back(r);
    s->cv.notify_one();
    s->cv_done.wait(lock, [&] { return r->done; });
    lock.unlock();
    const ih_status st = r->status;
    if (st == IH_OK) {
        std::memcpy(hists_host, r->hists_h, nq * (size_t)r->B * 4);
        if (frame_ticket) *frame_ticket = r->frame_ticket;
    }
    release_pinned(s, *r);
    if (st != IH_OK) return fail(st, "%s", r->detail.c_str());
    return IH_OK;
}

ih_status ih_server_stats(ih_server* s, ih_server_counters* c)
{
    if (!s || !c) return fail(IH_ERR_INVALID_ARG, "bad arguments");
    std::lock_guard<std::mutex> lock(s->mu);
    c->pending = (int64_t)s->pending.size();
    c->admitted = (int64_t)s->admitted;
    c->retained = s->retained;
    c->device_bytes_used = (uint64_t)s->res.arena().used();
    c->device_bytes_peak = (uint64_t)s->res.arena().peak();
    c->budget_blocked = s->budget_blocked;
    return IH_OK;
}

ih_status ih_server_hold(ih_server* s, int32_t hold)
{
    if (!s) return fail(IH_ERR_INVALID_ARG, "server must be non-null");
    {
        std::lock_guard<std::mutex> lock(s->mu);
        s->hold = hold != 0;
    }
    s->cv.notify_one();
    return IH_OK;
}

ih_status ih_server_destroy(ih_server* s)
{
    if (!s) return IH_OK;
    {
        std::lock_guard<std::mutex> lock(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    if (s->worker.joinable()) s->worker.join();
    // every batch has completed; release device and host resources
    for (hipEvent_t e : s->event_pool) (void)hipEventDestroy(e);
    for (auto& pair : s->slots)
        for (ImageSlot& sl : pair) {
            if (sl.d) (void)hipFree(sl.d);
            if (sl.h) (void)hipHostFree(sl.h);
        }
    for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
    if (s->d_arena) (void)hipFree(s->d_arena);
    for (auto& kv : s->by_ticket) release_pinned(s, *kv.second);
    delete s;
    return IH_OK;
}

}  // extern "C"
