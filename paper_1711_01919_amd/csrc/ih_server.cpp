// Serving loop: frame + region-query requests from many video streams,
// admitted FIFO under an HBM budget, batched continuously onto several HIP
// streams, with integral histograms kept resident on the device.
//
// Threads: callers submit and poll from any thread; one scheduler thread owns
// every HIP call of the server.  A request moves pending -> admitted
// (device memory reserved, part of a dispatched batch) -> done (results in
// pinned host memory) -> collected by ih_poll.
#include "ih.h"
#include "ih_internal.h"
#include "ih_launch.h"
#include "ih_util.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <memory>
#include <mutex>
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

// First-fit allocator over one device allocation; offsets only (host-side
// bookkeeping), neighbours merged on free.  Thread-safe.
class Arena {
public:
    void reset(size_t size)
    {
        std::lock_guard<std::mutex> lock(mu_);
        size_ = size;
        free_.clear();
        if (size) free_[0] = size;
        used_ = 0;
    }
    bool alloc(size_t bytes, size_t* off)
    {
        std::lock_guard<std::mutex> lock(mu_);
        bytes = ih::align_up(std::max<size_t>(bytes, 1), kAlign);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes;
            const size_t at = it->first + bytes;
            free_.erase(it);
            if (rest) free_[at] = rest;
            used_ += bytes;
            peak_ = std::max(peak_, used_);
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        std::lock_guard<std::mutex> lock(mu_);
        bytes = ih::align_up(std::max<size_t>(bytes, 1), kAlign);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const
    {
        std::lock_guard<std::mutex> lock(mu_);
        return used_;
    }
    size_t size() const
    {
        std::lock_guard<std::mutex> lock(mu_);
        return size_;
    }
    size_t peak() const
    {
        std::lock_guard<std::mutex> lock(mu_);
        return peak_;
    }

private:
    mutable std::mutex mu_;
    size_t size_ = 0, used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;
};

// Pinned host staging: one block allocated on first use and carved by an
// Arena; requests that do not fit it fall back to recycled size-class buffers.
class PinnedPool {
public:
    explicit PinnedPool(size_t arena_bytes = 0) : arena_bytes_(arena_bytes) {}
    ~PinnedPool()
    {
        for (auto& kv : free_)
            for (void* p : kv.second) (void)hipHostFree(p);
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
            return nullptr;
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
    std::mutex mu_;
    size_t arena_bytes_ = 0;
    bool tried_ = false;
    void* base_ = nullptr;
    Arena arena_;
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
    ih_timing t{0, 0, 0};
    ih_status status = IH_OK;
    std::string detail;      // error text recorded on the scheduler thread
    bool done = false;
};

struct Batch {
    std::vector<std::shared_ptr<Request>> reqs;
    size_t img_off = 0, img_bytes = 0;
    void* img_h = nullptr; size_t img_cap = 0;
    hipEvent_t done = nullptr;
    int stream = 0;
};

}  // namespace

struct ih_server {
    ih_server_config cfg{};
    int device = 0;
    // shared state (mu)
    std::mutex mu;
    std::condition_variable cv;
    bool stop = false;
    bool hold = false;                                     // queue requests without admitting them
    uint64_t budget_blocked = 0;                           // admissions deferred for device memory
    uint64_t next_ticket = 1;
    std::deque<std::shared_ptr<Request>> pending;
    std::unordered_map<uint64_t, std::shared_ptr<Request>> by_ticket;
    size_t admitted = 0;                                   // requests reserved, not yet done
    // scheduler-thread state
    std::thread worker;
    bool hip_ready = false;
    ih_status hip_status = IH_OK;
    char* d_arena = nullptr;
    Arena arena;
    std::vector<hipStream_t> streams;
    std::vector<int> inflight_per_stream;
    std::list<Batch> inflight;
    std::vector<hipEvent_t> event_pool;
    PinnedPool pinned;
    // retention: latest integral histogram per video stream (LRU order)
    struct Retained { uint64_t ticket; int32_t H, W, B; size_t off, bytes; };
    std::map<int32_t, Retained> retained;
    std::list<int32_t> retained_lru;
    std::mutex retained_mu;                                // guards retained + its arena blocks for queries
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

// Scheduler thread: create streams and the arena on first use.
ih_status init_hip(ih_server* s)
{
    if (s->hip_ready) return s->hip_status;
    s->hip_ready = true;
    hipError_t e = hipSetDevice(s->device);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&s->d_arena), s->cfg.hbm_budget_bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        s->hip_status = hip_fail(e, "server arena");
        return s->hip_status;
    }
    s->arena.reset(s->cfg.hbm_budget_bytes);
    for (int k = 0; k < s->cfg.n_hip_streams; ++k) {
        hipStream_t st = nullptr;
        e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e != hipSuccess) {
            s->hip_status = hip_fail(e, "hipStreamCreate");
            return s->hip_status;
        }
        s->streams.push_back(st);
        s->inflight_per_stream.push_back(0);
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

// Free the least recently retained histograms until `bytes` more fit (or
// nothing is left to evict).  Scheduler thread.
void evict_for(ih_server* s, size_t bytes)
{
    std::lock_guard<std::mutex> lock(s->retained_mu);
    while (!s->retained_lru.empty() && s->arena.size() - s->arena.used() < bytes) {
        const int32_t sid = s->retained_lru.front();
        s->retained_lru.pop_front();
        auto it = s->retained.find(sid);
        if (it != s->retained.end()) {
            s->arena.release(it->second.off, it->second.bytes);
            s->retained.erase(it);
        }
    }
}

bool reserve(ih_server* s, Request& r)
{
    const size_t need = ih::align_up(r.ih_bytes, kAlign) + ih::align_up(r.work_bytes, kAlign);
    if (s->arena.size() - s->arena.used() < need) evict_for(s, need);
    size_t a = 0, b = 0;
    if (!s->arena.alloc(r.ih_bytes, &a)) {
        evict_for(s, s->arena.size());       // fragmentation: drop every retained histogram
        if (!s->arena.alloc(r.ih_bytes, &a)) return false;
    }
    if (!s->arena.alloc(r.work_bytes, &b)) {
        s->arena.release(a, r.ih_bytes);
        return false;
    }
    r.ih_off = a;
    r.work_off = b;
    return true;
}

// Enqueue one batch on stream k: uploads, the three phases for every frame,
// the queries, the result downloads, and a completion event.
ih_status dispatch(ih_server* s, Batch& bt)
{
    hipStream_t st = s->streams[bt.stream];
    std::vector<ih::FrameArgs> frames;
    std::vector<char> nt;
    for (auto& rp : bt.reqs) {
        Request& r = *rp;
        char* work = s->d_arena + r.work_off;
        uint8_t* d_frame = reinterpret_cast<uint8_t*>(work);
        ih_rect* d_rects = reinterpret_cast<ih_rect*>(work + ih::align_up((size_t)r.H * r.W, kAlign));
        uint32_t* d_hists = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(d_rects) +
                                                        ih::align_up(r.nq * sizeof(ih_rect), kAlign));
        uint32_t* d_scratch = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(d_hists) +
                                                          ih::align_up(r.nq * r.B * 4, kAlign));
        uint32_t* d_out = reinterpret_cast<uint32_t*>(s->d_arena + r.ih_off);
        uint32_t* d_lut = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(d_scratch) +
                                                      ih::align_up(ih::frame_scratch_words(r.geom) * 4, kAlign));
        hipError_t e = hipMemcpyAsync(d_frame, r.frame_h, (size_t)r.H * r.W, hipMemcpyHostToDevice, st);
        if (e == hipSuccess && r.nq)
            e = hipMemcpyAsync(d_rects, r.rects_h, r.nq * sizeof(ih_rect), hipMemcpyHostToDevice, st);
        if (e == hipSuccess && r.has_lut) e = ih::launch_lut_store(r.lut, d_lut, st);
        if (e != hipSuccess) return hip_fail(e, "request upload");
        frames.push_back(ih::frame_args(d_frame, d_out, d_scratch, r.geom,
                                        r.has_lut ? reinterpret_cast<const uint8_t*>(d_lut) : nullptr));
        nt.push_back(0);
    }
    ih::BatchImage img;
    ih::build_batch_image(frames, nt, &img);
    bt.img_bytes = img.bytes();
    if (!s->arena.alloc(bt.img_bytes, &bt.img_off)) return fail(IH_ERR_OOM, "batch tables do not fit the budget");
    bt.img_h = s->pinned.get(bt.img_bytes, &bt.img_cap);
    if (!bt.img_h) return fail(IH_ERR_OOM, "pinned staging");
    std::memcpy(bt.img_h, img.host.data(), bt.img_bytes);
    void* d_img = s->d_arena + bt.img_off;
    hipError_t e = hipMemcpyAsync(d_img, bt.img_h, bt.img_bytes, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = ih::enqueue_batch(img, d_img, -1, st);
    for (size_t k = 0; e == hipSuccess && k < bt.reqs.size(); ++k) {
        Request& r = *bt.reqs[k];
        if (!r.nq) continue;
        const ih::FrameArgs& f = frames[k];
        const char* work = s->d_arena + r.work_off;
        const int32_t* d_rects = reinterpret_cast<const int32_t*>(work + ih::align_up((size_t)r.H * r.W, kAlign));
        uint32_t* d_hists = reinterpret_cast<uint32_t*>(const_cast<char*>(work) + ih::align_up((size_t)r.H * r.W, kAlign) +
                                                        ih::align_up(r.nq * sizeof(ih_rect), kAlign));
        e = ih::launch_query(f.out, r.H, r.W, r.B, d_rects, (int64_t)r.nq, d_hists, nullptr, false, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(r.hists_h, d_hists, r.nq * r.B * 4, hipMemcpyDeviceToHost, st);
    }
    if (e != hipSuccess) return hip_fail(e, "batch enqueue");
    bt.done = get_event(s);
    if (!bt.done) return fail(IH_ERR_HIP, "hipEventCreate failed");
    e = hipEventRecord(bt.done, st);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    return IH_OK;
}

// Complete finished batches: stamp, release device memory (keeping the latest
// histogram of each stream when retention is on).  Returns true if any finished.
bool reap(ih_server* s)
{
    bool any = false;
    for (auto it = s->inflight.begin(); it != s->inflight.end();) {
        hipError_t q = hipEventQuery(it->done);
        if (q == hipErrorNotReady) { ++it; continue; }
        const ih_status st = q == hipSuccess ? IH_OK : hip_fail(q, "batch execution");
        const uint64_t t = now_ns();
        s->arena.release(it->img_off, it->img_bytes);
        s->pinned.put(it->img_h, it->img_cap);
        s->event_pool.push_back(it->done);
        s->inflight_per_stream[it->stream] -= 1;
        {
            std::lock_guard<std::mutex> lock(s->mu);
            for (auto& rp : it->reqs) {
                Request& r = *rp;
                s->arena.release(r.work_off, r.work_bytes);
                bool keep = false;
                if (s->cfg.retain && st == IH_OK) {
                    std::lock_guard<std::mutex> rl(s->retained_mu);
                    auto old = s->retained.find(r.stream_id);
                    if (old != s->retained.end()) {
                        s->arena.release(old->second.off, old->second.bytes);
                        s->retained_lru.remove(r.stream_id);
                    }
                    s->retained[r.stream_id] = ih_server::Retained{r.ticket, r.H, r.W, r.B, r.ih_off, r.ih_bytes};
                    s->retained_lru.push_back(r.stream_id);
                    keep = true;
                }
                if (!keep) s->arena.release(r.ih_off, r.ih_bytes);
                r.t.t_done_ns = t;
                r.status = st;
                if (st != IH_OK) r.detail = ih_last_error();
                r.done = true;
                s->admitted -= 1;
            }
        }
        it = s->inflight.erase(it);
        any = true;
    }
    return any;
}

}  // namespace

namespace {

void fail_pending(ih_server* s, ih_status st)
{
    // caller holds s->mu
    const uint64_t t = now_ns();
    for (auto& rp : s->pending) {
        rp->status = st;
        rp->detail = ih_last_error();
        rp->done = true;
        rp->t.t_done_ns = t;
    }
    s->pending.clear();
}

void scheduler(ih_server* s)
{
    for (;;) {
        bool progressed = false;
        if (!s->inflight.empty()) progressed |= reap(s);

        std::unique_lock<std::mutex> lock(s->mu);
        if (s->stop && s->inflight.empty()) {
            fail_pending(s, IH_ERR_SHUTDOWN);
            return;
        }
        if (!s->stop && !s->hold && !s->pending.empty()) {
            lock.unlock();
            const ih_status hs = init_hip(s);
            lock.lock();
            if (hs != IH_OK) {
                fail_pending(s, hs);
                continue;
            }
            // Continuous batching: every stream with room takes the requests at
            // the head of the queue that fit (FIFO, no overtaking).
            for (size_t k = 0; k < s->streams.size() && !s->pending.empty(); ++k) {
                if (s->inflight_per_stream[k] >= 2) continue;
                Batch bt;
                bt.stream = (int)k;
                while (!s->pending.empty() && (int)bt.reqs.size() < s->cfg.max_batch &&
                       (int)s->admitted < s->cfg.max_slots) {
                    std::shared_ptr<Request> r = s->pending.front();
                    if (!reserve(s, *r)) {
                        s->budget_blocked += 1;
                        break;
                    }
                    s->pending.pop_front();
                    r->t.t_admit_ns = now_ns();
                    s->admitted += 1;
                    bt.reqs.push_back(r);
                }
                if (bt.reqs.empty()) break;
                lock.unlock();
                ih_status st = dispatch(s, bt);
                lock.lock();
                s->inflight_per_stream[k] += 1;
                if (st != IH_OK && !bt.done) {
                    // nothing recorded: finish the batch here with the error
                    for (auto& rp : bt.reqs) {
                        s->arena.release(rp->work_off, rp->work_bytes);
                        s->arena.release(rp->ih_off, rp->ih_bytes);
                        rp->status = st;
                        rp->detail = ih_last_error();
                        rp->done = true;
                        rp->t.t_done_ns = now_ns();
                        s->admitted -= 1;
                    }
                    if (bt.img_bytes && bt.img_h) s->pinned.put(bt.img_h, bt.img_cap);
                    s->inflight_per_stream[k] -= 1;
                } else {
                    s->inflight.push_back(std::move(bt));
                }
                progressed = true;
            }
        }
        if (!progressed) {
            // Wake on submit/shutdown, or poll the device again shortly.
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
    for (int v = 0; lut_host && v < 256; ++v) {
        if ((int32_t)lut_host[v] >= B)
            return fail(IH_ERR_INVALID_ARG, "lut[%d]=%d is not a bin below B=%d", v, lut_host[v], B);
        if (v > 0 && lut_host[v] < lut_host[v - 1])
            return fail(IH_ERR_INVALID_ARG, "lut decreases at %d (%d after %d)", v, lut_host[v], lut_host[v - 1]);
    }
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
    std::lock_guard<std::mutex> rl(s->retained_mu);
    auto it = s->retained.find(stream_id);
    if (it == s->retained.end()) return fail(IH_ERR_INVALID_ARG, "stream %d has no resident integral histogram", stream_id);
    const ih_server::Retained& k = it->second;
    if (frame_ticket) *frame_ticket = k.ticket;
    if (nq == 0) return IH_OK;
    ih_view v{reinterpret_cast<const uint32_t*>(s->d_arena + k.off), k.H, k.W, k.B, nullptr};
    uint32_t* d_hists = nullptr;
    hipError_t e = hipMalloc(&d_hists, nq * k.B * 4);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(IH_ERR_OOM, "query output");
    }
    hipStream_t st = nullptr;
    e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e != hipSuccess) {
        (void)hipFree(d_hists);
        return hip_fail(e, "hipStreamCreate");
    }
    v.stream = st;
    ih_status r = ih_query(&v, rects_host, nq, d_hists);
    if (r == IH_OK) {
        e = hipMemcpyAsync(hists_host, d_hists, nq * k.B * 4, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) r = hip_fail(e, "query download");
    }
    (void)hipStreamDestroy(st);
    (void)hipFree(d_hists);
    return r;
}

ih_status ih_server_stats(ih_server* s, ih_server_counters* c)
{
    if (!s || !c) return fail(IH_ERR_INVALID_ARG, "bad arguments");
    std::lock_guard<std::mutex> lock(s->mu);
    c->pending = (int64_t)s->pending.size();
    c->admitted = (int64_t)s->admitted;
    c->device_bytes_used = (uint64_t)s->arena.used();
    c->device_bytes_peak = (uint64_t)s->arena.peak();
    c->budget_blocked = s->budget_blocked;
    {
        std::lock_guard<std::mutex> rl(s->retained_mu);
        c->retained = (int64_t)s->retained.size();
    }
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
    for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
    if (s->d_arena) (void)hipFree(s->d_arena);
    for (auto& kv : s->by_ticket) release_pinned(s, *kv.second);
    delete s;
    return IH_OK;
}

}  // extern "C"
