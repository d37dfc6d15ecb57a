// C ABI of libih.so (declared in include/ih.h): argument validation, scratch
// management and dispatch to the HIP kernels.  No arithmetic of the method
// happens here; every step runs on the GPU.
#include "ih.h"
#include "ih_internal.h"

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

namespace {

thread_local std::string g_last_error;

ih_status fail(ih_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

ih_status hip_fail(hipError_t e, const char* where)
{
    return fail(IH_ERR_HIP, "%s: %s", where, hipGetErrorString(e));
}

// Checks shared by every entry point that takes a frame shape.
ih_status check_shape(int32_t H, int32_t W, int32_t B)
{
    if (H <= 0 || W <= 0) return fail(IH_ERR_INVALID_ARG, "H=%d and W=%d must be >= 1", H, W);
    if (B < 1 || B > 256) return fail(IH_ERR_INVALID_ARG, "B=%d must be in [1, 256]", B);
    if ((uint64_t)H * (uint64_t)W >= (1ull << 32))
        return fail(IH_ERR_RANGE, "H*W=%llu must be below 2^32", (unsigned long long)H * (unsigned long long)W);
    return IH_OK;
}

// Device scratch per (device, stream).  Work on one stream is ordered, so one
// buffer per stream is never used by two launches at once.
struct ScratchCache {
    std::mutex mu;
    std::map<std::pair<int, hipStream_t>, std::pair<void*, size_t>> bufs;
};
ScratchCache& cache()
{
    static ScratchCache* c = new ScratchCache;   // never destroyed: freed with the process
    return *c;
}

ih_status get_scratch(hipStream_t stream, size_t bytes, void** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    ScratchCache& c = cache();
    std::lock_guard<std::mutex> lock(c.mu);
    auto key = std::make_pair(dev, stream);
    auto it = c.bufs.find(key);
    if (it != c.bufs.end() && it->second.second >= bytes) {
        *out = it->second.first;
        return IH_OK;
    }
    if (it != c.bufs.end()) {
        // Earlier launches on this stream may still read the old buffer.
        e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
        (void)hipFree(it->second.first);
        c.bufs.erase(it);
    }
    void* p = nullptr;
    const size_t want = bytes < 4096 ? 4096 : bytes;
    e = hipMalloc(&p, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(IH_ERR_OOM, "hipMalloc(%zu) for scratch failed: %s", want, hipGetErrorString(e));
    }
    c.bufs[key] = std::make_pair(p, want);
    *out = p;
    return IH_OK;
}

// Per-phase event timing (off unless ih_profile_enable(1) was called).
struct Profiler {
    std::mutex mu;
    bool on = false;
    struct Rec { hipEvent_t a, b; int phase; };
    std::vector<Rec> pending;
    std::vector<hipEvent_t> pool;
    double ms[ih::kNumPhases] = {0, 0, 0};
    uint64_t frames = 0;

    hipEvent_t get()
    {
        if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    hipError_t drain()
    {
        for (Rec& r : pending) {
            hipError_t e = hipEventSynchronize(r.b);
            if (e != hipSuccess) return e;
            float t = 0.f;
            e = hipEventElapsedTime(&t, r.a, r.b);
            if (e != hipSuccess) return e;
            ms[r.phase] += t;
            pool.push_back(r.a);
            pool.push_back(r.b);
        }
        pending.clear();
        return hipSuccess;
    }
};
Profiler& profiler()
{
    static Profiler* p = new Profiler;
    return *p;
}

}  // namespace

extern "C" {

ih_status ih_profile_enable(int on)
{
    Profiler& p = profiler();
    std::lock_guard<std::mutex> lock(p.mu);
    hipError_t e = p.drain();
    if (e != hipSuccess) return hip_fail(e, "profile drain");
    p.on = on != 0;
    for (double& m : p.ms) m = 0;
    p.frames = 0;
    return IH_OK;
}

ih_status ih_profile_read(ih_phase_times* t)
{
    if (!t) return fail(IH_ERR_INVALID_ARG, "t must be non-null");
    Profiler& p = profiler();
    std::lock_guard<std::mutex> lock(p.mu);
    hipError_t e = p.drain();
    if (e != hipSuccess) return hip_fail(e, "profile drain");
    t->agg_ms = p.ms[0];
    t->scan_ms = p.ms[1];
    t->tile_ms = p.ms[2];
    t->frames = p.frames;
    return IH_OK;
}

// The three phases of one frame on one stream, with optional event timing.
static ih_status enqueue_frame(const uint8_t* frame, uint32_t* out, uint32_t* scratch,
                               const ih::Geom& g, bool nt, hipStream_t s)
{
    Profiler& p = profiler();
    std::unique_lock<std::mutex> lock(p.mu);
    const bool prof = p.on;
    if (!prof) lock.unlock();
    for (int ph = 0; ph < ih::kNumPhases; ++ph) {
        hipEvent_t a = nullptr, b = nullptr;
        if (prof) {
            a = p.get(); b = p.get();
            if (!a || !b) return fail(IH_ERR_HIP, "hipEventCreate failed");
            hipError_t e = hipEventRecord(a, s);
            if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
        }
        hipError_t e = ih::launch_phase(static_cast<ih::Phase>(ph), frame, out, scratch, g, nt, s);
        if (e != hipSuccess) return hip_fail(e, "kernel launch");
        if (prof) {
            e = hipEventRecord(b, s);
            if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
            p.pending.push_back(Profiler::Rec{a, b, ph});
        }
    }
    if (prof) p.frames += 1;
    return IH_OK;
}

const char* ih_status_str(ih_status s)
{
    switch (s) {
    case IH_OK: return "IH_OK";
    case IH_ERR_INVALID_ARG: return "IH_ERR_INVALID_ARG";
    case IH_ERR_RANGE: return "IH_ERR_RANGE";
    case IH_ERR_OOM: return "IH_ERR_OOM";
    case IH_ERR_HIP: return "IH_ERR_HIP";
    case IH_ERR_BUDGET: return "IH_ERR_BUDGET";
    case IH_NOT_READY: return "IH_NOT_READY";
    case IH_ERR_UNKNOWN_TICKET: return "IH_ERR_UNKNOWN_TICKET";
    case IH_ERR_SHUTDOWN: return "IH_ERR_SHUTDOWN";
    }
    return "IH_STATUS_UNKNOWN";
}

const char* ih_last_error(void) { return g_last_error.c_str(); }

const char* ih_version(void) { return "ih 0.1 (gfx950)"; }

ih_status ih_compute(const uint8_t* frame, int32_t H, int32_t W, int32_t B,
                     uint32_t* out, ih_stream_t stream)
{
    if (!frame || !out) return fail(IH_ERR_INVALID_ARG, "frame and out must be non-null");
    if (ih_status st = check_shape(H, W, B)) return st;
    if (reinterpret_cast<uintptr_t>(out) & 3u) return fail(IH_ERR_INVALID_ARG, "out must be 4-byte aligned");

    const ih::TileChoice t = ih::default_tile(H, W, B);
    const ih::Geom g = ih::make_geom(H, W, B, t);
    const ih::ScratchLayout sl = ih::scratch_layout(g);
    void* scratch = nullptr;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (ih_status st = get_scratch(s, sl.words * sizeof(uint32_t), &scratch)) return st;
    return enqueue_frame(frame, out, static_cast<uint32_t*>(scratch), g, t.nontemporal, s);
}

static ih_status check_view(const ih_view* ih)
{
    if (!ih || !ih->data) return fail(IH_ERR_INVALID_ARG, "view and its data must be non-null");
    return check_shape(ih->H, ih->W, ih->B);
}

ih_status ih_query(const ih_view* ih, const ih_rect* rects, size_t n, uint32_t* hists)
{
    if (ih_status st = check_view(ih)) return st;
    if (n == 0) return IH_OK;
    if (!rects || !hists) return fail(IH_ERR_INVALID_ARG, "rects and hists must be non-null");
    if (n > (size_t)INT64_MAX / 256) return fail(IH_ERR_RANGE, "too many rectangles");
    for (size_t r = 0; r < n; ++r) {
        const ih_rect& q = rects[r];
        if (q.x0 < 0 || q.x0 > q.x1 || q.x1 >= ih->W || q.y0 < 0 || q.y0 > q.y1 || q.y1 >= ih->H)
            return fail(IH_ERR_INVALID_ARG, "rectangle %zu {%d,%d,%d,%d} is outside the %dx%d frame",
                        r, q.x0, q.y0, q.x1, q.y1, ih->W, ih->H);
    }
    hipStream_t s = static_cast<hipStream_t>(ih->stream);
    void* d = nullptr;
    hipError_t e = hipMallocAsync(&d, n * sizeof(ih_rect), s);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(IH_ERR_OOM, "hipMallocAsync for %zu rectangles: %s", n, hipGetErrorString(e));
    }
    // Pageable source: the copy is staged before the call returns, so the
    // caller may reuse rects at once.
    e = hipMemcpyAsync(d, rects, n * sizeof(ih_rect), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = ih::launch_query(ih->data, ih->H, ih->W, ih->B, static_cast<const int32_t*>(d),
                             (int64_t)n, hists, nullptr, s);
    hipError_t e2 = hipFreeAsync(d, s);
    if (e != hipSuccess) return hip_fail(e, "query");
    if (e2 != hipSuccess) return hip_fail(e2, "hipFreeAsync");
    return IH_OK;
}

ih_status ih_query_device(const ih_view* ih, const ih_rect* rects_dev, size_t n,
                          uint32_t* hists, uint32_t* bad_count)
{
    if (ih_status st = check_view(ih)) return st;
    if (n == 0) return IH_OK;
    if (!rects_dev || !hists) return fail(IH_ERR_INVALID_ARG, "rects and hists must be non-null");
    if (n > (size_t)INT64_MAX / 256) return fail(IH_ERR_RANGE, "too many rectangles");
    hipError_t e = ih::launch_query(ih->data, ih->H, ih->W, ih->B,
                                    reinterpret_cast<const int32_t*>(rects_dev), (int64_t)n, hists,
                                    bad_count, static_cast<hipStream_t>(ih->stream));
    if (e != hipSuccess) return hip_fail(e, "query");
    return IH_OK;
}

}  // extern "C"
