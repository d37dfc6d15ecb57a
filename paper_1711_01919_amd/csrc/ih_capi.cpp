// Single-frame entry points of libih.so (declared in include/ih.h): argument
// validation, per-stream scratch and dispatch to the HIP kernels.  No
// arithmetic of the method happens here; every step runs on the GPU.
#include "ih.h"
#include "ih_internal.h"
#include "ih_util.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <map>
#include <mutex>
#include <utility>

namespace {

using ih::fail;
using ih::hip_fail;

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
    // the fused schedule's arrival counters start at zero (stream order puts
    // this before every kernel that uses the buffer)
    e = hipMemsetAsync(p, 0, std::min(want, (size_t)ih::kCounterWords * sizeof(uint32_t)), stream);
    if (e != hipSuccess) {
        (void)hipFree(p);
        return hip_fail(e, "hipMemsetAsync");
    }
    c.bufs[key] = std::make_pair(p, want);
    *out = p;
    return IH_OK;
}

// The three phases of one frame on one stream, timed when profiling is on.
ih_status enqueue_frame(const uint8_t* frame, uint32_t* out, uint32_t* scratch,
                        const ih::Geom& g, bool nt, hipStream_t s, const uint8_t* lut = nullptr,
                        bool lut_general = false)
{
    const ih::FrameArgs fa = ih::frame_args(frame, out, scratch, g, lut, lut_general);
    ih::PhaseTimer timer;
    for (int ph = 0; ph < ih::kNumPhases; ++ph) {
        if (ih_status st = timer.begin(ph, s)) return st;
        hipError_t e = ih::launch_phase(static_cast<ih::Phase>(ph), fa, nt, s);
        if (e != hipSuccess) return hip_fail(e, "kernel launch");
        if (ih_status st = timer.end(s)) return st;
    }
    if (ih::profiling_on()) ih::profiling_add_frames(1);
    return IH_OK;
}

ih_status check_view(const ih_view* ih)
{
    if (!ih || !ih->data) return fail(IH_ERR_INVALID_ARG, "view and its data must be non-null");
    return ih::check_shape(ih->H, ih->W, ih->B);
}

// Region queries (Eq. 2) on either layout: host rectangles are validated on
// the host and staged through stream-ordered device memory; device
// rectangles are checked by the kernel.
ih_status query_host(const ih_view* ih, const ih_rect* rects, size_t n, uint32_t* hists, bool binmajor)
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
                             (int64_t)n, hists, nullptr, binmajor, s);
    hipError_t e2 = hipFreeAsync(d, s);
    if (e != hipSuccess) return hip_fail(e, "query");
    if (e2 != hipSuccess) return hip_fail(e2, "hipFreeAsync");
    return IH_OK;
}

ih_status query_dev(const ih_view* ih, const ih_rect* rects_dev, size_t n, uint32_t* hists,
                    uint32_t* bad_count, bool binmajor)
{
    if (ih_status st = check_view(ih)) return st;
    if (n == 0) return IH_OK;
    if (!rects_dev || !hists) return fail(IH_ERR_INVALID_ARG, "rects and hists must be non-null");
    if (n > (size_t)INT64_MAX / 256) return fail(IH_ERR_RANGE, "too many rectangles");
    hipError_t e = ih::launch_query(ih->data, ih->H, ih->W, ih->B,
                                    reinterpret_cast<const int32_t*>(rects_dev), (int64_t)n, hists,
                                    bad_count, binmajor, static_cast<hipStream_t>(ih->stream));
    if (e != hipSuccess) return hip_fail(e, "query");
    return IH_OK;
}

}  // namespace

extern "C" {

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

const char* ih_version(void) { return "ih 0.2 (gfx950)"; }

ih_status ih_compute(const uint8_t* frame, int32_t H, int32_t W, int32_t B,
                     uint32_t* out, ih_stream_t stream)
{
    if (!frame || !out) return fail(IH_ERR_INVALID_ARG, "frame and out must be non-null");
    if (ih_status st = ih::check_shape(H, W, B)) return st;
    if (reinterpret_cast<uintptr_t>(out) & 3u) return fail(IH_ERR_INVALID_ARG, "out must be 4-byte aligned");

    const ih::TileChoice t = ih::default_tile(H, W, B);
    const ih::Geom g = ih::make_geom(H, W, B, t);
    const ih::ScratchLayout sl = ih::scratch_layout(g);
    void* scratch = nullptr;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (ih_status st = get_scratch(s, sl.words * sizeof(uint32_t), &scratch)) return st;
    return enqueue_frame(frame, out, static_cast<uint32_t*>(scratch), g, t.nontemporal, s);
}

ih_status ih_compute_binmajor(const uint8_t* frame, int32_t H, int32_t W, int32_t B, uint32_t* out,
                              ih_stream_t stream)
{
    if (!frame || !out) return fail(IH_ERR_INVALID_ARG, "frame and out must be non-null");
    if (ih_status st = ih::check_shape(H, W, B)) return st;
    if (reinterpret_cast<uintptr_t>(out) & 3u) return fail(IH_ERR_INVALID_ARG, "out must be 4-byte aligned");
    const ih::Geom g = ih::make_geom(H, W, B, ih::binmajor_tile(H, W, B));
    void* scratch = nullptr;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (ih_status st = get_scratch(s, ih::scratch_layout(g).words * sizeof(uint32_t), &scratch)) return st;
    const ih::FrameArgs fa = ih::frame_args(frame, out, static_cast<uint32_t*>(scratch), g);
    ih::PhaseTimer timer;
    for (int ph = 0; ph < ih::kNumPhases; ++ph) {
        if (ih_status st = timer.begin(ph, s)) return st;
        hipError_t e = ph == static_cast<int>(ih::Phase::kTile) ? ih::launch_tile_bm(fa, s)
                                                                : ih::launch_phase(static_cast<ih::Phase>(ph), fa, false, s);
        if (e != hipSuccess) return hip_fail(e, "kernel launch");
        if (ih_status st = timer.end(s)) return st;
    }
    if (ih::profiling_on()) ih::profiling_add_frames(1);
    return IH_OK;
}

ih_status ih_compute_lut(const uint8_t* frame, int32_t H, int32_t W, int32_t B, const uint8_t* lut_host,
                         uint32_t* out, ih_stream_t stream)
{
    if (!frame || !out || !lut_host) return fail(IH_ERR_INVALID_ARG, "frame, lut and out must be non-null");
    if (ih_status st = ih::check_shape(H, W, B)) return st;
    if (reinterpret_cast<uintptr_t>(out) & 3u) return fail(IH_ERR_INVALID_ARG, "out must be 4-byte aligned");
    for (int v = 0; v < 256; ++v)
        if ((int32_t)lut_host[v] >= B)
            return fail(IH_ERR_INVALID_ARG, "lut[%d]=%d is not a bin below B=%d", v, lut_host[v], B);
    const ih::TileChoice t = ih::default_tile(H, W, B);
    const ih::Geom g = ih::make_geom(H, W, B, t);
    const size_t carry_bytes = (ih::scratch_layout(g).words * sizeof(uint32_t) + 255) / 256 * 256;
    void* scratch = nullptr;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (ih_status st = get_scratch(s, carry_bytes + 256, &scratch)) return st;
    uint32_t* dlut = reinterpret_cast<uint32_t*>(static_cast<unsigned char*>(scratch) + carry_bytes);
    // the table goes into this stream's scratch in stream order, after the
    // kernels of earlier calls that read the previous table
    hipError_t e = ih::launch_lut_store(lut_host, dlut, s);
    if (e != hipSuccess) return hip_fail(e, "bin table upload");
    return enqueue_frame(frame, out, static_cast<uint32_t*>(scratch), g, t.nontemporal, s,
                         reinterpret_cast<const uint8_t*>(dlut), ih::lut_is_general(lut_host));
}

ih_status ih_write_reference(uint32_t* out, int32_t H, int32_t W, int32_t B, int32_t tile_x, int32_t tile_y,
                             ih_stream_t stream)
{
    if (!out) return fail(IH_ERR_INVALID_ARG, "out must be non-null");
    if (ih_status st = ih::check_shape(H, W, B)) return st;
    if (B > 64) return fail(IH_ERR_INVALID_ARG, "the write reference takes B <= 64 (one bin per lane)");
    if (tile_x != 32 && tile_x != 64 && tile_x != 128) return fail(IH_ERR_INVALID_ARG, "tile_x must be 32, 64 or 128");
    if (tile_y < 1) return fail(IH_ERR_INVALID_ARG, "tile_y must be >= 1");
    if (reinterpret_cast<uintptr_t>(out) & 3u) return fail(IH_ERR_INVALID_ARG, "out must be 4-byte aligned");
    hipError_t e = ih::launch_write_reference(out, H, W, B, tile_x, tile_y, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return IH_OK;
}

ih_status ih_query(const ih_view* ih, const ih_rect* rects, size_t n, uint32_t* hists)
{
    return query_host(ih, rects, n, hists, false);
}

ih_status ih_query_device(const ih_view* ih, const ih_rect* rects_dev, size_t n,
                          uint32_t* hists, uint32_t* bad_count)
{
    return query_dev(ih, rects_dev, n, hists, bad_count, false);
}

ih_status ih_query_binmajor(const ih_view* ih, const ih_rect* rects, size_t n, uint32_t* hists)
{
    return query_host(ih, rects, n, hists, true);
}

ih_status ih_query_binmajor_device(const ih_view* ih, const ih_rect* rects_dev, size_t n,
                                   uint32_t* hists, uint32_t* bad_count)
{
    return query_dev(ih, rects_dev, n, hists, bad_count, true);
}

}  // extern "C"
