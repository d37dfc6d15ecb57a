// Host-transfer pipeline (Sec. 4.4, Algorithm 6): frames in host memory go to
// the device, through the three phases, and their whole integral histograms
// come back to host memory, with the copies and kernels of consecutive frames
// overlapped (two buffer slots = the paper's double buffering).  Every step of
// the method runs in the same kernels as ih_compute; this file only orders
// copies and launches.
#include "ih.h"
#include "ih_internal.h"
#include "ih_util.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

namespace {

using ih::fail;
using ih::hip_fail;

// Device buffers of one slot: frame k uses slot k mod n_slots.
struct Slot {
    uint8_t* frame = nullptr;
    uint32_t* out = nullptr;
    uint32_t* scratch = nullptr;
};

// Uploads and kernels run in frame order on the compute stream, downloads in
// frame order on the copy stream: one download at a time keeps the
// device-to-host link at full rate, and the next frames' uploads and kernels
// proceed beside it.  Events order the two streams.
struct PipelineState {
    hipStream_t compute = nullptr, copy = nullptr;
    std::vector<Slot> slots;
    std::vector<hipEvent_t> computed;   // per frame: its kernels finished (compute stream)
    std::vector<hipEvent_t> copied;     // per frame: its download finished (copy stream)
    std::vector<hipEvent_t> ev;         // timing, 4 per frame: before upload, after upload, after kernels
                                        // (compute stream), before download (copy stream); copied[] ends it
    ~PipelineState()
    {
        if (compute) (void)hipStreamSynchronize(compute);
        if (copy) (void)hipStreamSynchronize(copy);
        for (Slot& l : slots) {
            if (l.frame) (void)hipFree(l.frame);
            if (l.out) (void)hipFree(l.out);
            if (l.scratch) (void)hipFree(l.scratch);
        }
        for (hipEvent_t e : computed) (void)hipEventDestroy(e);
        for (hipEvent_t e : copied) (void)hipEventDestroy(e);
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
        if (compute) (void)hipStreamDestroy(compute);
        if (copy) (void)hipStreamDestroy(copy);
    }
};

float elapsed(hipEvent_t a, hipEvent_t b)
{
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.f;
    return ms;
}

}  // namespace

extern "C" {

ih_status ih_transfer_pipeline(const uint8_t* const* frames_host, uint32_t* const* outs_host, size_t n,
                               int32_t H, int32_t W, int32_t B, int32_t n_streams,
                               ih_pipeline_stats* stats)
{
    if (!frames_host || !outs_host) return fail(IH_ERR_INVALID_ARG, "frame and output arrays must be non-null");
    if (n == 0) return fail(IH_ERR_INVALID_ARG, "need at least one frame");
    if (n > (1u << 24)) return fail(IH_ERR_RANGE, "too many frames (%zu)", n);
    if (n_streams < 1 || n_streams > 8) return fail(IH_ERR_INVALID_ARG, "n_streams=%d must be in [1, 8]", n_streams);
    if (ih_status st = ih::check_shape(H, W, B)) return st;
    for (size_t k = 0; k < n; ++k)
        if (!frames_host[k] || !outs_host[k]) return fail(IH_ERR_INVALID_ARG, "frame %zu: null pointer", k);

    const ih::TileChoice t = ih::default_tile(H, W, B);
    const ih::Geom g = ih::make_geom(H, W, B, t);
    const size_t frame_bytes = (size_t)H * W;
    const size_t out_bytes = (size_t)H * W * B * sizeof(uint32_t);
    const size_t scratch_bytes = ih::scratch_layout(g).words * sizeof(uint32_t);

    PipelineState ps;
    ps.slots.resize((size_t)n_streams);
    hipError_t e = hipStreamCreateWithFlags(&ps.compute, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&ps.copy, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
    for (Slot& l : ps.slots) {
        if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&l.frame), frame_bytes);
        if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&l.out), out_bytes);
        if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&l.scratch), scratch_bytes < 256 ? 256 : scratch_bytes);
        // the fused schedule's arrival counters start at zero
        if (e == hipSuccess)
            e = hipMemsetAsync(l.scratch, 0, std::min(scratch_bytes, (size_t)ih::kCounterWords * 4), ps.compute);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(IH_ERR_OOM, "pipeline buffers: %s", hipGetErrorString(e));
    }
    ps.computed.assign(n, nullptr);
    ps.copied.assign(n, nullptr);
    for (size_t k = 0; k < n && e == hipSuccess; ++k) {
        e = hipEventCreateWithFlags(&ps.computed[k], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ps.copied[k], stats ? 0 : hipEventDisableTiming);
    }
    const bool timed = stats != nullptr;
    if (timed) {
        ps.ev.resize(4 * n, nullptr);
        for (hipEvent_t& ev : ps.ev)
            if (e == hipSuccess) e = hipEventCreate(&ev);
    }
    if (e != hipSuccess) return hip_fail(e, "hipEventCreate");

    // Breadth first, in frame order: frame k's upload waits (on the compute
    // stream) for the download of the frame that used its slot before, its
    // kernels follow the upload, and its download waits (on the copy stream)
    // for its kernels.
    const size_t ns = ps.slots.size();
    for (size_t k = 0; k < n && e == hipSuccess; ++k) {
        Slot& l = ps.slots[k % ns];
        hipEvent_t* ev = timed ? &ps.ev[4 * k] : nullptr;
        if (k >= ns) e = hipStreamWaitEvent(ps.compute, ps.copied[k - ns], 0);
        if (e == hipSuccess && timed) e = hipEventRecord(ev[0], ps.compute);
        if (e == hipSuccess) e = hipMemcpyAsync(l.frame, frames_host[k], frame_bytes, hipMemcpyHostToDevice, ps.compute);
        if (e == hipSuccess && timed) e = hipEventRecord(ev[1], ps.compute);
        const ih::FrameArgs fa = ih::frame_args(l.frame, l.out, l.scratch, g);
        for (int ph = 0; e == hipSuccess && ph < ih::kNumPhases; ++ph)
            e = ih::launch_phase(static_cast<ih::Phase>(ph), fa, t.nontemporal, ps.compute);
        if (e == hipSuccess && timed) e = hipEventRecord(ev[2], ps.compute);
        if (e == hipSuccess) e = hipEventRecord(ps.computed[k], ps.compute);
        if (e == hipSuccess) e = hipStreamWaitEvent(ps.copy, ps.computed[k], 0);
        if (e == hipSuccess && timed) e = hipEventRecord(ev[3], ps.copy);
        if (e == hipSuccess) e = hipMemcpyAsync(outs_host[k], l.out, out_bytes, hipMemcpyDeviceToHost, ps.copy);
        if (e == hipSuccess) e = hipEventRecord(ps.copied[k], ps.copy);
    }
    if (e != hipSuccess) return hip_fail(e, "pipeline enqueue");
    e = hipStreamSynchronize(ps.compute);
    if (e == hipSuccess) e = hipStreamSynchronize(ps.copy);
    if (e != hipSuccess) return hip_fail(e, "pipeline");
    if (timed) {
        ih_pipeline_stats st{};
        // wall: first upload start to last download end
        st.wall_ms = elapsed(ps.ev[0], ps.copied[n - 1]);
        for (size_t k = 0; k < n; ++k) {
            st.h2d_ms += elapsed(ps.ev[4 * k], ps.ev[4 * k + 1]);
            st.kernel_ms += elapsed(ps.ev[4 * k + 1], ps.ev[4 * k + 2]);
            st.d2h_ms += elapsed(ps.ev[4 * k + 3], ps.copied[k]);
        }
        st.frames_per_s = st.wall_ms > 0.0 ? (double)n / (st.wall_ms / 1e3) : 0.0;
        *stats = st;
    }
    return IH_OK;
}

}  // extern "C"
