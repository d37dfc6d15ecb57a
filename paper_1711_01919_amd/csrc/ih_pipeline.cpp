// Host-transfer pipeline (Sec. 4.4, Algorithm 6): frames in host memory go to
// the device, through the three phases, and their whole integral histograms
// come back to host memory, with the copies and kernels of consecutive frames
// overlapped on several HIP streams (two streams = the paper's double
// buffering).  Every step of the method runs in the same kernels as
// ih_compute; this file only orders copies and launches.
#include "ih.h"
#include "ih_internal.h"
#include "ih_util.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

namespace {

using ih::fail;
using ih::hip_fail;

// Device buffers and events of one pipeline stream.
struct Lane {
    hipStream_t s = nullptr;
    uint8_t* frame = nullptr;
    uint32_t* out = nullptr;
    uint32_t* scratch = nullptr;
};

struct PipelineState {
    std::vector<Lane> lanes;
    std::vector<hipEvent_t> ev;      // 4 per frame: before upload, after upload, after kernels, after download
    ~PipelineState()
    {
        for (Lane& l : lanes) {
            if (l.s) (void)hipStreamSynchronize(l.s);
        }
        for (Lane& l : lanes) {
            if (l.frame) (void)hipFree(l.frame);
            if (l.out) (void)hipFree(l.out);
            if (l.scratch) (void)hipFree(l.scratch);
            if (l.s) (void)hipStreamDestroy(l.s);
        }
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
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
    ps.lanes.resize((size_t)n_streams);
    hipError_t e = hipSuccess;
    for (Lane& l : ps.lanes) {
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&l.s, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&l.frame), frame_bytes);
        if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&l.out), out_bytes);
        if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&l.scratch), scratch_bytes < 256 ? 256 : scratch_bytes);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(IH_ERR_OOM, "pipeline buffers: %s", hipGetErrorString(e));
    }
    const bool timed = stats != nullptr;
    if (timed) {
        ps.ev.resize(4 * n, nullptr);
        for (hipEvent_t& ev : ps.ev)
            if (e == hipSuccess) e = hipEventCreate(&ev);
        if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    }

    // Frame k runs on lane k mod n_streams: its upload waits for that lane's
    // previous download (stream order), and the other lanes' copies and
    // kernels proceed meanwhile.
    for (size_t k = 0; k < n && e == hipSuccess; ++k) {
        Lane& l = ps.lanes[k % ps.lanes.size()];
        hipEvent_t* ev = timed ? &ps.ev[4 * k] : nullptr;
        if (timed) e = hipEventRecord(ev[0], l.s);
        if (e == hipSuccess) e = hipMemcpyAsync(l.frame, frames_host[k], frame_bytes, hipMemcpyHostToDevice, l.s);
        if (e == hipSuccess && timed) e = hipEventRecord(ev[1], l.s);
        const ih::FrameArgs fa = ih::frame_args(l.frame, l.out, l.scratch, g);
        for (int ph = 0; e == hipSuccess && ph < ih::kNumPhases; ++ph)
            e = ih::launch_phase(static_cast<ih::Phase>(ph), fa, t.nontemporal, l.s);
        if (e == hipSuccess && timed) e = hipEventRecord(ev[2], l.s);
        if (e == hipSuccess) e = hipMemcpyAsync(outs_host[k], l.out, out_bytes, hipMemcpyDeviceToHost, l.s);
        if (e == hipSuccess && timed) e = hipEventRecord(ev[3], l.s);
    }
    if (e != hipSuccess) return hip_fail(e, "pipeline enqueue");
    for (Lane& l : ps.lanes) {
        e = hipStreamSynchronize(l.s);
        if (e != hipSuccess) return hip_fail(e, "pipeline");
    }
    if (timed) {
        ih_pipeline_stats st{};
        // wall: earliest upload start (among each lane's first frame) to the
        // latest download end (among each lane's last frame), on frame 0's clock
        const size_t m = std::min(n, ps.lanes.size());
        double t0 = 0.0, t1 = 0.0;
        for (size_t k = 0; k < m; ++k) t0 = std::min(t0, (double)elapsed(ps.ev[0], ps.ev[4 * k]));
        for (size_t k = n - m; k < n; ++k) t1 = std::max(t1, (double)elapsed(ps.ev[0], ps.ev[4 * k + 3]));
        st.wall_ms = t1 - t0;
        for (size_t k = 0; k < n; ++k) {
            st.h2d_ms += elapsed(ps.ev[4 * k], ps.ev[4 * k + 1]);
            st.kernel_ms += elapsed(ps.ev[4 * k + 1], ps.ev[4 * k + 2]);
            st.d2h_ms += elapsed(ps.ev[4 * k + 2], ps.ev[4 * k + 3]);
        }
        st.frames_per_s = st.wall_ms > 0.0 ? (double)n / (st.wall_ms / 1e3) : 0.0;
        *stats = st;
    }
    return IH_OK;
}

}  // extern "C"
