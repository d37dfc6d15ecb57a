// Allocation-free form of ih_compute: the same tile choice and the same
// kernels, with the carries in a fixed device array of this library instead
// of the per-stream scratch cache, so a call never allocates device memory.
//
// The array is a file-scope __device__ variable: every GPU the library runs
// on holds its own copy, at its own address, until the process ends.  In
// host code its name is only a host-side handle; the device address of the
// current GPU's copy comes from hipGetSymbolAddress, taken once per device at
// the first call on it, and only that address is ever passed to kernels.
#include "ih.h"
#include "ih_internal.h"
#include "ih_util.h"

#include <hip/hip_runtime.h>

#include <mutex>

// IH_NOALLOC_SCRATCH_BYTES (64 MiB) of carries: enough for ih_compute's
// tiles of every frame up to 3840 x 2160 pixels at B <= 64 (at most 59.8 MiB,
// for 2160 x 3584); the carries are about 1/TX + 1/TY of the output.
static constexpr size_t kNoAllocWords = IH_NOALLOC_SCRATCH_BYTES / sizeof(uint32_t);
static __device__ __align__(256) uint32_t scratch[kNoAllocWords];

namespace {

using ih::fail;
using ih::hip_fail;

constexpr int kMaxDevices = 64;

struct NoAllocState {
    std::mutex mu;
    uint32_t* ptr[kMaxDevices] = {};
};
NoAllocState& state()
{
    static NoAllocState* s = new NoAllocState;   // never destroyed: lives as long as the arrays
    return *s;
}

// Device address of the current GPU's array, looked up on its first use.
ih_status scratch_ptr(uint32_t** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(IH_ERR_INVALID_ARG, "device %d is beyond the %d supported", dev, kMaxDevices);
    NoAllocState& s = state();
    std::lock_guard<std::mutex> lock(s.mu);
    if (!s.ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(IH_ERR_HIP, "hipGetSymbolAddress(scratch) returned null");
        s.ptr[dev] = static_cast<uint32_t*>(p);
    }
    *out = s.ptr[dev];
    return IH_OK;
}

// Zero the first n words of the array: the fused carry schedule's arrival
// counters.  A kernel, not a memset, so the call can be captured in a graph.
__global__ __launch_bounds__(256) void clear_words_kernel(uint32_t* p, int32_t n)
{
    const int32_t i = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < n) p[i] = 0u;
}

}  // namespace

extern "C" {

ih_status ih_compute_noalloc(const uint8_t* frame, int32_t H, int32_t W, int32_t B, uint32_t* out,
                             ih_stream_t stream)
{
    if (!frame || !out) return fail(IH_ERR_INVALID_ARG, "frame and out must be non-null");
    if (ih_status st = ih::check_shape(H, W, B)) return st;
    if (reinterpret_cast<uintptr_t>(out) & 3u) return fail(IH_ERR_INVALID_ARG, "out must be 4-byte aligned");

    const ih::TileChoice t = ih::default_tile(H, W, B);
    const ih::Geom g = ih::make_geom(H, W, B, t);
    const ih::ScratchLayout sl = ih::scratch_layout(g);
    if (sl.words > kNoAllocWords)
        return fail(IH_ERR_RANGE, "a %dx%d frame with B=%d needs %zu carry bytes; the allocation-free form holds %zu",
                    H, W, B, sl.words * sizeof(uint32_t), kNoAllocWords * sizeof(uint32_t));

    uint32_t* buf = nullptr;
    if (ih_status st = scratch_ptr(&buf)) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (g.K) {
        const int32_t n = g.nTX + g.nS;
        hipLaunchKernelGGL(clear_words_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, buf, n);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "kernel launch");
    }
    const ih::FrameArgs fa = ih::frame_args(frame, out, buf, g);
    for (int ph = 0; ph < ih::kNumPhases; ++ph) {
        hipError_t e = ih::launch_phase(static_cast<ih::Phase>(ph), fa, t.nontemporal, s);
        if (e != hipSuccess) return hip_fail(e, "kernel launch");
    }
    return IH_OK;
}

}  // extern "C"
