// Device-side helpers shared by the kernel sources of libih: address-space
// casts, scalar table loads, the job lookup of batched launches and the
// binning of pixel values.
#pragma once

#include "ih_internal.h"

namespace ih {

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Every buffer the kernels touch is device (global) memory.  Pointers read
// from a device table carry no address space, and accesses through them would
// compile to flat instructions, which also count against the LDS/scalar
// counter; casting to the global address space keeps them global_*.
#define IH_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ IH_GLOBAL T* gmem(T* p)
{
    return (IH_GLOBAL T*)p;
}

// The frame and job tables of a batched launch are read-only for the whole
// launch and indexed by wave-uniform values; reading them through the
// constant address space lets them come in with scalar loads, so everything
// derived from them (sizes, loop bounds, pointers) stays wave-uniform.
#define IH_CONST __attribute__((address_space(4)))
template <class T>
__device__ __forceinline__ const IH_CONST T* cmem(const T* p)
{
    return (const IH_CONST T*)p;
}
template <class T>
__device__ __forceinline__ T cload(const T* table, int64_t idx)
{
    T v;
    __builtin_memcpy(&v, cmem(table) + idx, sizeof(T));
    return v;
}

// Index of the calling wave within its workgroup.  The value is the same on
// every lane of a wave, and saying so keeps what is derived from it (work
// item, frame, loop bounds) in scalar registers.
__device__ __forceinline__ int wave_in_block()
{
    return __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
}

// Entry e of a frame's left carries (uint16 or uint32 by the frame's RC16).
__device__ __forceinline__ uint32_t left_carry(const FrameArgs& f, size_t e)
{
    if (f.g.RC16) return gmem(reinterpret_cast<const uint16_t*>(f.rowc))[e];
    return gmem(f.rowc)[e];
}

// Entry e of a frame's column carries (uint16 or uint32 by the frame's CC16).
__device__ __forceinline__ uint32_t top_carry(const FrameArgs& f, size_t e)
{
    if (f.g.CC16) return gmem(reinterpret_cast<const uint16_t*>(f.colc))[e];
    return gmem(f.colc)[e];
}

// Largest job whose `begin` is <= idx (jobs sorted by begin, jobs[0].begin == 0).
// idx is uniform across the caller's wave, so the loads stay scalar.
__device__ __forceinline__ int find_job(const IH_CONST Job* jobs, int32_t njobs, int64_t idx)
{
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].begin <= idx) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Bin of a pixel value.  A frame either uses the uniform bins floor(v B / 256)
// or a table of 256 bins, which the count kernels stage in LDS, four entries
// per word.
__device__ __forceinline__ void stage_lut(const FrameArgs& f, uint32_t* lutw, int tid, int nthreads)
{
    if (f.lut)
        for (int e = tid; e < 64; e += nthreads) lutw[e] = reinterpret_cast<const IH_GLOBAL uint32_t*>(gmem(f.lut))[e];
}
__device__ __forceinline__ uint32_t bin_of(const FrameArgs& f, const uint32_t* lutw, uint32_t v, uint32_t B)
{
    return f.lut ? (lutw[v >> 2] >> (8 * (v & 3u))) & 0xFFu : (v * B) >> 8;
}

// Entries of a non-decreasing 256-entry bin table below bin b, i.e. the first
// value of bin b (binary search in nine halving steps).
__device__ __forceinline__ uint32_t lut_count_below(const IH_GLOBAL uint8_t* lut, uint32_t b)
{
    uint32_t pos = 0;
#pragma unroll 1
    for (uint32_t step = 256; step > 0; step >>= 1)
        if (pos + step <= 256 && lut[pos + step - 1] < b) pos += step;
    return pos;
}


}  // namespace ih
