// Host-side helpers shared by the C-ABI entry points of libih: error
// reporting, argument checks and the per-phase event profiler.
#pragma once

#include "ih.h"

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ih {

// Record an error message for ih_last_error() and return st.
ih_status fail(ih_status st, const char* fmt, ...);
ih_status hip_fail(hipError_t e, const char* where);

// H, W >= 1, B in [1, 256], H*W < 2^32.
ih_status check_shape(int32_t H, int32_t W, int32_t B);

// Per-phase timing (ih_profile_enable / ih_profile_read).
bool profiling_on();
void profiling_add_frames(uint64_t n);

// Brackets one phase of work on a stream with a pair of HIP events when the
// profiler is on; a no-op otherwise.
class PhaseTimer {
public:
    ih_status begin(int phase, hipStream_t s);
    ih_status end(hipStream_t s);

private:
    hipEvent_t a_ = nullptr, b_ = nullptr;
    int phase_ = -1;
};

}  // namespace ih
