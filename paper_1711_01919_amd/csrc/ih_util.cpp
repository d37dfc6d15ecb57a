// Host-side helpers of libih: error text, argument checks, event profiler.
#include "ih_util.h"
#include "ih_internal.h"

#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <mutex>
#include <string>
#include <vector>

namespace ih {

namespace {
thread_local std::string g_last_error;

struct Profiler {
    std::mutex mu;
    std::atomic<bool> on{false};
    struct Rec { hipEvent_t a, b; int phase; };
    std::vector<Rec> pending;
    std::vector<hipEvent_t> pool;
    double ms[kNumPhases] = {0, 0, 0};
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
    static Profiler* p = new Profiler;   // never destroyed: lives for the process
    return *p;
}
}  // namespace

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

ih_status check_shape(int32_t H, int32_t W, int32_t B)
{
    if (H <= 0 || W <= 0) return fail(IH_ERR_INVALID_ARG, "H=%d and W=%d must be >= 1", H, W);
    if (B < 1 || B > 256) return fail(IH_ERR_INVALID_ARG, "B=%d must be in [1, 256]", B);
    if ((uint64_t)H * (uint64_t)W >= (1ull << 32))
        return fail(IH_ERR_RANGE, "H*W=%llu must be below 2^32",
                    (unsigned long long)H * (unsigned long long)W);
    return IH_OK;
}

bool profiling_on() { return profiler().on.load(); }

void profiling_add_frames(uint64_t n)
{
    Profiler& p = profiler();
    std::lock_guard<std::mutex> lock(p.mu);
    p.frames += n;
}

ih_status PhaseTimer::begin(int phase, hipStream_t s)
{
    Profiler& p = profiler();
    if (!p.on.load()) return IH_OK;
    std::lock_guard<std::mutex> lock(p.mu);
    a_ = p.get();
    b_ = p.get();
    if (!a_ || !b_) return fail(IH_ERR_HIP, "hipEventCreate failed");
    phase_ = phase;
    hipError_t e = hipEventRecord(a_, s);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    return IH_OK;
}

ih_status PhaseTimer::end(hipStream_t s)
{
    if (phase_ < 0) return IH_OK;
    Profiler& p = profiler();
    std::lock_guard<std::mutex> lock(p.mu);
    hipError_t e = hipEventRecord(b_, s);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    p.pending.push_back(Profiler::Rec{a_, b_, phase_});
    phase_ = -1;
    return IH_OK;
}

}  // namespace ih

extern "C" {

const char* ih_last_error(void) { return ih::g_last_error.c_str(); }

ih_status ih_profile_enable(int on)
{
    ih::Profiler& p = ih::profiler();
    std::lock_guard<std::mutex> lock(p.mu);
    hipError_t e = p.drain();
    if (e != hipSuccess) return ih::hip_fail(e, "profile drain");
    p.on.store(on != 0);
    for (double& m : p.ms) m = 0;
    p.frames = 0;
    return IH_OK;
}

ih_status ih_profile_read(ih_phase_times* t)
{
    if (!t) return ih::fail(IH_ERR_INVALID_ARG, "t must be non-null");
    ih::Profiler& p = ih::profiler();
    std::lock_guard<std::mutex> lock(p.mu);
    hipError_t e = p.drain();
    if (e != hipSuccess) return ih::hip_fail(e, "profile drain");
    t->agg_ms = p.ms[0];
    t->scan_ms = p.ms[1];
    t->tile_ms = p.ms[2];
    t->frames = p.frames;
    return IH_OK;
}

}  // extern "C"
