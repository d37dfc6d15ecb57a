// Batched integral histograms: many frames of uneven size and bin count in
// one launch per phase, captured in a hipGraph, with an autotuner that picks
// the tile shape and store flavour per (H, W, B) class by timing candidates.
#include "ih.h"
#include "ih_internal.h"
#include "ih_launch.h"
#include "ih_util.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <tuple>
#include <vector>

namespace {

using ih::fail;
using ih::hip_fail;

}  // namespace

struct ih_batch_plan {
    int device = 0;
    std::vector<ih_frame_desc> descs;
    std::vector<ih::TileChoice> tiles;
    void* d_scratch = nullptr;
    void* d_image = nullptr;
    ih::BatchImage image;
    bool use_graph = true;
    hipGraphExec_t exec_all = nullptr;
    hipGraphExec_t exec_phase[ih::kNumPhases] = {nullptr, nullptr, nullptr};
    int64_t entries = 0;
};

namespace {

// Enqueue the launches of the given phase (-1: all), in order.
hipError_t enqueue(const ih_batch_plan* p, int phase, hipStream_t s)
{
    return ih::enqueue_batch(p->image, p->d_image, phase, s);
}

void free_plan(ih_batch_plan* p)
{
    if (!p) return;
    if (p->exec_all) (void)hipGraphExecDestroy(p->exec_all);
    for (auto& e : p->exec_phase)
        if (e) (void)hipGraphExecDestroy(e);
    if (p->d_image) (void)hipFree(p->d_image);
    if (p->d_scratch) (void)hipFree(p->d_scratch);
    delete p;
}

// Lay out scratch, build the launch image and upload it.  Frames keep the
// order given; tiles[k] is frame k's tile choice.
ih_status build_plan(ih_batch_plan* p)
{
    const size_t n = p->descs.size();
    std::vector<size_t> off(n);
    std::vector<ih::Geom> geoms(n);
    size_t words = 0;
    for (size_t k = 0; k < n; ++k) {
        const ih_frame_desc& d = p->descs[k];
        geoms[k] = ih::make_geom(d.H, d.W, d.B, p->tiles[k]);
        off[k] = words;
        words += ih::frame_scratch_words(geoms[k]);
        p->entries += (int64_t)d.H * d.W * d.B;
    }
    hipError_t e = hipMalloc(&p->d_scratch, std::max<size_t>(words * 4, 256));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(IH_ERR_OOM, "batch scratch of %zu bytes: %s", words * 4, hipGetErrorString(e));
    }
    std::vector<ih::FrameArgs> frames(n);
    std::vector<char> nt(n);
    for (size_t k = 0; k < n; ++k) {
        frames[k] = ih::frame_args(p->descs[k].frame, p->descs[k].out,
                                   static_cast<uint32_t*>(p->d_scratch) + off[k], geoms[k]);
        nt[k] = p->tiles[k].nontemporal ? 1 : 0;
    }
    ih::build_batch_image(frames, nt, &p->image);
    e = hipMalloc(&p->d_image, p->image.bytes());
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(IH_ERR_OOM, "batch tables: %s", hipGetErrorString(e));
    }
    e = hipMemcpy(p->d_image, p->image.host.data(), p->image.bytes(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "upload batch tables");
    return IH_OK;
}

ih_status capture(ih_batch_plan* p, int phase, hipGraphExec_t* out)
{
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
    hipGraph_t graph = nullptr;
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t e1 = enqueue(p, phase, cs);
        hipError_t e2 = hipStreamEndCapture(cs, &graph);
        e = e1 != hipSuccess ? e1 : e2;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) return hip_fail(e, "graph capture");
    return IH_OK;
}

// ---------------------------------------------------------------------------
// autotuner
// ---------------------------------------------------------------------------
struct TuneKey {
    int32_t H, W, B;
    int32_t nb;          // frames of the class, as floor(log2(n)): tiles depend on the parallelism
    bool operator<(const TuneKey& o) const { return std::tie(H, W, B, nb) < std::tie(o.H, o.W, o.B, o.nb); }
};

int32_t log2_floor(size_t n)
{
    int32_t r = 0;
    while (n > 1) { n >>= 1; ++r; }
    return r;
}

struct TuneCache {
    std::mutex mu;
    std::map<TuneKey, ih::TileChoice> best;
    bool loaded = false;
};
TuneCache& tune_cache()
{
    static TuneCache* c = new TuneCache;
    return *c;
}

const char* cache_path() { return std::getenv("IH_AUTOTUNE_CACHE"); }

// The cache file holds one line per class: "gfx950 H W B NB TX TY NT".
void load_cache(TuneCache& c)
{
    if (c.loaded) return;
    c.loaded = true;
    const char* path = cache_path();
    if (!path) return;
    std::ifstream in(path);
    std::string arch;
    int H, W, B, NB, TX, TY, NT;
    while (in >> arch >> H >> W >> B >> NB >> TX >> TY >> NT) {
        if (arch != "gfx950") continue;
        ih::TileChoice t{TX, TY, NT != 0};
        if (ih::tile_supported(B, t)) c.best[TuneKey{H, W, B, NB}] = t;
    }
}

void save_cache(TuneCache& c)
{
    const char* path = cache_path();
    if (!path) return;
    std::ofstream out(path);
    for (auto& kv : c.best)
        out << "gfx950 " << kv.first.H << ' ' << kv.first.W << ' ' << kv.first.B << ' ' << kv.first.nb << ' ' << kv.second.TX
            << ' ' << kv.second.TY << ' ' << (kv.second.nontemporal ? 1 : 0) << '\n';
}

std::vector<ih::TileChoice> candidates(int32_t B)
{
    std::vector<ih::TileChoice> c;
    for (int tx : {32, 64, 128})
        for (int ty : {16, 32, 64, 128, 256})
            for (bool nt : {false, true}) {
                ih::TileChoice t{tx, ty, nt};
                if (ih::tile_supported(B, t)) c.push_back(t);
            }
    return c;
}

// Heuristic tile for frames of one bin count launched together: the tallest
// band (fewest carries) that still leaves at least 8192 independent waves
// across all of the frames.  For B = 64, 128-wide tiles (half the left-carry
// reads per stored byte) when a band of at least 64 rows still gives that
// many waves; otherwise the single-frame tile width.
ih::TileChoice batch_default_tile(const std::vector<ih_frame_desc>& descs, int32_t B)
{
    constexpr int64_t kMinWaves = 8192;
    auto waves_of = [&](int tx, int ty) {
        int64_t w = 0;
        for (const ih_frame_desc& d : descs) {
            const ih::Geom g = ih::make_geom(d.H, d.W, d.B, ih::TileChoice{tx, ty, false});
            w += (int64_t)g.nTY * g.nJG;
        }
        return w;
    };
    ih::TileChoice t = ih::default_tile(descs[0].H, descs[0].W, B);
    if (ih::tile_supported(B, ih::TileChoice{128, 64, false}) && waves_of(128, 64) >= kMinWaves)
        t.TX = 128;
    for (int ty : {256, 128, 64, 32, 16}) {
        t.TY = ty;
        if (waves_of(t.TX, ty) >= kMinWaves) break;
    }
    return t;
}

// Time one candidate on the frames of a class (all phases, no graph).
ih_status time_candidate(const std::vector<ih_frame_desc>& descs, const ih::TileChoice& t,
                         hipStream_t s, float* ms)
{
    ih_batch_plan* p = new ih_batch_plan;
    p->descs = descs;
    p->tiles.assign(descs.size(), t);
    p->use_graph = false;
    ih_status st = build_plan(p);
    hipEvent_t a = nullptr, b = nullptr;
    if (st == IH_OK) {
        hipError_t e = hipEventCreate(&a);
        if (e == hipSuccess) e = hipEventCreate(&b);
        if (e == hipSuccess) e = enqueue(p, -1, s);                      // warm-up
        std::vector<float> runs;
        for (int r = 0; r < 5 && e == hipSuccess; ++r) {
            e = hipEventRecord(a, s);
            if (e == hipSuccess) e = enqueue(p, -1, s);
            if (e == hipSuccess) e = hipEventRecord(b, s);
            if (e == hipSuccess) e = hipEventSynchronize(b);
            float m = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&m, a, b);
            runs.push_back(m);
        }
        std::sort(runs.begin(), runs.end());
        *ms = runs.empty() ? 1e30f : runs[runs.size() / 2];
        if (e != hipSuccess) st = hip_fail(e, "autotune run");
    }
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (p->d_scratch || p->d_image) (void)hipDeviceSynchronize();
    free_plan(p);
    return st;
}

// The class's frames measured alone: the heuristic tile first, then every
// candidate; a candidate replaces the incumbent only when its median time is
// more than 2% lower, so timing noise does not flip the choice.
ih_status autotune(ih_batch_plan* p, hipStream_t s)
{
    std::map<TuneKey, std::vector<size_t>> classes;
    for (size_t k = 0; k < p->descs.size(); ++k)
        classes[TuneKey{p->descs[k].H, p->descs[k].W, p->descs[k].B, 0}].push_back(k);
    TuneCache& c = tune_cache();
    std::lock_guard<std::mutex> lock(c.mu);
    load_cache(c);
    bool dirty = false;
    for (auto& kv : classes) {
        TuneKey key = kv.first;
        key.nb = log2_floor(kv.second.size());
        auto hit = c.best.find(key);
        if (hit == c.best.end()) {
            std::vector<ih_frame_desc> descs;
            for (size_t k : kv.second) descs.push_back(p->descs[k]);
            ih::TileChoice best = batch_default_tile(descs, kv.first.B);
            float best_ms = 1e30f;
            if (ih_status st = time_candidate(descs, best, s, &best_ms)) return st;
            for (const ih::TileChoice& t : candidates(kv.first.B)) {
                if (t.TX == best.TX && t.TY == best.TY && t.nontemporal == best.nontemporal) continue;
                float ms = 0.f;
                if (ih_status st = time_candidate(descs, t, s, &ms)) return st;
                if (ms < 0.98f * best_ms) { best_ms = ms; best = t; }
            }
            hit = c.best.emplace(key, best).first;
            dirty = true;
        }
        for (size_t k : kv.second) p->tiles[k] = hit->second;
    }
    if (dirty) save_cache(c);
    return IH_OK;
}

}  // namespace

extern "C" {

ih_status ih_batch_plan_create(const ih_frame_desc* frames, size_t n, const ih_batch_options* opt,
                               ih_stream_t stream, ih_batch_plan** plan)
{
    if (!plan) return fail(IH_ERR_INVALID_ARG, "plan must be non-null");
    *plan = nullptr;
    if (n == 0 || !frames) return fail(IH_ERR_INVALID_ARG, "need at least one frame");
    if (n > (1u << 20)) return fail(IH_ERR_RANGE, "too many frames (%zu)", n);
    ih_batch_options o{0, 1, 0, 0, -1};
    if (opt) o = *opt;
    const bool forced = o.tile_x > 0 || o.tile_y > 0;
    for (size_t k = 0; k < n; ++k) {
        const ih_frame_desc& d = frames[k];
        if (!d.frame || !d.out) return fail(IH_ERR_INVALID_ARG, "frame %zu: null pointer", k);
        if (ih_status st = ih::check_shape(d.H, d.W, d.B)) return st;
        if (reinterpret_cast<uintptr_t>(d.out) & 3u) return fail(IH_ERR_INVALID_ARG, "frame %zu: out misaligned", k);
        if (forced && !ih::tile_supported(d.B, ih::TileChoice{o.tile_x, o.tile_y, false}))
            return fail(IH_ERR_INVALID_ARG, "tile %dx%d not supported for B=%d", o.tile_x, o.tile_y, d.B);
    }
    ih_batch_plan* p = new ih_batch_plan;
    (void)hipGetDevice(&p->device);
    p->descs.assign(frames, frames + n);
    p->use_graph = o.use_graph != 0;
    p->tiles.resize(n);
    hipStream_t s = static_cast<hipStream_t>(stream);
    ih_status st = IH_OK;
    if (forced) {
        for (size_t k = 0; k < n; ++k) p->tiles[k] = ih::TileChoice{o.tile_x, o.tile_y, false};
    } else if (o.autotune) {
        st = autotune(p, s);
    } else {
        std::map<int32_t, std::vector<ih_frame_desc>> by_b;
        for (size_t k = 0; k < n; ++k) by_b[frames[k].B].push_back(frames[k]);
        std::map<int32_t, ih::TileChoice> choice;
        for (auto& kv : by_b) choice[kv.first] = batch_default_tile(kv.second, kv.first);
        for (size_t k = 0; k < n; ++k) p->tiles[k] = choice[frames[k].B];
    }
    if (st == IH_OK && o.nontemporal >= 0)
        for (auto& t : p->tiles) t.nontemporal = o.nontemporal != 0;
    if (st == IH_OK) st = build_plan(p);
    if (st == IH_OK && p->use_graph) {
        st = capture(p, -1, &p->exec_all);
        for (int ph = 0; st == IH_OK && ph < ih::kNumPhases; ++ph) st = capture(p, ph, &p->exec_phase[ph]);
    }
    if (st != IH_OK) {
        free_plan(p);
        return st;
    }
    *plan = p;
    return IH_OK;
}

ih_status ih_batch_plan_launch(ih_batch_plan* p, ih_stream_t stream)
{
    if (!p) return fail(IH_ERR_INVALID_ARG, "plan must be non-null");
    hipStream_t s = static_cast<hipStream_t>(stream);
    ih::PhaseTimer timer;
    const bool prof = ih::profiling_on();
    if (!prof) {
        hipError_t e = p->use_graph ? hipGraphLaunch(p->exec_all, s) : enqueue(p, -1, s);
        if (e != hipSuccess) return hip_fail(e, "batch launch");
        return IH_OK;
    }
    for (int ph = 0; ph < ih::kNumPhases; ++ph) {
        if (ih_status st = timer.begin(ph, s)) return st;
        hipError_t e = p->use_graph ? hipGraphLaunch(p->exec_phase[ph], s) : enqueue(p, ph, s);
        if (e != hipSuccess) return hip_fail(e, "batch launch");
        if (ih_status st = timer.end(s)) return st;
    }
    ih::profiling_add_frames((uint64_t)p->descs.size());
    return IH_OK;
}

ih_status ih_batch_plan_destroy(ih_batch_plan* p)
{
    if (!p) return IH_OK;
    hipError_t e = hipDeviceSynchronize();
    free_plan(p);
    if (e != hipSuccess) return hip_fail(e, "synchronize before destroy");
    return IH_OK;
}

ih_status ih_batch_plan_info(const ih_batch_plan* p, ih_batch_info* info)
{
    if (!p || !info) return fail(IH_ERR_INVALID_ARG, "plan and info must be non-null");
    info->frames = (int64_t)p->descs.size();
    info->entries = p->entries;
    info->kernel_launches = (int32_t)p->image.launches.size();
    info->graph = p->use_graph ? 1 : 0;
    int32_t tile_launches = 0;
    for (const ih::BatchLaunch& l : p->image.launches) tile_launches += l.kind == ih::BatchLaunch::kTile;
    info->tile_launches = tile_launches;
    return IH_OK;
}

ih_status ih_batch_plan_frame_tile(const ih_batch_plan* p, size_t k, int32_t* tile_x, int32_t* tile_y,
                                   int32_t* nontemporal)
{
    if (!p || k >= p->descs.size() || !tile_x || !tile_y || !nontemporal)
        return fail(IH_ERR_INVALID_ARG, "bad plan, index or output pointer");
    *tile_x = p->tiles[k].TX;
    *tile_y = p->tiles[k].TY;
    *nontemporal = p->tiles[k].nontemporal ? 1 : 0;
    return IH_OK;
}

}  // extern "C"
