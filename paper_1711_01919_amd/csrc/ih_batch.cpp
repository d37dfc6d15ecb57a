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

// Graph branches of the tile pass: at most kMaxTileBranches (the hardware
// queues a process gets by default), kDefaultTileBranches when the caller
// leaves the choice (the 256-frame uneven batch, 12 tile-pass launches:
// 25.48 ms per launch on one branch, 24.35 on two, 24.28 on three, 23.78 on
// four).
constexpr int32_t kMaxTileBranches = 4;
constexpr int32_t kDefaultTileBranches = 4;

}  // namespace

// A pipeline group: consecutive frames of the plan with their own launch
// image (job tables indexed by the group's frames).
struct PlanGroup {
    ih::BatchImage image;
    size_t dev_off = 0;         // byte offset of the image in the plan's device tables
    size_t frames = 0;          // consecutive frames of the plan in this group
};

struct ih_batch_plan {
    int device = 0;
    std::vector<ih_frame_desc> descs;
    std::vector<ih::TileChoice> tiles;
    void* d_scratch = nullptr;
    void* d_image = nullptr;
    std::vector<uint8_t> luts;            // copies of the frames' bin tables, 256 bytes each (any entries < B)
    std::vector<int32_t> lut_index;       // per frame: index into luts, or -1 (uniform bins)
    void* d_luts = nullptr;
    ih::BatchImage image;                 // one group: every frame
    std::vector<PlanGroup> groups;        // two or more: the pipelined form
    int64_t group_bytes = 0;              // requested (options), resolved at build
    hipStream_t side = nullptr;           // pipelined form: carry phases run here
    std::vector<hipEvent_t> ev_carry, ev_tile;
    hipEvent_t ev_start = nullptr;
    bool use_graph = true;
    hipGraphExec_t exec_all = nullptr;
    hipGraphExec_t exec_phase[ih::kNumPhases] = {nullptr, nullptr, nullptr};
    int64_t entries = 0;
    hipStream_t stream = nullptr;         // creation stream (clears scratch, runs the autotuner)
    hipEvent_t ev_done = nullptr;         // recorded after each launch; destroy waits for it
    bool launched = false;
    // Tile-pass launches spread over graph branches (one group only): the
    // branch streams, the fork and join events, and (launch index, branch)
    // in enqueue order.
    int32_t tile_branches = 1;
    std::vector<hipStream_t> branch;
    std::vector<hipEvent_t> ev_branch;
    hipEvent_t ev_fork = nullptr;
    std::vector<std::pair<size_t, int>> tile_order;
};

namespace {

// Enqueue the launches of the given phase (-1: all), in order.  Not for
// pipelined plans.  With tile branches, the tile-pass launches fork from s
// after the carry phases, run on the branch streams (each launch writes
// frames of its own, so they are independent) and join s again.
hipError_t enqueue(const ih_batch_plan* p, int phase, hipStream_t s)
{
    if (p->branch.empty() || (phase != -1 && phase != 2)) return ih::enqueue_batch(p->image, p->d_image, phase, s);
    hipError_t e = hipSuccess;
    for (int ph = 0; e == hipSuccess && phase == -1 && ph < 2; ++ph) e = ih::enqueue_batch(p->image, p->d_image, ph, s);
    if (e == hipSuccess) e = hipEventRecord(p->ev_fork, s);
    for (size_t b = 0; e == hipSuccess && b < p->branch.size(); ++b) e = hipStreamWaitEvent(p->branch[b], p->ev_fork, 0);
    for (size_t q = 0; e == hipSuccess && q < p->tile_order.size(); ++q)
        e = ih::enqueue_launch(p->image, p->d_image, p->tile_order[q].first, p->branch[p->tile_order[q].second]);
    for (size_t b = 0; e == hipSuccess && b < p->branch.size(); ++b) {
        e = hipEventRecord(p->ev_branch[b], p->branch[b]);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, p->ev_branch[b], 0);
    }
    return e;
}

// Tile-pass launches over the branches: largest output first, each to the
// branch with the least output so far.
void assign_branches(ih_batch_plan* p)
{
    std::vector<size_t> tiles;
    for (size_t i = 0; i < p->image.launches.size(); ++i)
        if (ih::phase_of(p->image.launches[i]) == 2) tiles.push_back(i);
    std::stable_sort(tiles.begin(), tiles.end(), [&](size_t a, size_t b) {
        return p->image.launches[a].out_bytes > p->image.launches[b].out_bytes;
    });
    std::vector<int64_t> load(p->branch.size(), 0);
    p->tile_order.clear();
    for (size_t i : tiles) {
        const int b = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        load[b] += p->image.launches[i].out_bytes;
        p->tile_order.emplace_back(i, b);
    }
}

// The pipelined form.  Group g's carry phases run on the side stream after
// group g-1's carries and after group g-2's tile pass (so at most two groups'
// carries are live in cache); its tile pass runs on s after group g-1's tile
// pass and its own carries.  The side stream first waits for everything
// already on s, and s ends after the last group's tile pass, which follows
// every carry launch.  With timed, each phase is bracketed by events.
hipError_t enqueue_pipelined(const ih_batch_plan* p, hipStream_t s, bool timed, ih_status* tst)
{
    const unsigned char* dev = static_cast<const unsigned char*>(p->d_image);
    hipError_t e = hipEventRecord(p->ev_start, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(p->side, p->ev_start, 0);
    ih::PhaseTimer ts, tm;
    for (size_t g = 0; e == hipSuccess && g < p->groups.size(); ++g) {
        const PlanGroup& G = p->groups[g];
        if (g >= 2) e = hipStreamWaitEvent(p->side, p->ev_tile[g - 2], 0);
        for (int ph = 0; e == hipSuccess && ph < 2; ++ph) {
            if (timed && (*tst = ts.begin(ph, p->side)) != IH_OK) return hipSuccess;
            e = ih::enqueue_batch(G.image, dev + G.dev_off, ph, p->side);
            if (e == hipSuccess && timed && (*tst = ts.end(p->side)) != IH_OK) return hipSuccess;
        }
        if (e == hipSuccess) e = hipEventRecord(p->ev_carry[g], p->side);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, p->ev_carry[g], 0);
        if (e == hipSuccess && timed && (*tst = tm.begin(2, s)) != IH_OK) return hipSuccess;
        if (e == hipSuccess) e = ih::enqueue_batch(G.image, dev + G.dev_off, 2, s);
        if (e == hipSuccess && timed && (*tst = tm.end(s)) != IH_OK) return hipSuccess;
        if (e == hipSuccess) e = hipEventRecord(p->ev_tile[g], s);
    }
    return e;
}

void free_plan(ih_batch_plan* p)
{
    if (!p) return;
    if (p->exec_all) (void)hipGraphExecDestroy(p->exec_all);
    for (auto& e : p->exec_phase)
        if (e) (void)hipGraphExecDestroy(e);
    for (hipEvent_t e : p->ev_carry) (void)hipEventDestroy(e);
    for (hipEvent_t e : p->ev_tile) (void)hipEventDestroy(e);
    if (p->ev_start) (void)hipEventDestroy(p->ev_start);
    if (p->ev_done) (void)hipEventDestroy(p->ev_done);
    if (p->side) (void)hipStreamDestroy(p->side);
    for (hipEvent_t e : p->ev_branch) (void)hipEventDestroy(e);
    if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
    for (hipStream_t b : p->branch) (void)hipStreamDestroy(b);
    if (p->d_image) (void)hipFree(p->d_image);
    if (p->d_luts) (void)hipFree(p->d_luts);
    if (p->d_scratch) (void)hipFree(p->d_scratch);
    delete p;
}

// Number of pipeline groups for a batch of total_out output bytes (at least
// two when pipelining is asked for).
int64_t group_count(int64_t total_out, int64_t group_bytes)
{
    if (group_bytes <= 0) return 1;
    return std::max<int64_t>(2, (total_out + group_bytes - 1) / group_bytes);
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
    // arrival counters of fused frames start at zero (and are zero again
    // after every launch)
    e = hipMemsetAsync(p->d_scratch, 0, std::max<size_t>(words * 4, 256), p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return hip_fail(e, "clear batch scratch");
    if (!p->luts.empty()) {
        e = hipMalloc(&p->d_luts, p->luts.size());
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(IH_ERR_OOM, "bin tables: %s", hipGetErrorString(e));
        }
        e = hipMemcpy(p->d_luts, p->luts.data(), p->luts.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "upload bin tables");
    }
    std::vector<ih::FrameArgs> frames(n);
    std::vector<char> nt(n), bm(n);
    int64_t total_out = 0;
    for (size_t k = 0; k < n; ++k) {
        bm[k] = p->descs[k].binmajor ? 1 : 0;
        const int32_t li = p->lut_index.empty() ? -1 : p->lut_index[k];
        const uint8_t* dl = li < 0 ? nullptr : static_cast<const uint8_t*>(p->d_luts) + (size_t)li * 256;
        const bool general = li >= 0 && ih::lut_is_general(p->luts.data() + (size_t)li * 256);
        frames[k] = ih::frame_args(p->descs[k].frame, p->descs[k].out,
                                   static_cast<uint32_t*>(p->d_scratch) + off[k], geoms[k], dl, general);
        nt[k] = p->tiles[k].nontemporal ? 1 : 0;
        total_out += (int64_t)p->descs[k].H * p->descs[k].W * p->descs[k].B * 4;
    }
    const int64_t ng = std::min<int64_t>(group_count(total_out, p->group_bytes), (int64_t)n);
    if (ng <= 1) {
        ih::build_batch_image(frames, nt, &p->image, false, &bm);
        e = hipMalloc(&p->d_image, p->image.bytes());
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(IH_ERR_OOM, "batch tables: %s", hipGetErrorString(e));
        }
        e = hipMemcpy(p->d_image, p->image.host.data(), p->image.bytes(), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "upload batch tables");
        int32_t tile_launches = 0;
        for (const ih::BatchLaunch& l : p->image.launches) tile_launches += ih::phase_of(l) == 2;
        const int32_t nb = std::min(p->tile_branches, tile_launches);
        if (nb > 1) {
            p->branch.assign((size_t)nb, nullptr);
            p->ev_branch.assign((size_t)nb, nullptr);
            for (int32_t b = 0; e == hipSuccess && b < nb; ++b) {
                e = hipStreamCreateWithFlags(&p->branch[(size_t)b], hipStreamNonBlocking);
                if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_branch[(size_t)b], hipEventDisableTiming);
            }
            if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming);
            if (e != hipSuccess) return hip_fail(e, "tile branches");
            assign_branches(p);
        }
        return IH_OK;
    }
    // Consecutive frames, group boundaries where the running output passes
    // total * (g + 1) / ng; every group holds at least one frame.
    size_t k0 = 0, bytes = 0;
    int64_t acc = 0;
    for (int64_t g = 0; g < ng && k0 < n; ++g) {
        const int64_t goal = total_out / ng * (g + 1);
        size_t k1 = k0;
        do {
            acc += (int64_t)p->descs[k1].H * p->descs[k1].W * p->descs[k1].B * 4;
            ++k1;
        } while (k1 < n && (acc < goal || g == ng - 1) && (int64_t)(n - k1) > ng - 1 - g);
        PlanGroup G;
        std::vector<ih::FrameArgs> sub(frames.begin() + k0, frames.begin() + k1);
        std::vector<char> subnt(nt.begin() + k0, nt.begin() + k1), subbm(bm.begin() + k0, bm.begin() + k1);
        ih::build_batch_image(sub, subnt, &G.image, true, &subbm);
        G.frames = k1 - k0;
        G.dev_off = bytes;
        bytes = ih::align_up(bytes + G.image.bytes(), 256);
        p->groups.push_back(std::move(G));
        k0 = k1;
    }
    e = hipMalloc(&p->d_image, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(IH_ERR_OOM, "batch tables: %s", hipGetErrorString(e));
    }
    for (const PlanGroup& G : p->groups) {
        e = hipMemcpy(static_cast<unsigned char*>(p->d_image) + G.dev_off, G.image.host.data(), G.image.bytes(),
                      hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "upload batch tables");
    }
    e = hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
    e = hipEventCreateWithFlags(&p->ev_start, hipEventDisableTiming);
    for (size_t g = 0; e == hipSuccess && g < p->groups.size(); ++g) {
        hipEvent_t a = nullptr, b = nullptr;
        e = hipEventCreateWithFlags(&a, hipEventDisableTiming);
        if (e == hipSuccess) p->ev_carry.push_back(a);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b, hipEventDisableTiming);
        if (e == hipSuccess) p->ev_tile.push_back(b);
    }
    if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
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
        ih_status unused = IH_OK;
        hipError_t e1 = p->groups.empty() ? enqueue(p, phase, cs) : enqueue_pipelined(p, cs, false, &unused);
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

// The cache file holds one line per class: "gfx950/3 H W B NB TX TY NT K"
// (K: tile bands per carry band of the fused schedule, 0 for
// reduce-then-scan, -2 for prefix counts).  Lines of any other tag are
// skipped.
constexpr const char* kCacheTag = "gfx950/3";
constexpr int32_t kPrefixCode = -2;       // the prefix-count schedule in the cache and the ABI

int32_t schedule_code(const ih::TileChoice& t) { return t.prefix ? kPrefixCode : t.K; }

void load_cache(TuneCache& c)
{
    if (c.loaded) return;
    c.loaded = true;
    const char* path = cache_path();
    if (!path) return;
    std::ifstream in(path);
    std::string line;
    while (std::getline(in, line)) {
        std::istringstream ls(line);
        std::string tag;
        int H, W, B, NB, TX, TY, NT, K;
        if (!(ls >> tag >> H >> W >> B >> NB >> TX >> TY >> NT >> K) || tag != kCacheTag) continue;
        if (H < 1 || W < 1 || B < 1 || B > 256 || (K < 0 && K != kPrefixCode)) continue;
        ih::TileChoice t{TX, TY, NT != 0, K > 0 ? K : 0, K == kPrefixCode};
        if (!ih::tile_supported(B, t)) continue;
        if (t.K && !ih::fused_supported(ih::make_geom(H, W, B, t))) continue;
        if (t.prefix && !ih::prefix_supported(ih::make_geom(H, W, B, t))) continue;
        c.best[TuneKey{H, W, B, NB}] = t;
    }
}

void save_cache(TuneCache& c)
{
    const char* path = cache_path();
    if (!path) return;
    std::ofstream out(path);
    for (auto& kv : c.best)
        out << kCacheTag << ' ' << kv.first.H << ' ' << kv.first.W << ' ' << kv.first.B << ' ' << kv.first.nb << ' '
            << kv.second.TX << ' ' << kv.second.TY << ' ' << (kv.second.nontemporal ? 1 : 0) << ' '
            << schedule_code(kv.second) << '\n';
}

bool same_choice(const ih::TileChoice& a, const ih::TileChoice& b)
{
    return a.TX == b.TX && a.TY == b.TY && a.nontemporal == b.nontemporal && a.K == b.K && a.prefix == b.prefix;
}

// Candidates of a class of H x W frames: every supported tile width, band
// height and store flavour, each under the three carry schedules
// (reduce-then-scan; fused with carry bands of ceil(nTY / 16) tile bands;
// prefix counts, for frames of at most kMaxPrefixBands bands, where its
// quadratic count work stays small).
std::vector<ih::TileChoice> candidates(int32_t H, int32_t W, int32_t B)
{
    std::vector<ih::TileChoice> c;
    for (int tx : {32, 64, 128})
        for (int ty : {8, 16, 32, 64, 128, 256})
            for (bool nt : {false, true})
                for (int sched : {0, 1, 2}) {
                    ih::TileChoice t{tx, ih::even_band_height(H, ty), nt, 0};
                    if (!ih::tile_supported(B, t)) continue;
                    const int32_t nTY = (H + t.TY - 1) / t.TY;
                    if (sched == 1) {
                        t.K = ih::fused_bands(nTY, 16);
                        if (!ih::fused_supported(ih::make_geom(H, W, B, t))) continue;
                    }
                    if (sched == 2) {
                        t.prefix = true;
                        if (nTY > ih::kMaxPrefixBands || !ih::prefix_supported(ih::make_geom(H, W, B, t))) continue;
                    }
                    bool dup = false;
                    for (const ih::TileChoice& u : c) dup |= same_choice(u, t);
                    if (!dup) c.push_back(t);
                }
    return c;
}

// Heuristic tile for frames of one bin count launched together: the tallest
// band (fewest carries) that still leaves at least kMinWaves independent
// waves across all of the frames, made even.  For B = 64, 128-wide tiles
// (half the left-carry reads per stored byte) when a band of at least 32 rows
// still gives that many waves.
ih::TileChoice batch_default_tile(const std::vector<ih_frame_desc>& descs, int32_t B,
                                  int64_t kMinWaves = 4096)
{
    auto waves_of = [&](int tx, int ty) {
        int64_t w = 0;
        for (const ih_frame_desc& d : descs) {
            const ih::Geom g = ih::make_geom(d.H, d.W, d.B, ih::TileChoice{tx, ty, false});
            w += (int64_t)g.nTY * g.nJG;
        }
        return w;
    };
    // Tile width: 32 for four bins per lane and for B <= 16 (more waves per
    // frame; measured faster than 64 for 1080p B=16 batches), 64 otherwise,
    // 128 for B = 64 when enough waves remain.
    ih::TileChoice t{ih::bins_per_lane(B) == 4 || B <= 16 ? 32 : 64, 16, false};
    if (ih::tile_supported(B, ih::TileChoice{128, 32, false}) && waves_of(128, 32) >= kMinWaves)
        t.TX = 128;
    for (int ty : {256, 128, 64, 32, 16}) {
        t.TY = ty;
        if (waves_of(t.TX, ty) >= kMinWaves) break;
    }
    t.TY = ih::even_band_height(descs[0].H, t.TY);    // bands of the class's first frame made even
    return t;
}

// Bin-major frames of a batch: tiles chosen over all of them together
// (binmajor_tiles); a forced tile height (forced_ty > 0) is taken as it is,
// with four columns per lane.
void binmajor_batch_tiles(ih_batch_plan* p, int32_t forced_ty)
{
    std::vector<size_t> ks;
    std::vector<ih::BinmajorShape> shapes;
    for (size_t k = 0; k < p->descs.size(); ++k)
        if (p->descs[k].binmajor) {
            ks.push_back(k);
            shapes.push_back(ih::BinmajorShape{p->descs[k].H, p->descs[k].W, p->descs[k].B});
        }
    if (ks.empty()) return;
    std::vector<ih::TileChoice> t(ks.size());
    ih::binmajor_tiles(shapes.data(), shapes.size(), t.data());
    for (size_t q = 0; q < ks.size(); ++q) {
        if (forced_ty > 0) {
            t[q].TY = forced_ty;
            t[q].bm_cpl = 4;
        }
        p->tiles[ks[q]] = t[q];
    }
}

// Time one candidate on the frames of a class (all phases, no graph).
ih_status time_candidate(const std::vector<ih_frame_desc>& descs, const ih::TileChoice& t,
                         hipStream_t s, float* ms)
{
    ih_batch_plan* p = new ih_batch_plan;
    p->descs = descs;
    p->tiles.assign(descs.size(), t);
    p->use_graph = false;
    p->group_bytes = -1;
    p->stream = s;
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
    // everything the candidate ran is on s
    if (p->d_scratch || p->d_image) (void)hipStreamSynchronize(s);
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
        if (p->descs[k].lut == nullptr && !p->descs[k].binmajor)   // table and bin-major frames keep their tile
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
            for (const ih::TileChoice& t : candidates(kv.first.H, kv.first.W, kv.first.B)) {
                if (same_choice(t, best)) continue;
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
    ih_batch_options o{0, 1, 0, 0, -1, 0, -1, 0};
    if (opt) o = *opt;
    if (o.tile_branches < 0 || o.tile_branches > kMaxTileBranches)
        return fail(IH_ERR_INVALID_ARG, "tile_branches=%d must be in [0, %d]", o.tile_branches, kMaxTileBranches);
    const bool forced = o.tile_x > 0 || o.tile_y > 0;
    if (o.carry_bands < kPrefixCode)
        return fail(IH_ERR_INVALID_ARG, "carry_bands=%d must be >= %d", o.carry_bands, kPrefixCode);
    for (size_t k = 0; k < n; ++k) {
        const ih_frame_desc& d = frames[k];
        if (!d.frame || !d.out) return fail(IH_ERR_INVALID_ARG, "frame %zu: null pointer", k);
        if (ih_status st = ih::check_shape(d.H, d.W, d.B)) return st;
        if (reinterpret_cast<uintptr_t>(d.out) & 3u) return fail(IH_ERR_INVALID_ARG, "frame %zu: out misaligned", k);
        if (forced && !d.binmajor && !ih::tile_supported(d.B, ih::TileChoice{o.tile_x, o.tile_y, false}))
            return fail(IH_ERR_INVALID_ARG, "tile %dx%d not supported for B=%d", o.tile_x, o.tile_y, d.B);
        if (forced && d.binmajor && (o.tile_y < 1 || o.tile_y > 65535))
            return fail(IH_ERR_INVALID_ARG, "frame %zu: tile_y=%d must be in [1, 65535]", k, o.tile_y);
        if (d.binmajor != 0 && d.binmajor != 1)
            return fail(IH_ERR_INVALID_ARG, "frame %zu: binmajor must be 0 or 1", k);
        if (d.binmajor && d.lut)
            return fail(IH_ERR_INVALID_ARG, "frame %zu: bin-major frames take uniform bins (lut must be NULL)", k);
        if (d.lut) {
            if (forced && o.tile_x > 64)
                return fail(IH_ERR_INVALID_ARG, "frame %zu: bin tables take tiles at most 64 wide", k);
            for (int v = 0; v < 256; ++v)
                if ((int32_t)d.lut[v] >= d.B)
                    return fail(IH_ERR_INVALID_ARG, "frame %zu: lut[%d]=%d is not a bin below B=%d", k, v, d.lut[v], d.B);
        }
    }
    ih_batch_plan* p = new ih_batch_plan;
    (void)hipGetDevice(&p->device);
    p->stream = static_cast<hipStream_t>(stream);
    p->descs.assign(frames, frames + n);
    for (size_t k = 0; k < n; ++k) {
        if (frames[k].lut) {
            if (p->lut_index.empty()) p->lut_index.assign(n, -1);
            p->lut_index[k] = (int32_t)(p->luts.size() / 256);
            p->luts.insert(p->luts.end(), frames[k].lut, frames[k].lut + 256);
        }
    }
    p->use_graph = o.use_graph != 0;
    p->group_bytes = o.group_bytes;
    p->tile_branches = o.tile_branches > 0 ? o.tile_branches : kDefaultTileBranches;
    p->tiles.resize(n);
    int64_t total_out = 0;
    for (size_t k = 0; k < n; ++k) total_out += (int64_t)frames[k].H * frames[k].W * frames[k].B * 4;
    const int64_t ng = std::min<int64_t>(group_count(total_out, o.group_bytes), (int64_t)n);
    hipStream_t s = static_cast<hipStream_t>(stream);
    ih_status st = IH_OK;
    if (forced) {
        for (size_t k = 0; k < n; ++k) p->tiles[k] = ih::TileChoice{o.tile_x, o.tile_y, false};
    } else {
        // the heuristic for every frame; the autotuner then replaces the
        // tiles of the frames it times (those with uniform bins)
        std::map<int32_t, std::vector<ih_frame_desc>> by_b;
        for (size_t k = 0; k < n; ++k) by_b[frames[k].B].push_back(frames[k]);
        std::map<int32_t, ih::TileChoice> choice;
        // Pipelined: at least 1792 waves per group (about two per SIMD of a
        // 256-CU device) for its tile pass, so bands stay tall and the two
        // live groups' carries small; non-temporal stores so the output
        // stream leaves the carries in cache.
        const int64_t min_waves = ng > 1 ? 1792 * ng : 4096;
        for (auto& kv : by_b) {
            choice[kv.first] = batch_default_tile(kv.second, kv.first, min_waves);
            choice[kv.first].nontemporal = ng > 1;
        }
        for (size_t k = 0; k < n; ++k) p->tiles[k] = choice[frames[k].B];
        if (o.autotune) st = autotune(p, s);
    }
    if (st == IH_OK && o.nontemporal >= 0)
        for (auto& t : p->tiles) t.nontemporal = o.nontemporal != 0;
    // A forced carry schedule: reduce-then-scan (0), prefix counts (-2), or
    // fused with that many tile bands per carry band, clamped to each frame's
    // band count; each kept only where the frame's geometry supports it.
    for (size_t k = 0; st == IH_OK && o.carry_bands != -1 && k < n; ++k) {
        ih::TileChoice& t = p->tiles[k];
        t.K = 0;
        t.prefix = false;
        if (o.carry_bands == 0) continue;
        if (o.carry_bands == kPrefixCode) {
            ih::TileChoice q = t;
            q.prefix = true;
            if (ih::prefix_supported(ih::make_geom(frames[k].H, frames[k].W, frames[k].B, q))) t = q;
            continue;
        }
        const int32_t nTY = (frames[k].H + t.TY - 1) / t.TY;
        ih::TileChoice f = t;
        f.K = std::min(o.carry_bands, nTY);
        if (ih::fused_supported(ih::make_geom(frames[k].H, frames[k].W, frames[k].B, f))) t = f;
    }
    // Frames with bin tables: the table kernels exist for tiles up to 64 wide
    // (regular stores); the caller's table pointers are not kept.
    for (size_t k = 0; st == IH_OK && k < n; ++k) {
        if (!p->descs[k].lut) continue;
        if (p->tiles[k].TX > 64) p->tiles[k].TX = 64;
        p->tiles[k].nontemporal = false;
        p->descs[k].lut = nullptr;
    }
    // Bin-major frames: 64-column carry tiles (what the bin-major pass is
    // written for), bands chosen over the batch's bin-major frames together
    // unless a tile is forced (its height is kept).
    if (st == IH_OK) binmajor_batch_tiles(p, forced ? o.tile_y : 0);
    if (st == IH_OK) st = build_plan(p);
    if (st == IH_OK && p->use_graph) {
        st = capture(p, -1, &p->exec_all);
        for (int ph = 0; st == IH_OK && p->groups.empty() && ph < ih::kNumPhases; ++ph)
            st = capture(p, ph, &p->exec_phase[ph]);
    }
    if (st != IH_OK) {
        free_plan(p);
        return st;
    }
    *plan = p;
    return IH_OK;
}

ih_status launch_plan(ih_batch_plan* p, hipStream_t s);

ih_status ih_batch_plan_launch(ih_batch_plan* p, ih_stream_t stream)
{
    if (!p) return fail(IH_ERR_INVALID_ARG, "plan must be non-null");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (ih_status st = launch_plan(p, s)) return st;
    // the plan's last launch, for destroy to wait on
    if (!p->ev_done) {
        hipError_t e = hipEventCreateWithFlags(&p->ev_done, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    }
    hipError_t e = hipEventRecord(p->ev_done, s);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    p->launched = true;
    return IH_OK;
}

ih_status launch_plan(ih_batch_plan* p, hipStream_t s)
{
    ih::PhaseTimer timer;
    const bool prof = ih::profiling_on();
    if (!p->groups.empty()) {
        ih_status tst = IH_OK;
        hipError_t e = p->use_graph && !prof ? hipGraphLaunch(p->exec_all, s) : enqueue_pipelined(p, s, prof, &tst);
        if (e != hipSuccess) return hip_fail(e, "batch launch");
        if (tst != IH_OK) return tst;
        if (prof) ih::profiling_add_frames((uint64_t)p->descs.size());
        return IH_OK;
    }
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
    // wait for the plan's own work only: the last launch (launches of one
    // plan are ordered, see ih_batch_plan_launch) and the creation stream
    hipError_t e = p->launched ? hipEventSynchronize(p->ev_done) : hipSuccess;
    hipError_t e2 = hipStreamSynchronize(p->stream);
    free_plan(p);
    if (e != hipSuccess) return hip_fail(e, "wait for the plan's last launch");
    if (e2 != hipSuccess) return hip_fail(e2, "synchronize the creation stream");
    return IH_OK;
}

ih_status ih_batch_plan_info(const ih_batch_plan* p, ih_batch_info* info)
{
    if (!p || !info) return fail(IH_ERR_INVALID_ARG, "plan and info must be non-null");
    info->frames = (int64_t)p->descs.size();
    info->entries = p->entries;
    info->graph = p->use_graph ? 1 : 0;
    info->groups = p->groups.empty() ? 1 : (int32_t)p->groups.size();
    int32_t launches = 0, tile_launches = 0;
    auto count = [&](const ih::BatchImage& img) {
        launches += (int32_t)img.launches.size();
        for (const ih::BatchLaunch& l : img.launches)
            tile_launches += l.kind == ih::BatchLaunch::kTile || l.kind == ih::BatchLaunch::kTileBM;
    };
    if (p->groups.empty()) count(p->image);
    for (const PlanGroup& G : p->groups) count(G.image);
    info->kernel_launches = launches;
    info->tile_launches = tile_launches;
    return IH_OK;
}

ih_status ih_batch_plan_frame_schedule(const ih_batch_plan* p, size_t k, ih_frame_schedule* sched)
{
    if (!p || k >= p->descs.size() || !sched) return fail(IH_ERR_INVALID_ARG, "bad plan, index or output pointer");
    sched->tile_x = p->tiles[k].TX;
    sched->tile_y = p->tiles[k].TY;
    sched->nontemporal = p->tiles[k].nontemporal ? 1 : 0;
    sched->carry_bands = schedule_code(p->tiles[k]);
    int32_t group = 0;
    for (size_t g = 0, first = 0; g < p->groups.size(); ++g) {
        const size_t frames_in = p->groups[g].frames;
        if (k >= first && k < first + frames_in) group = (int32_t)g;
        first += frames_in;
    }
    sched->group = group;
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
