// Batched launch images (see ih_launch.h).
#include "ih_launch.h"

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>

namespace ih {

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

size_t frame_scratch_words(const Geom& g) { return align_up(scratch_layout(g).words, 64); }

size_t batch_image_bound(size_t n)
{
    const size_t launches = 6 + 2 + 2 * n + 10;
    return align_up(n * sizeof(FrameArgs), 256) + launches * 256 + 7 * n * sizeof(Job) + 256 + 2 * n * 256;
}

int phase_of(const BatchLaunch& l)
{
    switch (l.kind) {
    case BatchLaunch::kCount: return 0;
    case BatchLaunch::kScan: return 1;
    default: return 2;
    }
}

// Resident workgroups per tile-kernel variant, asked of the runtime once.
static int32_t resident_blocks_cached(const TileVariant& v)
{
    static std::mutex mu;
    static std::map<TileVariant, int32_t>* cache = new std::map<TileVariant, int32_t>;
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache->find(v);
    if (it != cache->end()) return it->second;
    const int32_t r = tile_resident_blocks(v);
    (*cache)[v] = r;
    return r;
}

// Compute units of the current device, asked of the runtime once per device.
static int32_t cu_count_cached()
{
    static std::mutex mu;
    static std::map<int, int32_t>* cache = new std::map<int, int32_t>;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache->find(dev);
    if (it != cache->end()) return it->second;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        cus = 256;
    (*cache)[dev] = cus;
    return cus;
}

void build_batch_image(const std::vector<FrameArgs>& frames, const std::vector<char>& nontemporal,
                       BatchImage* img, bool leave_room, const std::vector<char>* binmajor)
{
    const size_t n = frames.size();
    std::vector<std::vector<Job>> tables;
    std::vector<BatchLaunch> launches;

    // Count phase, one launch per tile width and kind of schedule (fused or
    // not): per frame, row-carry blocks of four rows (jg_begin of the job
    // holds their count), then one block per tile (reduce-then-scan, prefix
    // counts) or per carry band and tile column (fused).
    for (int tx : {32, 64, 128})
    for (bool fused : {false, true}) {
        std::vector<Job> jobs;
        int64_t begin = 0;
        size_t lds = 0;
        for (size_t k = 0; k < n; ++k) {
            const Geom& g = frames[k].g;
            if (g.TX != tx || (g.K != 0) != fused) continue;
            const int32_t row_blocks = count_row_blocks(g);
            jobs.push_back(Job{begin, (int32_t)k, row_blocks, 0, 0});
            begin += row_blocks + count_tile_blocks(g);
            lds = std::max(lds, count_lds(g));
        }
        if (jobs.empty()) continue;
        BatchLaunch l;
        l.kind = BatchLaunch::kCount;
        l.tx = tx;
        l.fused = fused;
        l.lds = lds;
        l.n = begin;
        l.njobs = (int32_t)jobs.size();
        launches.push_back(l);
        tables.push_back(std::move(jobs));
    }
    // Scans: one launch per scan form (one thread per carry sequence, or
    // sequences split over the waves of a block).
    for (int parts : {1, kScanParts}) {
        std::vector<Job> jobs;
        int64_t begin = 0;
        for (size_t k = 0; k < n; ++k) {
            const Geom& g = frames[k].g;
            if (g.K || g.PC) continue;  // fused or prefix counts: carries ready after the count launch
            if (scan_parts(g.nTY) != parts) continue;
            const int64_t nb = scan_blocks(g);
            if (nb == 0) continue;
            jobs.push_back(Job{begin, (int32_t)k, 0, 0, 0});
            begin += nb;
        }
        if (jobs.empty()) continue;
        BatchLaunch l;
        l.kind = BatchLaunch::kScan;
        l.parts = parts;
        l.n = begin;
        l.njobs = (int32_t)jobs.size();
        launches.push_back(l);
        tables.push_back(std::move(jobs));
    }
    // Tile jobs per kernel variant, the jobs with the largest work items
    // first (a persistent wave takes the next item when it finishes one, so
    // the small items fill in at the end).
    struct TileJob { Job job; int64_t items, item_bytes; };
    std::map<TileVariant, std::vector<TileJob>> pending;
    std::map<TileVariant, int64_t> obytes;
    for (size_t k = 0; k < n; ++k) {
        if (binmajor && (*binmajor)[k]) continue;
        const Geom& g = frames[k].g;
        const int32_t n_int = interior_groups(g, frames[k].frame, frames[k].out);
        const int32_t parts[2][2] = {{0, n_int}, {n_int, g.nJG - n_int}};
        for (int q = 0; q < 2; ++q) {
            if (parts[q][1] <= 0) continue;
            const TileVariant v = tile_variant(g, nontemporal[k] != 0, q == 1, frames[k].lut != nullptr);
            const int64_t item_bytes = (int64_t)g.TY * std::min<int64_t>((int64_t)g.S * g.TX, g.W) * g.B * 4;
            pending[v].push_back(TileJob{Job{0, (int32_t)k, parts[q][0], parts[q][1], 0},
                                         (int64_t)g.nTY * parts[q][1], item_bytes});
            obytes[v] += (int64_t)g.H * g.W * g.B * 4 * parts[q][1] / g.nJG;
        }
    }
    std::map<TileVariant, std::vector<Job>> byv;
    std::map<TileVariant, int64_t> items;
    for (auto& kv : pending) {
        std::stable_sort(kv.second.begin(), kv.second.end(),
                         [](const TileJob& a, const TileJob& b) { return a.item_bytes > b.item_bytes; });
        int64_t& b = items[kv.first];
        for (TileJob& t : kv.second) {
            t.job.begin = b;
            byv[kv.first].push_back(t.job);
            b += t.items;
        }
    }
    for (auto& kv : byv) {
        BatchLaunch l;
        l.kind = BatchLaunch::kTile;
        l.v = kv.first;
        l.n = items[kv.first];
        l.out_bytes = obytes[kv.first];
        l.njobs = (int32_t)kv.second.size();
        const int64_t want = (l.n + kWavesPerBlock - 1) / kWavesPerBlock;
        int32_t cap = resident_blocks_cached(kv.first);
        if (leave_room) {
            const int32_t cus = cu_count_cached();
            const int32_t per_cu = cap / cus;
            if (per_cu >= 2) cap = (per_cu - 1) * cus;
        }
        l.grid = (int32_t)std::min<int64_t>(want, cap);
        launches.push_back(l);
        tables.push_back(std::move(kv.second));
    }
    // Bin-major frames: one launch per bin-group width and columns per lane,
    // one wave per item.
    for (int cpl : {4, 1})
    for (int bg : {16, 8, 4, 2, 1}) {
        if (!binmajor) break;
        std::vector<Job> jobs;
        int64_t begin = 0, bm_bytes = 0;
        for (size_t k = 0; k < n; ++k) {
            if (!(*binmajor)[k] || bm_group(frames[k].g.B) != bg || frames[k].g.CPL != cpl) continue;
            jobs.push_back(Job{begin, (int32_t)k, 0, 0, 0});
            begin += tile_bm_items(frames[k].g);
            bm_bytes += (int64_t)frames[k].g.H * frames[k].g.W * frames[k].g.B * 4;
        }
        if (jobs.empty()) continue;
        BatchLaunch l;
        l.kind = BatchLaunch::kTileBM;
        l.bg = bg;
        l.cpl = cpl;
        l.out_bytes = bm_bytes;
        l.n = begin;
        l.njobs = (int32_t)jobs.size();
        launches.push_back(l);
        tables.push_back(std::move(jobs));
    }

    size_t bytes = align_up(n * sizeof(FrameArgs), 256);
    for (size_t t = 0; t < tables.size(); ++t) {
        launches[t].jobs_off = bytes;
        bytes = align_up(bytes + tables[t].size() * sizeof(Job), 256);
    }
    // scheduling counters of the tile launches, zero in the image, each in a
    // 256-byte line of its own (away from the tables, which are read through
    // the scalar cache)
    for (BatchLaunch& l : launches) {
        if (l.kind != BatchLaunch::kTile) continue;
        l.sched_off = bytes;
        bytes += 256;
    }
    img->host.assign(bytes, 0);
    std::memcpy(img->host.data(), frames.data(), n * sizeof(FrameArgs));
    for (size_t t = 0; t < tables.size(); ++t)
        std::memcpy(img->host.data() + launches[t].jobs_off, tables[t].data(), tables[t].size() * sizeof(Job));
    img->launches = std::move(launches);
}

hipError_t enqueue_launch(const BatchImage& img, const void* dev_image, size_t i, hipStream_t s)
{
    const unsigned char* base = static_cast<const unsigned char*>(dev_image);
    const FrameArgs* fr = reinterpret_cast<const FrameArgs*>(base);
    const BatchLaunch& l = img.launches[i];
    const Job* jobs = reinterpret_cast<const Job*>(base + l.jobs_off);
    switch (l.kind) {
    case BatchLaunch::kCount: return launch_count_batch(l.tx, l.fused, fr, jobs, l.njobs, l.n, l.lds, s);
    case BatchLaunch::kScan: return launch_scan_batch(l.parts, fr, jobs, l.njobs, l.n, s);
    case BatchLaunch::kTile:
        return launch_tile_batch(l.v, fr, jobs, l.njobs, l.n, l.grid,
                                 l.sched_off ? reinterpret_cast<uint32_t*>(const_cast<unsigned char*>(base) + l.sched_off)
                                             : nullptr,
                                 s);
    case BatchLaunch::kTileBM: return launch_tile_bm_batch(l.bg, l.cpl, fr, jobs, l.njobs, l.n, s);
    }
    return hipErrorInvalidValue;
}

hipError_t enqueue_batch(const BatchImage& img, const void* dev_image, int phase, hipStream_t s)
{
    for (size_t i = 0; i < img.launches.size(); ++i) {
        if (phase >= 0 && phase_of(img.launches[i]) != phase) continue;
        if (hipError_t e = enqueue_launch(img, dev_image, i, s)) return e;
    }
    return hipSuccess;
}

}  // namespace ih
