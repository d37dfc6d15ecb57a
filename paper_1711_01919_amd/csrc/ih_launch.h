// Batched launch images: the device tables (frame descriptors + job tables)
// and the launch list that run the three phases for many frames at once.
// Used by batch plans (fixed buffers, replayed from a hipGraph) and by the
// serving loop (a fresh image per dispatch).
#pragma once

#include "ih_internal.h"

#include <vector>

namespace ih {

struct BatchLaunch {
    enum Kind { kCount, kScan, kTile, kTileBM } kind = kCount;
    int tx = 64;               // kCount: tile width of the frames it covers
    bool fused = false;        // kCount: its frames take the fused carry schedule
    int parts = 1;             // kScan: scan form (scan_parts of its frames)
    int bg = 0;                // kTileBM: bins per work item of its frames
    int cpl = 1;               // kTileBM: columns per lane of its frames
    TileVariant v{};           // kTile: compiled kernel variant
    size_t jobs_off = 0;       // byte offset of this launch's job table in the image
    int32_t njobs = 0;
    int64_t n = 0;             // blocks (kCount, kScan) or work items (kTile, kTileBM)
    int32_t grid = 0;          // kTile: persistent workgroups
    size_t lds = 0;            // kCount: dynamic LDS bytes
    int64_t out_bytes = 0;     // kTile, kTileBM: output bytes the launch writes (for balancing branches)
    size_t sched_off = 0;      // kTile: byte offset of its two-word scheduling counter in the image (zero there)
};

struct BatchImage {
    std::vector<unsigned char> host;      // FrameArgs[n] at offset 0, then job tables
    std::vector<BatchLaunch> launches;
    size_t bytes() const { return host.size(); }
};

size_t align_up(size_t v, size_t a);

// Bytes of the largest launch image build_batch_image can make for n frames
// (FrameArgs table, at most six count, two scan, 2 n tile and ten
// bin-major launches, seven jobs per frame, each table aligned to 256 bytes,
// and a 256-byte scheduling counter per tile launch).
size_t batch_image_bound(size_t n);

// Scratch words a frame needs for the given tile.
size_t frame_scratch_words(const Geom& g);

// Fill img from fully set-up frames (device pointers, scratch included).
// nontemporal[k] picks the store flavour of frame k.  With leave_room, the
// persistent tile grid keeps one workgroup slot per compute unit free (when
// the kernel fits two or more per unit) for kernels running beside it.
// binmajor (may be null): frames whose output takes the bin-major layout
// (their geometry has 64-column tiles; their tile pass is tile_bm).
void build_batch_image(const std::vector<FrameArgs>& frames, const std::vector<char>& nontemporal,
                       BatchImage* img, bool leave_room = false, const std::vector<char>* binmajor = nullptr);

// Enqueue the image's launches of one phase (-1: all phases) on s.  dev_image
// is a device copy of img.host that stays valid until the work has run.
hipError_t enqueue_batch(const BatchImage& img, const void* dev_image, int phase, hipStream_t s);
// Enqueue launch i of the image on s.
hipError_t enqueue_launch(const BatchImage& img, const void* dev_image, size_t i, hipStream_t s);

int phase_of(const BatchLaunch& l);

}  // namespace ih
