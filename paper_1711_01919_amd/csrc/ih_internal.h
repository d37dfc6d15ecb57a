// Internal declarations shared by the kernels and the C-ABI layer of libih.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

namespace ih {

constexpr int kWave = 64;            // CDNA wavefront width
constexpr int kWavesPerBlock = 4;    // independent waves per workgroup in the tile pass

// Tile decomposition of one frame.  A tile is TY rows x TX columns.  In the
// tile pass a wave covers S horizontally adjacent tiles ("segments"); inside a
// segment, L lanes each own BPL consecutive bins.
struct Geom {
    int32_t H, W, B;
    int32_t TX, TY;          // tile width (columns) and height (rows)
    int32_t nTX, nTY;        // tiles across and down
    int32_t BPL, L, S;       // bins per lane, lanes per segment, segments per wave
    int32_t nJG;             // column groups (ceil(nTX / S)) = waves per tile row
};

// Scratch layout (uint32 words) for one frame:
//   rowc   [H][nTX][B]    row counts per tile segment, scanned to left carries
//   colc   [nTY][W][B]    column counts per tile band, scanned to top carries
//   corner [nTY][nTX][B]  per-tile totals, scanned to top-left corner counts
struct ScratchLayout {
    size_t rowc, colc, corner, words;
};

ScratchLayout scratch_layout(const Geom& g);

// Tile choice (TX, TY, store flavour) for a frame shape.
struct TileChoice {
    int32_t TX, TY;
    bool nontemporal;
};

Geom make_geom(int32_t H, int32_t W, int32_t B, const TileChoice& t);
TileChoice default_tile(int32_t H, int32_t W, int32_t B);
bool tile_supported(int32_t B, const TileChoice& t);

// Column groups that run the unguarded tile kernel (the rest run the guarded one).
int32_t interior_groups(const Geom& g, const uint8_t* frame, const uint32_t* out);

// The three phases of one frame, enqueued in this order on one stream:
// per-tile counts, carry scans, tile pass.
enum class Phase { kAgg = 0, kScan = 1, kTile = 2 };
constexpr int kNumPhases = 3;
hipError_t launch_phase(Phase ph, const uint8_t* frame, uint32_t* out, uint32_t* scratch,
                        const Geom& g, bool nontemporal, hipStream_t stream);

// Enqueue the four-corner query kernel.
hipError_t launch_query(const uint32_t* ih, int32_t H, int32_t W, int32_t B,
                        const int32_t* rects, int64_t n, uint32_t* hists,
                        uint32_t* bad_count, hipStream_t stream);

}  // namespace ih
