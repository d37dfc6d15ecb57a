// Internal declarations shared by the kernels, the C-ABI layer and the batch
// planner of libih.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

namespace ih {

constexpr int kWave = 64;            // CDNA wavefront width
constexpr int kWavesPerBlock = 4;    // independent waves per workgroup in the tile pass
constexpr int kScanThreads = 256;    // threads per block of the scan kernels
constexpr int kAggThreads = 256;     // threads per block of the per-tile count kernel

// Tile decomposition of one frame.  A tile is TY rows x TX columns.  In the
// tile pass a wave covers S horizontally adjacent tiles ("segments"); inside a
// segment, L lanes each own BPL consecutive bins.
//
// Carry schedule.  K == 0, PC == 0: reduce-then-scan -- the count launch
// counts each tile, then two scan launches turn the counts into carries, then
// the tile pass.  K >= 1: fused -- the count launch counts carry bands of K
// tile bands (nS of them) and scans the carries itself (the last block to
// finish a tile column scans that column, the last block to finish a carry
// band scans that band), so the tile pass follows it directly.  PC == 1:
// prefix counts -- each tile block of the count launch counts every row above
// its band, which gives the band's top carries with no scan, and their
// tile-column totals; the tile pass sums the totals of the tile columns to
// its left for its corner.  No scan launch and no inter-block communication;
// the count work grows with the square of the band count.
struct Geom {
    int32_t H, W, B;
    int32_t TX, TY;          // tile width (columns) and height (rows)
    int32_t nTX, nTY;        // tiles across and down
    int32_t BPL, L, S;       // bins per lane, lanes per segment, segments per wave
    int32_t nJG;             // column groups (ceil(nTX / S)) = waves per tile row
    int32_t K, nS;           // fused schedule: tile bands per carry band, carry bands (0, 0: reduce-then-scan)
    int32_t PC;              // 1: prefix-count schedule (then K == 0)
    int32_t CPL;             // bin-major tile pass: columns per lane (1 or 4); 0 for H x W x B frames
    int32_t RC16;            // 1: left carries stored as uint16 (W <= 65536, so every one is below 2^16)
    int32_t CC16;            // 1: column carries (colc) stored as uint16: reduce-then-scan or prefix
                             // counts with H <= 65536, so every count and top carry is below 2^16
};

// Arrival counters of the fused schedule sit in the first kCounterWords words
// of every frame's scratch, whatever the schedule, so that no carry of any
// frame ever lands on them.  They start at zero (cleared when the scratch is
// allocated) and the last block to arrive resets its counter, so they are
// zero again after every launch.
constexpr int32_t kCounterWords = 4096;

// Longest look-back of the prefix-count schedule's tile pass: the tile
// columns to the left of a tile whose totals it adds up for its corner.
constexpr int32_t kMaxPrefixTileColumns = 256;
// Bands of the frames that take the prefix-count schedule by default (the
// single-frame heuristic and the autotuner's candidates): its count work is
// about bands / 2 reads of the frame.
constexpr int32_t kMaxPrefixBands = 64;
// Pixels the count blocks of a single frame may read under the prefix-count
// schedule before the single-frame heuristic takes taller bands.
constexpr int64_t kPrefixCountPixels = 40 << 20;
// Single frames of at most kMidFramePixels with one bin per lane (B <= 64)
// take 32-column tiles and the tallest band that leaves at least
// kMidFrameWaves work items of at most kMidFrameItemBytes output each, under
// prefix counts while those read at most kMidPrefixPixels.
constexpr int64_t kMidFramePixels = 1920 * 1080;
constexpr int64_t kMidFrameWaves = 450;
constexpr int64_t kMidFrameItemBytes = 640 << 10;
constexpr int64_t kMidPrefixPixels = 20 << 20;
// Other single frames: about kMinWaves work items, or kMinWaves4K for frames
// above kMidFramePixels and of at most k4KFramePixels with B <= 128 (which
// take non-temporal stores).
constexpr int64_t kMinWaves = 960;
constexpr int64_t kMinWaves4K = 480;
constexpr int64_t k4KFramePixels = 3840 * 2160;

// Scratch layout (uint32 words) for one frame:
//   cnt    [kCounterWords]  fused schedule: arrivals per tile column (nTX), then
//                           per carry band (nS)
//   rowc   [nTX][H][B]      left carries: pixels of row y left of segment j, per bin
//                           (segment-major, so a tile's rows are one contiguous run);
//                           uint16 when RC16 (half the bytes the tile pass reads
//                           beside its write stream), else uint32
//   reduce-then-scan (colc uint16 when CC16, else uint32):
//   colc   [nTY][W][B]      column counts per tile band, scanned to top carries
//   corner [nTY][nTX][B]    per-tile totals, scanned to top-left corner counts
//   prefix counts:
//   colc   [nTY][W][B]      pixels of every row above band i, per column: the
//                           band's top carries as they are
//   corner [nTY][nTX][B]    their totals over each tile column
//   fused (carry band I, snapshot s < K):
//   colc   [nS][K][W][B]    s < K-1: column counts of the band's first s+1 tile
//                           bands; s = K-1: of the whole band, scanned down the
//                           bands to top carries
//   corner [nS][K][nTX][B]  the same for tile-column totals, each snapshot
//                           scanned across the tile columns
struct ScratchLayout {
    size_t cnt, rowc, colc, corner, words;
};
ScratchLayout scratch_layout(const Geom& g);

// Everything a kernel needs about one frame.
struct FrameArgs {
    const uint8_t* frame;
    uint32_t* out;
    uint32_t* rowc;
    uint32_t* colc;
    uint32_t* corner;
    uint32_t* cnt;
    const uint8_t* lut;      // device bin table (256 entries, each < B); null: floor(v B / 256)
    int32_t lut_general;     // 1: the table decreases somewhere (a bin need not be one range of values)
    Geom g;
};
FrameArgs frame_args(const uint8_t* frame, uint32_t* out, uint32_t* scratch, const Geom& g,
                     const uint8_t* lut = nullptr, bool lut_general = false);
// Whether a host bin table decreases somewhere.
bool lut_is_general(const uint8_t* lut_host);

// A job maps a contiguous range of a batched launch -- blocks for the count
// and scan kernels, work items (one per wave) for the tile kernel -- to one
// frame.  Jobs of a launch are sorted by `begin`.
struct Job {
    int64_t begin;
    int32_t frame;       // index into the FrameArgs table
    int32_t jg_begin;    // tile pass: first column group of the job; count phase: row-carry blocks
    int32_t jg_count;    // tile pass: column groups per tile band
    int32_t pad;
};

// Tile choice (TX, TY, store flavour, carry schedule) for a frame shape.
struct TileChoice {
    int32_t TX, TY;
    bool nontemporal;
    int32_t K = 0;           // 0: reduce-then-scan; >= 1: fused with K tile bands per carry band
    bool prefix = false;     // prefix-count schedule (K == 0)
    int32_t bm_cpl = 0;      // bin-major frames: columns per lane of the tile pass (1 or 4)
};

int bins_per_lane(int B);
Geom make_geom(int32_t H, int32_t W, int32_t B, const TileChoice& t);
TileChoice default_tile(int32_t H, int32_t W, int32_t B);
// Bin-major tile pass: a work item covers 64 * CPL columns (CPL per lane) of
// a band for a group of up to 16 bins, on the carries of 64-column tiles.
__host__ __device__ inline int32_t bm_segments(int32_t W, int32_t cpl)
{
    const int32_t cols = 64 * (cpl == 4 ? 4 : 1);
    return (W + cols - 1) / cols;
}
__host__ __device__ inline int64_t tile_bm_items_of(const Geom& g, int32_t bg)
{
    return (int64_t)g.nTY * bm_segments(g.W, g.CPL) * (g.B / bg);
}
// Tiles of bin-major frames launched together (one frame for
// ih_compute_binmajor, all of a plan's bin-major frames): four columns per
// lane (1 KB store runs) and the tallest band, up to 512 rows, that leaves
// kBmItemsWide items, when 64-row bands leave that many; otherwise one column
// per lane and the tallest band that leaves kBmItemsNarrow items (small
// frames need the items more than long runs).  Each frame's bands are then
// made even.
constexpr int64_t kBmItemsWide = 960;
constexpr int64_t kBmItemsNarrow = 3840;
struct BinmajorShape { int32_t H, W, B; };
void binmajor_tiles(const BinmajorShape* frames, size_t n, TileChoice* tiles);
TileChoice binmajor_tile(int32_t H, int32_t W, int32_t B);
// The same number of bands as TY gives, made equally tall (the last band is
// no shorter than the others by more than one row): a short last band makes
// short work items that leave the device half idle at the end of a launch.
int32_t even_band_height(int32_t H, int32_t TY);
bool tile_supported(int32_t B, const TileChoice& t);
// The fused schedule for this geometry: enough arrival counters, and carry
// bands whose per-column counts fit 16 bits.
bool fused_supported(const Geom& g);
// The prefix-count schedule for this geometry: column counts of the rows
// above a band fit the 16-bit LDS counters, and the tile pass's look-back
// over the tile columns to its left stays short.
bool prefix_supported(const Geom& g);
// Carry bands of about `target` tile bands' worth for the fused schedule:
// the K that leaves at most `max_bands` carry bands.
int32_t fused_bands(int32_t nTY, int32_t max_bands);
// Blocks of a frame's count launch: row-carry blocks, then tile (or carry
// band) blocks.
int64_t count_tile_blocks(const Geom& g);

// Column groups [0, n) run the unguarded tile kernel; the rest the guarded
// one.  Unguarded groups hold S whole TX-wide segments, 16-byte aligned.
int32_t interior_groups(const Geom& g, const uint8_t* frame, const uint32_t* out);

// Which compiled tile kernel serves a frame part.
struct TileVariant {
    int32_t bpl, tx, bc;     // bins per lane, tile width, compile-time B (0: runtime B)
    bool nt, guard;
    bool table;              // bins from a table (runtime B, regular stores, TX <= 64)
    bool operator<(const TileVariant& o) const;
    bool operator==(const TileVariant& o) const;
};
TileVariant tile_variant(const Geom& g, bool nontemporal, bool guard, bool table = false);

// ---- single frame: the three phases in order on one stream ----------------
// kAgg: the count launch (row carries and per-tile column counts).
enum class Phase { kAgg = 0, kScan = 1, kTile = 2 };
constexpr int kNumPhases = 3;
hipError_t launch_phase(Phase ph, const FrameArgs& f, bool nontemporal, hipStream_t stream);

// ---- batched launches over a device FrameArgs table ----------------------
// Count phase (row carries + tile column counts) of many frames of tile width
// TX and one kind of schedule (fused, or not) in one launch; a job's jg_begin
// holds its frame's row-carry block count.
hipError_t launch_count_batch(int TX, bool fused, const FrameArgs* frames, const Job* jobs, int32_t njobs,
                              int64_t nblocks, size_t lds_bytes, hipStream_t stream);
// Row-carry blocks (four rows each) and dynamic LDS bytes of a frame's count phase.
int32_t count_row_blocks(const Geom& g);
size_t count_lds(const Geom& g);
// The scan phase of many frames in one launch; `parts` is scan_parts(nTY) of
// every frame the launch covers.
hipError_t launch_scan_batch(int parts, const FrameArgs* frames, const Job* jobs, int32_t njobs,
                             int64_t nblocks, hipStream_t stream);
// Persistent tile launch: `grid` workgroups loop over `nitems` work items,
// taking them from the scheduling counter `sched` (two words, zero at launch
// and zero again after it) or, when it is null, striding over them.
hipError_t launch_tile_batch(const TileVariant& v, const FrameArgs* frames, const Job* jobs,
                             int32_t njobs, int64_t nitems, int32_t grid, uint32_t* sched, hipStream_t stream);
// Workgroups of the tile kernel that fit on the device at once.
int32_t tile_resident_blocks(const TileVariant& v);

// Blocks of the scan launch for one frame.
// Carry sequences longer than one 16-element chunk are split over the
// kScanParts waves of a scan block; shorter ones take one thread each.  The
// column-count sequences run over the nTY bands; the tile totals are scanned
// in two dimensions by blocks of corner_bins_per_block bins each: grids of at
// most 64 x 64 tiles take one sequence per lane and pass (split over the
// block's waves), larger ones one bin per block and one sequence per thread.
constexpr int kScanParts = kScanThreads / kWave;
inline int scan_parts(int len) { return len > 16 ? kScanParts : 1; }
inline int scan_per_block(int len) { return kScanThreads / scan_parts(len); }
__host__ __device__ inline int corner_bins_per_block(const Geom& g)
{
    const int m = g.nTX > g.nTY ? g.nTX : g.nTY;
    const int nb = m > kWave ? 1 : kWave / m;
    return nb < g.B ? nb : g.B;
}
int64_t scan_blocks(const Geom& g);

// Tile pass writing the bin-major layout (entry (x, y, b) at (b*H + y)*W + x)
// from the carries of a frame whose geometry has 64-column tiles.
hipError_t launch_tile_bm(const FrameArgs& f, hipStream_t stream);
// Bins per bin-major work item (largest power of two up to 16 dividing B),
// work items of a frame, and the batched pass over frames sharing one group
// width bg (a job per frame, `begin` its first item).
int bm_group(int B);
int64_t tile_bm_items(const Geom& g);
hipError_t launch_tile_bm_batch(int bg, int cpl, const FrameArgs* frames, const Job* jobs, int32_t njobs,
                                int64_t nitems, hipStream_t stream);

// Copy a host bin table (256 bytes, passed by value as a kernel argument) to
// device memory dst (64 uint32, 4-byte aligned), in stream order.
hipError_t launch_lut_store(const uint8_t* lut_host, uint32_t* dst, hipStream_t stream);

// Write reference: the tile pass's store stream (B <= 64, TX in {32, 64,
// 128}) without loads or arithmetic.
hipError_t launch_write_reference(uint32_t* out, int32_t H, int32_t W, int32_t B, int32_t TX, int32_t TY,
                                  hipStream_t stream);

// Load every kernel's code object now (hipFuncGetAttributes on one kernel of
// each), so that no request pays for it on a kernel's first launch.
hipError_t preload_kernels();

// ---- region query ---------------------------------------------------------
// binmajor: ih holds the b x h x w layout instead of H x W x B.
hipError_t launch_query(const uint32_t* ih, int32_t H, int32_t W, int32_t B,
                        const int32_t* rects, int64_t n, uint32_t* hists,
                        uint32_t* bad_count, bool binmajor, hipStream_t stream);

}  // namespace ih
