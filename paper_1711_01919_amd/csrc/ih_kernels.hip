// HIP kernels (gfx950) for the exact integral histogram and its region query.
//
// The integral histogram (Sec. 2.1, Eq. 1) is a 2-D inclusive prefix count
// per bin.  It is computed by reduce-then-scan over TY x TX tiles:
//
//   1. agg     per tile: bin counts of every tile-row segment, of every tile
//              column, and of the whole tile (LDS atomics, one pass over the
//              uint8 pixels).
//   2. scan    exclusive scans of those counts across tiles, giving each tile
//              its left carry per row, its top carry per column, and its
//              top-left corner count.
//   3. tile    the hot pass: each lane owns BPL bins of one tile segment; it
//              bins each pixel of the row (binning is fused here -- the
//              one-hot tensor is never stored), scans the row in-lane, adds
//              the row into TX column accumulators held in VGPRs, and stores
//              the finished H x W x B entries.
//
// For entry (x, y, b) of a tile whose top-left pixel is (x0, y0):
//   H(x,y,b) = corner(b) + sum_{x0<=x'<=x} top(x',b)
//            + sum_{y0<=y'<=y} left(y',b) + local(x,y,b)
// where top/left/corner count the pixels above / left of / above-left of the
// tile: the inclusion-exclusion of Eq. 1 over four regions, exact in uint32.
//
// Each phase has one per-frame body.  Single-frame kernels take the frame by
// value; batched kernels map their blocks (or work items) to frames through a
// sorted job table and run the same body.
#include "ih_device.h"
#include "ih_tile_fns.h"

#include <algorithm>
#include <cstring>
#include <vector>

namespace ih {

// ---------------------------------------------------------------------------
// Phase 1a: left carries of every row (rowcarry)
// ---------------------------------------------------------------------------
// One wave per frame row.  For a chunk of up to kSegChunk tile segments the
// wave bins the row's pixels into per-segment histograms in LDS (8-bit
// counters: a segment holds at most TX <= 128 pixels), then each lane walks
// the segments for its bins and stores the exclusive running count: rowc[j][y][b]
// = pixels of row y left of segment j in bin b.
constexpr int kSegChunk = 32;
constexpr int kRowThreads = kWave;     // one row per wave

__device__ __forceinline__ void lds_inc8(uint32_t* h, uint32_t e)
{
    atomicAdd(&h[e >> 2], 1u << ((e & 3u) << 3));
}
__device__ __forceinline__ uint32_t lds_get8(const uint32_t* h, uint32_t e)
{
    return (h[e >> 2] >> ((e & 3u) << 3)) & 0xFFu;
}

// The row-carry work is one wave's own: its LDS region is private and it
// synchronizes within the wave only (all memory counters drained), so a
// workgroup may hold several row waves, or row waves beside other work.
__device__ __forceinline__ void wave_sync()
{
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// The running counts of a row-carry wave over ns segments of a chunk, for
// the lane's 2 <= bpl <= 4 bins: segment by segment, the counters of all of
// the lane's bins are read from LDS together, then stored together (a wave's
// stores of one segment and row are one contiguous run; storing bin by bin
// over all segments instead would leave half-written lines to be written
// back twice).
__device__ __forceinline__ void rowcarry_walk(const FrameArgs& f, const uint32_t* lds, int lane, int bpl, int j0,
                                              int ns, size_t row_off, size_t seg_stride, uint32_t (&run)[4])
{
    const Geom& g = f.g;
    const int B = g.B;
#pragma unroll 1
    for (int sg = 0; sg < ns; ++sg) {
        uint32_t c[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int b = lane * bpl + t;
            const bool ok = t < bpl && b < B;
            const uint32_t v = lds_get8(lds, ok ? (uint32_t)(sg * B + b) : 0u);
            c[t] = ok ? v : 0u;
        }
        const size_t o = row_off + (size_t)(j0 + sg) * seg_stride + (size_t)lane * bpl;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            if (t < bpl && lane * bpl + t < B) {
                if (g.RC16) gmem(reinterpret_cast<uint16_t*>(f.rowc))[o + t] = (uint16_t)run[t];
                else gmem(f.rowc)[o + t] = run[t];
            }
            run[t] += c[t];
        }
    }
}

// Bin of byte c of a loaded word w: floor(v B / 256) (kBinScaled), the same
// as one bit-field extract when B = 2^k with k >= 1 (kBinShift; bs = 8 - k,
// so 8 c + bs <= 31), the bin table staged in LDS (kBinTable), or either of
// the first and the last as the frame has it (kBinAny).
enum BinForm { kBinScaled, kBinShift, kBinTable, kBinAny };
template <int BF>
__device__ __forceinline__ uint32_t bin_in_word(const FrameArgs& f, const uint32_t* lutw, uint32_t w, int c,
                                                uint32_t B, int bs)
{
    if constexpr (BF == kBinShift) {
        return (w >> (8 * c + bs)) & (B - 1u);
    } else {
        const uint32_t v = (w >> (8 * c)) & 0xFFu;
        if constexpr (BF == kBinTable) return (lutw[v >> 2] >> (8 * (v & 3u))) & 0xFFu;
        else if constexpr (BF == kBinScaled) return (v * B) >> 8;
        else return bin_of(f, lutw, v, B);
    }
}

// The pixels [x0, x0 + npx) of a row added to the 8-bit counters of their
// segments (one 16-byte chunk per lane and round, four rounds in flight),
// compiled per bin form; whole chunks take no per-pixel bound check.
template <int BF>
__device__ __forceinline__ void rowcarry_count(const FrameArgs& f, const IH_GLOBAL uint8_t* prow, uint32_t* lds,
                                               const uint32_t* lutw, int lane, int x0, int npx, bool vec, int bs)
{
    const Geom& g = f.g;
    const uint32_t B = (uint32_t)g.B;
    const int TX = g.TX;
    const int nchunks = (npx + 15) / 16;
    for (int c0 = 0; c0 < nchunks; c0 += 4 * kRowThreads) {
        // up to four 16-byte chunks per lane in flight before any counting
        u32x4 w[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int c = c0 + u * kRowThreads + lane;
            const int p = c * 16;
            if (c < nchunks && vec && p + 16 <= npx) {
                w[u] = *reinterpret_cast<const IH_GLOBAL u32x4*>(prow + x0 + p);
            } else {
                uint32_t b4[4] = {0u, 0u, 0u, 0u};
                for (int k = 0; c < nchunks && k < 16 && p + k < npx; ++k)
                    b4[k / 4] |= (uint32_t)prow[x0 + p + k] << (8 * (k % 4));
                w[u] = u32x4{b4[0], b4[1], b4[2], b4[3]};
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int c = c0 + u * kRowThreads + lane;
            if (c >= nchunks) continue;
            const int p = c * 16;
            const uint32_t seg = (uint32_t)((p / TX) * (int)B);
            const uint32_t words[4] = {w[u].x, w[u].y, w[u].z, w[u].w};
            if (p + 16 <= npx) {
#pragma unroll
                for (int k = 0; k < 16; ++k) lds_inc8(lds, seg + bin_in_word<BF>(f, lutw, words[k / 4], k % 4, B, bs));
            } else {
#pragma unroll
                for (int k = 0; k < 16; ++k)
                    if (p + k < npx) lds_inc8(lds, seg + bin_in_word<BF>(f, lutw, words[k / 4], k % 4, B, bs));
            }
        }
    }
}

__device__ __forceinline__ void rowcarry_body(const FrameArgs& f, int64_t y, uint32_t* lds)
{
    const Geom& g = f.g;
    const int B = g.B, TX = g.TX, bpl = g.BPL;
    const int lane = threadIdx.x % kWave;
    uint32_t run[4] = {0u, 0u, 0u, 0u};
    const IH_GLOBAL uint8_t* prow = gmem(f.frame) + y * g.W;
    // rowc is segment-major, [j][y][b]: a tile wave's rows are contiguous;
    // uint16 entries when RC16
    const size_t row_off = (size_t)y * B;
    const size_t seg_stride = (size_t)g.H * B;
    // 16-byte chunks never straddle a segment (TX is a multiple of 16)
    const bool vec = ((reinterpret_cast<uintptr_t>(prow) & 15) == 0);
    // the bin table sits after the counters of the largest segment chunk
    uint32_t* lutw = lds + (((kSegChunk < g.nTX ? kSegChunk : g.nTX) * B + 3) / 4);
    stage_lut(f, lutw, lane, kRowThreads);      // visible after the first barrier below
    const bool pow2 = B >= 2 && (B & (B - 1)) == 0;
    const int bs = 8 - (31 - __builtin_clz((uint32_t)B));
    for (int j0 = 0; j0 < g.nTX; j0 += kSegChunk) {
        const int ns = min(kSegChunk, g.nTX - j0);
        for (int w = lane; w < (ns * B + 3) / 4; w += kRowThreads) lds[w] = 0u;
        wave_sync();
        const int x0 = j0 * TX;
        const int npx = min(ns * TX, g.W - x0);
        if (f.lut) rowcarry_count<kBinTable>(f, prow, lds, lutw, lane, x0, npx, vec, bs);
        else if (pow2) rowcarry_count<kBinShift>(f, prow, lds, lutw, lane, x0, npx, vec, bs);
        else rowcarry_count<kBinScaled>(f, prow, lds, lutw, lane, x0, npx, vec, bs);
        wave_sync();
        if (bpl == 1) {
            // one bin per lane: four segments at a time
            const int b = lane;
            if (b < B) {
                uint32_t r = run[0];
#pragma unroll 1
                for (int s0 = 0; s0 < ns; s0 += 4) {
                    uint32_t c[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const bool ok = s0 + u < ns;
                        const uint32_t v = lds_get8(lds, ok ? (uint32_t)((s0 + u) * B + b) : 0u);
                        c[u] = ok ? v : 0u;
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        if (s0 + u < ns) {
                            const size_t o = row_off + (size_t)(j0 + s0 + u) * seg_stride + b;
                            if (g.RC16) gmem(reinterpret_cast<uint16_t*>(f.rowc))[o] = (uint16_t)r;
                            else gmem(f.rowc)[o] = r;
                        }
                        r += c[u];
                    }
                }
                run[0] = r;
            }
        } else {
            rowcarry_walk(f, lds, lane, bpl, j0, ns, row_off, seg_stride, run);
        }
        wave_sync();
    }
}

// LDS bytes a row-carry workgroup needs for a frame: 8-bit counters for the
// segments of one chunk, then the 256-entry bin table.
__host__ __device__ inline size_t rowcarry_lds_bytes(const Geom& g)
{
    const int ns = g.nTX < kSegChunk ? g.nTX : kSegChunk;
    return ((size_t)ns * g.B + 3) / 4 * 4 + 256;
}

// ---------------------------------------------------------------------------
// Phase 1b: per-tile column counts (agg)
// ---------------------------------------------------------------------------
// One 256-thread block per TY x TX tile: per-column bin counts of the tile
// (LDS counters, <= TY pixels each), written to colc[i][x][b], and the
// tile's total per bin, written to corner[i][j][b].

// Column counters of a tile: one 32-bit word per bin where the tile's
// counters fit kWideColWords words, else two 16-bit counters per word (bins b
// and b ^ 1 of a column; column counts are <= 65535, so a carry never crosses
// halves).  Separate words take fewer same-address collisions among the
// lanes of one LDS increment, the packed form half the LDS of wide tiles with
// many bins.  sh is 0 for the first form, 1 for the second.  A column takes
// col_words words, one more than its counters need, so that the words of
// neighbouring columns start on different LDS banks.
constexpr int kWideColWords = 64 * 65;
__host__ __device__ inline int col_shift(int TX, int B) { return TX * (B + 1) <= kWideColWords ? 0 : 1; }
__host__ __device__ inline int col_words(int TX, int B) { return col_shift(TX, B) ? (B + 1) / 2 + 1 : B + 1; }
__device__ __forceinline__ void col_inc(uint32_t* h, int cw, int sh, int x, uint32_t b)
{
    atomicAdd(&h[x * cw + (int)(b >> sh)], 1u << ((b & (uint32_t)sh) << 4));
}
template <int SH>
__device__ __forceinline__ void col_inc(uint32_t* h, int cw, int sh, int x, uint32_t b)
{
    if constexpr (SH == 0) atomicAdd(&h[x * cw + (int)b], 1u);
    else if constexpr (SH == 1) atomicAdd(&h[x * cw + (int)(b >> 1)], 1u << ((b & 1u) << 4));
    else col_inc(h, cw, sh, x, b);
}

__device__ __forceinline__ uint32_t col_get(const uint32_t* h, int cw, int sh, int x, int b)
{
    const uint32_t w = h[x * cw + (b >> sh)];
    return sh ? (w >> ((b & 1) << 4)) & 0xFFFFu : w;
}

// Pixels of rows [ya, yb) and columns [x0, x0 + tw) added to the per-column
// bin counters colh.  Rows whose four-byte words are aligned (W a multiple
// of 4, frame 4-byte aligned; tw is then a multiple of 4 too): thread tid
// takes the four columns 4 (tid % (TX/4)) .. + 3 of every (kAggThreads /
// (TX/4))-th row with one load.  Otherwise thread tid takes column tid % TX
// of every (kAggThreads / TX)-th row.  Compiled per counter form (SH: 0 or
// 1 as col_shift, -1 for the form given by sh) and bin form (BF), so that an
// increment costs the fewest instructions.
template <int TX, int SH, int BF>
__device__ __forceinline__ void count_rows_as(const FrameArgs& f, const uint32_t* lutw, uint32_t* colh, int ya, int yb,
                                              int x0, int tw, int sh, int bs)
{
    const Geom& g = f.g;
    const uint32_t B = (uint32_t)g.B;
    const int cw = col_words(TX, g.B);
    if ((g.W % 4) == 0 && (reinterpret_cast<uintptr_t>(f.frame) & 3) == 0) {
        constexpr int TPR = TX / 4;                    // threads per row
        constexpr int kRowsPerPass4 = kAggThreads / TPR;
        const int tr = (int)threadIdx.x / TPR, tq = (int)threadIdx.x % TPR;
        if (4 * tq >= tw) return;
        const int th = yb - ya;
        const size_t stride = (size_t)(g.W / 4);
        const IH_GLOBAL uint32_t* p =
            reinterpret_cast<const IH_GLOBAL uint32_t*>(gmem(f.frame) + (size_t)ya * g.W + x0) + tq;
        constexpr int U = 8;
        for (int r0 = tr; r0 < th; r0 += U * kRowsPerPass4) {
            uint32_t v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int r = r0 + u * kRowsPerPass4;
                v[u] = r < th ? p[(size_t)r * stride] : 0u;
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (r0 + u * kRowsPerPass4 < th)
#pragma unroll
                    for (int c = 0; c < 4; ++c)
                        col_inc<SH>(colh, cw, sh, 4 * tq + c, bin_in_word<BF>(f, lutw, v[u], c, B, bs));
        }
        return;
    }
    constexpr int kRowsPerPass = kAggThreads / TX;
    const int tr = (int)threadIdx.x / TX, tx = (int)threadIdx.x % TX;
    if (tx >= tw) return;
    const int th = yb - ya;
    const IH_GLOBAL uint8_t* p = gmem(f.frame) + (size_t)ya * g.W + x0 + tx;
    constexpr int U = 8;                       // rows whose pixels are in flight together
    for (int r0 = tr; r0 < th; r0 += U * kRowsPerPass) {
        uint32_t v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int r = r0 + u * kRowsPerPass;
            v[u] = r < th ? (uint32_t)p[(size_t)r * g.W] : 0u;
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (r0 + u * kRowsPerPass < th)
                col_inc<SH>(colh, cw, sh, tx, bin_in_word<BF>(f, lutw, v[u], 0, B, bs));
    }
}

template <int TX>
__device__ __forceinline__ void count_rows(const FrameArgs& f, const uint32_t* lutw, uint32_t* colh, int ya, int yb,
                                           int x0, int tw)
{
    const int B = f.g.B;
    const int bs = 8 - (31 - __builtin_clz((uint32_t)B));
    const bool wide = col_shift(TX, B) == 0;
    if (f.lut) {
        if (wide) count_rows_as<TX, 0, kBinTable>(f, lutw, colh, ya, yb, x0, tw, 0, bs);
        else count_rows_as<TX, 1, kBinTable>(f, lutw, colh, ya, yb, x0, tw, 1, bs);
    } else if (B >= 2 && (B & (B - 1)) == 0) {
        if (wide) count_rows_as<TX, 0, kBinShift>(f, lutw, colh, ya, yb, x0, tw, 0, bs);
        else count_rows_as<TX, 1, kBinShift>(f, lutw, colh, ya, yb, x0, tw, 1, bs);
    } else {
        if (wide) count_rows_as<TX, 0, kBinScaled>(f, lutw, colh, ya, yb, x0, tw, 0, bs);
        else count_rows_as<TX, 1, kBinScaled>(f, lutw, colh, ya, yb, x0, tw, 1, bs);
    }
}

// Reduce-then-scan: the pixels of tile (i, j) itself.  Prefix counts: the
// pixels of every row above band i in tile column j (rows [0, y0); counts
// below 2^16 since H <= 65536), so colc holds the band's top carries as they
// are and corner their tile-column totals.  The blocks of the lowest bands
// count the most rows, so they come first in the launch.
template <int TX>
__device__ __forceinline__ void agg_body(const FrameArgs& f, int64_t tile, uint32_t* colh, uint32_t* lutw)
{
    const Geom& g = f.g;
    const int B = g.B;
    const int r = (int)(tile / g.nTX);
    const int j = (int)(tile - (int64_t)r * g.nTX);
    const int i = g.PC ? g.nTY - 1 - r : r;
    const int x0 = j * TX, y0 = i * g.TY;
    const int tw = min(TX, g.W - x0);
    const int ya = g.PC ? 0 : y0;
    const int yb = g.PC ? y0 : min(g.H, y0 + g.TY);
    const int tid = threadIdx.x;

    const int cw = col_words(TX, B), sh = col_shift(TX, B);
    for (int e = tid; e < TX * cw; e += kAggThreads) colh[e] = 0;
    stage_lut(f, lutw, tid, kAggThreads);
    __syncthreads();
    count_rows<TX>(f, lutw, colh, ya, yb, x0, tw);
    __syncthreads();
    const size_t cbase = ((size_t)i * g.W + x0) * B;
    for (int e = tid; e < tw * B; e += kAggThreads) {
        const int x = e / B, b = e - x * B;
        const uint32_t v = col_get(colh, cw, sh, x, b);
        if (g.CC16) gmem(reinterpret_cast<uint16_t*>(f.colc))[cbase + e] = (uint16_t)v;
        else gmem(f.colc)[cbase + e] = v;
    }
    for (int b = tid; b < B; b += kAggThreads) {
        uint32_t s = 0;
        for (int x = 0; x < tw; ++x) s += col_get(colh, cw, sh, x, b);
        gmem(f.corner)[((size_t)i * g.nTX + j) * B + b] = s;
    }
}

// Exclusive scan of p[0], p[stride], ... p[(len-1)*stride] in place, starting
// from `run`.  Loads of a chunk are issued before its stores so that many are
// in flight at once.
template <typename T>
__device__ __forceinline__ void scan_seq(IH_GLOBAL T* p, int64_t stride, int len, uint32_t run)
{
    // chunks of C elements, the last one masked: all loads of a chunk go out
    // before any of its stores (a store may alias a later load as far as the
    // compiler knows, so a load issued after it would wait for it)
    constexpr int C = 16;
    for (int k = 0; k < len; k += C) {
        uint32_t v[C];
#pragma unroll
        for (int u = 0; u < C; ++u) v[u] = k + u < len ? p[(k + u) * stride] : 0u;
#pragma unroll
        for (int u = 0; u < C; ++u) {
            if (k + u < len) p[(k + u) * stride] = (T)run;
            run += v[u];
        }
    }
}

template <typename T>
__device__ __forceinline__ uint32_t sum_seq(const IH_GLOBAL T* p, int64_t stride, int len)
{
    constexpr int C = 16;
    uint32_t s = 0;
    for (int k = 0; k < len; k += C) {
        uint32_t v[C];
#pragma unroll
        for (int u = 0; u < C; ++u) v[u] = k + u < len ? p[(k + u) * stride] : 0u;
#pragma unroll
        for (int u = 0; u < C; ++u) s += v[u];
    }
    return s;
}

// ---------------------------------------------------------------------------
// Phase 1, fused schedule: counts and carries of a carry band in one launch
// ---------------------------------------------------------------------------
// One 256-thread block per (carry band I, tile column j): the column counts of
// the band's rows are accumulated tile band by tile band, and after each tile
// band but the last the block stores a snapshot -- the counts so far of every
// column and their sum over the tile column -- for the tile band below it.
// After the last it stores the band's totals.  Then the block reports its
// arrival on two counters.  The last block of tile column j scans the band
// totals of its columns down the carry bands (exclusive, in place): top
// carries at each carry band's first row.  The last block of carry band I
// scans every snapshot of tile-column totals across the tile columns
// (exclusive, in place): counts of the band's rows left of each tile column.
// No block waits for another.  Stores are made visible device-wide before a
// block reports its arrival, and the last block fences before it reads.
template <int TX>
__device__ __forceinline__ void agg_fused_body(const FrameArgs& f, int64_t blk, uint32_t* colh, uint32_t* lutw,
                                               uint32_t* tot, uint32_t* flag)
{
    const Geom& g = f.g;
    const int B = g.B, K = g.K;
    const int I = (int)(blk / g.nTX);
    const int j = (int)(blk - (int64_t)I * g.nTX);
    const int x0 = j * TX;
    const int tw = min(TX, g.W - x0);
    const int Ys = I * K * g.TY;
    const int Ye = min(g.H, Ys + K * g.TY);
    const int nk = (Ye - Ys + g.TY - 1) / g.TY;          // tile bands in this carry band
    const int tid = threadIdx.x;
    IH_GLOBAL uint32_t* colc = gmem(f.colc);
    IH_GLOBAL uint32_t* corner = gmem(f.corner);

    const int cw = col_words(TX, B), sh = col_shift(TX, B);
    for (int e = tid; e < TX * cw; e += kAggThreads) colh[e] = 0;
    for (int b = tid; b < B; b += kAggThreads) tot[b] = 0;
    stage_lut(f, lutw, tid, kAggThreads);
    __syncthreads();
    // A carry band of at most kPre passes of rows: every thread loads and bins
    // all of its pixels of the band at once (one round of loads), then counts
    // them tile band by tile band.  Taller bands load per tile band.
    constexpr int kRowsPerPass = kAggThreads / TX;
    constexpr int kPre = 16;
    const int tr = tid / TX, tx = tid % TX;
    const int rows = Ye - Ys;
    const bool pre = rows <= kPre * kRowsPerPass;           // uniform over the block
    uint32_t q[kPre];
    if (pre) {
        const IH_GLOBAL uint8_t* p = gmem(f.frame) + (size_t)Ys * g.W + x0 + tx;
        uint32_t v[kPre];
#pragma unroll
        for (int u = 0; u < kPre; ++u) {
            const int r = tr + u * kRowsPerPass;
            v[u] = (tx < tw && r < rows) ? (uint32_t)p[(size_t)r * g.W] : 0u;
        }
#pragma unroll
        for (int u = 0; u < kPre; ++u) q[u] = bin_of(f, lutw, v[u], (uint32_t)B);
    }
    for (int k = 0; k < nk; ++k) {
        const int ya = Ys + k * g.TY;
        if (pre) {
            if (tx < tw) {
#pragma unroll
                for (int u = 0; u < kPre; ++u) {
                    const int r = Ys + tr + u * kRowsPerPass;
                    if (r >= ya && r < min(Ye, ya + g.TY)) col_inc(colh, cw, sh, tx, q[u]);
                }
            }
        } else {
            count_rows_as<TX, -1, kBinAny>(f, lutw, colh, ya, min(Ye, ya + g.TY), x0, tw, sh, 0);
        }
        __syncthreads();
        // snapshot k for tile band k + 1 of the carry band, the totals (K - 1) after the last
        const int snap = k + 1 < nk ? k : K - 1;
        const size_t row = (size_t)I * K + snap;
        IH_GLOBAL uint32_t* cdst = colc + (row * g.W + x0) * B;
        if ((kAggThreads % B) == 0) {
            // every element a thread takes is of bin tid % B
            uint32_t part = 0;
            for (int e = tid; e < tw * B; e += kAggThreads) {
                const int x = e / B;
                const uint32_t v = col_get(colh, cw, sh, x, e - x * B);
                cdst[e] = v;
                part += v;
            }
            if (tid < tw * B) atomicAdd(&tot[tid % B], part);
        } else {
            for (int e = tid; e < tw * B; e += kAggThreads) {
                const int x = e / B;
                const uint32_t v = col_get(colh, cw, sh, x, e - x * B);
                cdst[e] = v;
                atomicAdd(&tot[e - x * B], v);
            }
        }
        __syncthreads();
        for (int b = tid; b < B; b += kAggThreads) {
            corner[(row * g.nTX + j) * B + b] = tot[b];
            tot[b] = 0;
        }
    }

    __threadfence();                                      // this block's stores, device-wide
    __syncthreads();
    if (tid == 0) {
        uint32_t* cnt = f.cnt;
        const uint32_t a_col = atomicAdd(&cnt[j], 1u);
        const uint32_t a_band = atomicAdd(&cnt[g.nTX + I], 1u);
        const uint32_t last_col = a_col == (uint32_t)(g.nS - 1);
        const uint32_t last_band = a_band == (uint32_t)(g.nTX - 1);
        // nobody else touches a counter after its last arrival: reset it for the next launch
        if (last_col) atomicExch(&cnt[j], 0u);
        if (last_band) atomicExch(&cnt[g.nTX + I], 0u);
        __threadfence();
        flag[0] = last_col;
        flag[1] = last_band;
    }
    __syncthreads();
    const bool last_col = flag[0] != 0, last_band = flag[1] != 0;
    if (!last_col && !last_band) return;
    __threadfence();                                      // the other blocks' stores, before reading them
    if (last_col) {
        // band totals of columns [x0, x0 + tw): sequences down the carry bands
        IH_GLOBAL uint32_t* base = colc + ((size_t)(K - 1) * g.W + x0) * B;
        const int64_t stride = (int64_t)K * g.W * B;
        for (int e = tid; e < tw * B; e += kAggThreads) scan_seq(base + e, stride, g.nS, 0u);
    }
    if (last_band) {
        // every snapshot row of this carry band, across the tile columns
        // snapshot rows 0 .. nk-2 and the totals (row K-1): nk rows
        for (int q = tid; q < nk * B; q += kAggThreads) {
            const int sidx = q / B, b = q - sidx * B;
            const int snap = sidx < nk - 1 ? sidx : K - 1;
            scan_seq(corner + ((size_t)I * K + snap) * g.nTX * B + b, B, g.nTX, 0u);
        }
    }
}

// Phase 1 of a single frame in one launch: blocks [0, row_blocks) hold four
// row-carry waves each (rows 4 b .. 4 b + 3), the other blocks one tile of
// column counts each; both kinds run side by side and use the dynamic LDS
// buffer by role.  The batched form does the same per frame: a job's jg_begin
// holds its frame's row-block count, followed by the frame's tile blocks.
constexpr int kRowsPerCountBlock = kAggThreads / kWave;

// LDS of a tile block: column counters, the bin table, and for the
// fused schedule B tile-column totals and two flags.
__host__ __device__ inline size_t agg_lds_bytes(int TX, int B)
{
    return (size_t)TX * col_words(TX, B) * 4 + 256 + (size_t)B * 4 + 8;
}

// The tile-block role of the count launch, by schedule.  The fused
// schedule's blocks hold a band of pixels in registers; it is compiled into
// kernels of its own (FUSED), so that the other count kernels keep a small
// register footprint and every block of a launch is resident at once.
template <int TX, bool FUSED>
__device__ __forceinline__ void agg_role(const FrameArgs& f, int64_t blk, uint32_t* lds)
{
    uint32_t* colh = lds;
    uint32_t* lutw = colh + (size_t)TX * col_words(TX, f.g.B);
    if constexpr (FUSED) {
        uint32_t* tot = lutw + 64;
        agg_fused_body<TX>(f, blk, colh, lutw, tot, tot + f.g.B);
    } else {
        agg_body<TX>(f, blk, colh, lutw);
    }
}

template <int TX, bool FUSED>
__global__ __launch_bounds__(kAggThreads)
void count_kernel(FrameArgs f, int32_t row_blocks)
{
    extern __shared__ uint32_t lds[];
    if ((int32_t)blockIdx.x < row_blocks) {
        const int w = wave_in_block();
        const int64_t y = (int64_t)blockIdx.x * kRowsPerCountBlock + w;
        if (y < f.g.H) rowcarry_body(f, y, lds + (size_t)w * (rowcarry_lds_bytes(f.g) / 4));
        return;
    }
    agg_role<TX, FUSED>(f, (int64_t)blockIdx.x - row_blocks, lds);
}

template <int TX, bool FUSED>
__global__ __launch_bounds__(kAggThreads)
void count_batch_kernel(const FrameArgs* __restrict__ frames, const Job* __restrict__ jobs, int32_t njobs)
{
    extern __shared__ uint32_t lds[];
    const Job jb = cload(jobs, find_job(cmem(jobs), njobs, blockIdx.x));
    const FrameArgs f = cload(frames, jb.frame);
    const int64_t local = (int64_t)blockIdx.x - jb.begin;
    if (local < jb.jg_begin) {
        const int w = wave_in_block();
        const int64_t y = local * kRowsPerCountBlock + w;
        if (y < f.g.H) rowcarry_body(f, y, lds + (size_t)w * (rowcarry_lds_bytes(f.g) / 4));
        return;
    }
    agg_role<TX, FUSED>(f, local - jb.jg_begin, lds);
}

// ---------------------------------------------------------------------------
// Phase 2: exclusive scans of the per-tile counts
// ---------------------------------------------------------------------------
// Sequences longer than one chunk are split over the four waves of a block:
// each wave takes a quarter of every sequence of its block's 64, the part
// totals meet in LDS, and each wave rescans its part from the total of the
// parts before it.  The loads of a sequence then go out in one round instead
// of one per chunk.  Shorter sequences take one thread each.

// P is scan_parts(len) (each kernel is compiled for one of the two forms, so
// the one-thread form keeps its small register footprint).  active == false:
// the thread has no sequence but still takes part in the block's exchange
// (every thread of a block sees the same len).  `stride` is the same for the
// whole block, so address arithmetic stays scalar.
template <int P, typename T = uint32_t>
__device__ __forceinline__ void scan_seq_parts(IH_GLOBAL T* p, int64_t stride, int len, bool active,
                                               uint32_t* sums)
{
    if constexpr (P == 1) {
        if (active) scan_seq(p, stride, len, 0u);
        return;
    }
    constexpr int C = 16;
    const int part = (int)threadIdx.x / kWave, lane = (int)threadIdx.x % kWave;
    const int lo = (int)((int64_t)len * part / P), hi = (int)((int64_t)len * (part + 1) / P);
    const bool fits = hi - lo <= C;
    uint32_t v[C];
    uint32_t tot = 0;
    if (active) {
        if (fits) {
#pragma unroll
            for (int u = 0; u < C; ++u) v[u] = lo + u < hi ? p[(int64_t)(lo + u) * stride] : 0u;
#pragma unroll
            for (int u = 0; u < C; ++u) tot += v[u];
        } else {
            tot = sum_seq(p + (int64_t)lo * stride, stride, hi - lo);
        }
    }
    sums[part * kWave + lane] = tot;
    __syncthreads();
    uint32_t run = 0;
    for (int w = 0; w < part; ++w) run += sums[w * kWave + lane];
    if (!active) return;
    if (fits) {
#pragma unroll
        for (int u = 0; u < C; ++u)
            if (lo + u < hi) {
                p[(int64_t)(lo + u) * stride] = (T)run;
                run += v[u];
            }
    } else {
        scan_seq(p + (int64_t)lo * stride, stride, hi - lo, run);
    }
}

// The scan launch.  Its first blocks scan the column counts down the tile
// bands (independent sequences of length nTY, one per column and bin): top
// carries.  The rest scan the tile totals in two dimensions, each block for
// its own bins: first down the bands for every tile column, then -- after a
// block barrier, which makes the first pass's stores visible to the whole
// block -- across the tile columns for every band, leaving corner[i][j][b] =
// the pixels above and to the left of tile (i, j).  `blk` is the block's
// index within the frame's scan blocks.
__device__ __forceinline__ void corner_scan(const FrameArgs& f, int64_t cb, uint32_t* sums)
{
    const Geom& g = f.g;
    const int B = g.B;
    const int nb = corner_bins_per_block(g);
    const int b_lo = (int)cb * nb;
    const int nbh = min(nb, B - b_lo);
    IH_GLOBAL uint32_t* corner = gmem(f.corner) + b_lo;
    const int64_t row = (int64_t)g.nTX * B;                  // words between bands
    if (max(g.nTX, g.nTY) <= kWave) {
        // one sequence per lane and pass, each split over the block's waves
        const int lane = (int)threadIdx.x % kWave;
        const int q1 = g.nTX * nbh, q2 = g.nTY * nbh;         // both <= kWave
        {
            const int j = lane < q1 ? lane / nbh : 0, t = lane < q1 ? lane - j * nbh : 0;
            scan_seq_parts<kScanParts>(corner + (int64_t)j * B + t, row, g.nTY, lane < q1, sums);
        }
        __syncthreads();
        {
            const int i = lane < q2 ? lane / nbh : 0, t = lane < q2 ? lane - i * nbh : 0;
            scan_seq_parts<kScanParts>(corner + i * row + t, B, g.nTX, lane < q2, sums);
        }
        return;
    }
    // larger grids (one bin per block): one sequence per thread
    const int q1 = g.nTX, q2 = g.nTY;
    for (int q = (int)threadIdx.x; q < q1; q += kScanThreads) scan_seq(corner + (int64_t)q * B, row, g.nTY, 0u);
    __syncthreads();
    for (int q = (int)threadIdx.x; q < q2; q += kScanThreads) scan_seq(corner + q * row, B, g.nTX, 0u);
}

template <int P>
__device__ __forceinline__ void scan_body(const FrameArgs& f, int64_t blk, uint32_t* sums)
{
    const Geom& g = f.g;
    const int64_t B = g.B;
    constexpr int per = kScanThreads / P;
    const int64_t ncol = (int64_t)g.W * B;
    const int64_t col_blocks = (ncol + per - 1) / per;
    if (blk >= col_blocks) {                                  // uniform over the block
        corner_scan(f, blk - col_blocks, sums);
        return;
    }
    const int64_t t = blk * per + (int)threadIdx.x % per;
    if (g.CC16)
        scan_seq_parts<P>(gmem(reinterpret_cast<uint16_t*>(f.colc)) + t, (int64_t)g.W * B, g.nTY, t < ncol, sums);
    else
        scan_seq_parts<P>(gmem(f.colc) + t, (int64_t)g.W * B, g.nTY, t < ncol, sums);
}

template <int P>
__global__ __launch_bounds__(kScanThreads)
void scan_kernel(FrameArgs f)
{
    __shared__ uint32_t sums[kScanThreads];
    scan_body<P>(f, blockIdx.x, sums);
}

template <int P>
__global__ __launch_bounds__(kScanThreads)
void scan_batch_kernel(const FrameArgs* __restrict__ frames, const Job* __restrict__ jobs, int32_t njobs)
{
    __shared__ uint32_t sums[kScanThreads];
    const Job jb = cload(jobs, find_job(cmem(jobs), njobs, blockIdx.x));
    const FrameArgs f = cload(frames, jb.frame);
    scan_body<P>(f, (int64_t)blockIdx.x - jb.begin, sums);
}

// ---------------------------------------------------------------------------
// Region query (Sec. 2.1, Eq. 2)
// ---------------------------------------------------------------------------
// Lanes run over bins.  For B >= 64 a wave answers one rectangle (its corners
// are wave-uniform and come in through scalar loads) in chunks of 64 bins;
// for B < 64 a wave answers floor(64 / B) rectangles side by side.  Each
// lane gathers its bin from the four corners -- B contiguous uint32 per
// corner across the lanes -- and writes h(R, b).
constexpr int kQueryThreads = 256;

// Index of entry (x, y, b): bins innermost (H x W x B), or, with BM, the
// bin-major b x h x w layout, where the four corners of a bin lie in its own
// H x W plane (scattered 4-byte gathers instead of B contiguous values).
template <bool BM>
__device__ __forceinline__ size_t entry(int32_t H, int32_t W, int32_t B, int32_t x, int32_t y, int b)
{
    return BM ? ((size_t)b * H + y) * W + x : ((size_t)y * W + x) * B + b;
}

template <bool BM>
__device__ __forceinline__ uint32_t four_corners(const IH_GLOBAL uint32_t* ih, int32_t H, int32_t W, int32_t B,
                                                 int32_t x0, int32_t y0, int32_t x1, int32_t y1, int b)
{
    uint32_t h = ih[entry<BM>(H, W, B, x1, y1, b)];
    if (x0 > 0) h -= ih[entry<BM>(H, W, B, x0 - 1, y1, b)];
    if (y0 > 0) {
        h -= ih[entry<BM>(H, W, B, x1, y0 - 1, b)];
        if (x0 > 0) h += ih[entry<BM>(H, W, B, x0 - 1, y0 - 1, b)];
    }
    return h;
}

template <bool BM>
__global__ __launch_bounds__(kQueryThreads)
void query_kernel(const uint32_t* __restrict__ ih_, int32_t H, int32_t W, int32_t B,
                  const int32_t* __restrict__ rects, int64_t n,
                  uint32_t* __restrict__ hists_, uint32_t* __restrict__ bad)
{
    const IH_GLOBAL uint32_t* ih = gmem(ih_);
    IH_GLOBAL uint32_t* hists = gmem(hists_);
    const int lane = threadIdx.x % kWave;
    const int64_t wave = (int64_t)blockIdx.x * (kQueryThreads / kWave) + wave_in_block();
    if (B >= kWave) {
        const int64_t r = wave;
        if (r >= n) return;
        const IH_CONST int32_t* rc = cmem(rects) + 4 * r;     // one rectangle per wave: scalar loads
        const int32_t x0 = rc[0], y0 = rc[1], x1 = rc[2], y1 = rc[3];
        const bool ok = x0 >= 0 && x0 <= x1 && x1 < W && y0 >= 0 && y0 <= y1 && y1 < H;
        if (!ok && lane == 0 && bad) atomicAdd(bad, 1u);
        for (int b = lane; b < B; b += kWave)
            hists[r * B + b] = ok ? four_corners<BM>(ih, H, W, B, x0, y0, x1, y1, b) : 0u;
    } else {
        const int per = kWave / B;                            // rectangles per wave
        const int sub = lane / B;
        const int b = lane - sub * B;
        const int64_t r = wave * per + sub;
        if (sub >= per || r >= n) return;
        const IH_GLOBAL int32_t* rc = gmem(rects) + 4 * r;
        const int32_t x0 = rc[0], y0 = rc[1], x1 = rc[2], y1 = rc[3];
        const bool ok = x0 >= 0 && x0 <= x1 && x1 < W && y0 >= 0 && y0 <= y1 && y1 < H;
        if (!ok && b == 0 && bad) atomicAdd(bad, 1u);
        hists[r * B + b] = ok ? four_corners<BM>(ih, H, W, B, x0, y0, x1, y1, b) : 0u;
    }
}

// ---------------------------------------------------------------------------
// Phase 3, bin-major layout (the paper's b x h x w, Sec. 3.1 Fig. 2)
// ---------------------------------------------------------------------------
// Entry (x, y, b) at (b * H + y) * W + x.  One wave per (tile band, segment of
// 64 * CPL columns, group of BG <= 16 bins, BG a power of two dividing B);
// lane l owns the CPL columns x0 + CPL l .. x0 + CPL l + CPL - 1, so each bin
// plane gets 256 * CPL contiguous bytes per row from the wave (one store of
// CPL dwords per lane).  CPL = 4 (1 KB runs) suits launches with many items;
// CPL = 1 gives four times the items for small single frames.  For a row and
// a bin, a lane counts the hits h among its CPL pixels; the exclusive prefix
// of those counts across the lanes comes from one ballot per bit of h and
// mbcnt; adding the row's left carry and the lane's own running hits gives
// each column's in-row count.  The column accumulators V[t][c] start from the
// corner and the prefix of the top carries along the segment.  The carry
// phases are the same as for the H x W x B layout with 64-column tiles: a
// segment J starts at carry tile j = CPL * J.
__device__ __forceinline__ uint32_t wave_inclusive_sum(uint32_t v, int lane)
{
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t u = (uint32_t)__builtin_amdgcn_ds_bpermute((lane >= d ? lane - d : lane) * 4, (int)v);
        v += lane >= d ? u : 0u;
    }
    return v;
}

__device__ __forceinline__ uint32_t lanes_below(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

template <int CPL>
__device__ __forceinline__ void store_run(IH_GLOBAL uint32_t* o, const uint32_t (&v)[CPL])
{
    if constexpr (CPL == 1) {
        *o = v[0];
    } else {
        *reinterpret_cast<IH_GLOBAL u32x4*>(o) = u32x4{v[0], v[1], v[2], v[3]};
    }
}

template <int BG, int CPL>
__device__ __forceinline__ void tile_bm_body(const FrameArgs& f, int64_t item)
{
    static_assert(CPL == 1 || CPL == 4, "one or four columns per lane");
    constexpr int kBits = CPL == 1 ? 1 : 3;                          // bits of a lane's hit count (<= CPL)
    const Geom& g = f.g;
    const int B = g.B, H = g.H, W = g.W;
    const int n_groups = B / BG;
    const int nseg = bm_segments(W, CPL);
    const int lane = threadIdx.x % kWave;
    const int grp = (int)(item % n_groups);
    const int64_t seg_item = item / n_groups;
    const int i = (int)(seg_item / nseg), J = (int)(seg_item - (int64_t)i * nseg);
    const int j = J * CPL;                               // carry tile of the segment's first column
    const int xl = J * kWave * CPL + CPL * lane;          // the lane's first column
    const int y0 = i * g.TY, y1 = min(H, y0 + g.TY);
    const int b_lo = grp * BG;
    const int nvalid = max(0, min(CPL, W - xl));         // the lane's columns inside the frame
    // whole, aligned runs: one load of the lane's pixels, one store per bin and row
    const bool vec = nvalid == CPL && (W % CPL) == 0 && ((reinterpret_cast<uintptr_t>(f.frame) & (CPL - 1)) == 0) &&
                     ((reinterpret_cast<uintptr_t>(f.out) & (4 * CPL - 1)) == 0);

    uint32_t V[BG][CPL];
    {
        const IH_GLOBAL uint32_t* cp = gmem(f.corner) + ((size_t)i * g.nTX + j) * B + b_lo;
        const size_t tbase = ((size_t)i * W + xl) * B + b_lo;
        const uint32_t corner = lane < BG ? cp[lane] : 0u;     // lane t: corner of bin b_lo + t
#pragma unroll
        for (int t = 0; t < BG; ++t) {
            uint32_t top[CPL], sum = 0;
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                top[c] = c < nvalid ? top_carry(f, tbase + (size_t)c * B + t) : 0u;
                sum += top[c];
            }
            uint32_t run = (uint32_t)__builtin_amdgcn_readlane((int)corner, t) + wave_inclusive_sum(sum, lane) - sum;
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                run += top[c];
                V[t][c] = run;
            }
        }
    }
    const IH_GLOBAL uint8_t* frame = gmem(f.frame);
    const size_t rowc_base = (size_t)j * H * B + b_lo;
    IH_GLOBAL uint32_t* out = gmem(f.out);
    const size_t plane = (size_t)H * W;
    // Pixels (CPL per lane, packed) and left carries come 8 rows at a time, a
    // chunk ahead: lane t holds the carry of bin b_lo + t; rows past the band
    // are clamped.
    constexpr int CH = 8;
    uint32_t cq[CH], cc[CH], nq[CH], nc[CH];
    auto load_chunk = [&](int yc, uint32_t (&q)[CH], uint32_t (&c)[CH]) {
#pragma unroll
        for (int r = 0; r < CH; ++r) {
            const int row = min(yc + r, y1 - 1);
            const IH_GLOBAL uint8_t* p = frame + (size_t)row * W + xl;
            if constexpr (CPL == 4) {
                if (vec) {
                    q[r] = *reinterpret_cast<const IH_GLOBAL uint32_t*>(p);
                } else {
                    uint32_t w = 0;
                    for (int k = 0; k < nvalid; ++k) w |= (uint32_t)p[k] << (8 * k);
                    q[r] = w;
                }
            } else {
                uint32_t w = 0;
#pragma unroll
                for (int k = 0; k < CPL; ++k)
                    if (k < nvalid) w |= (uint32_t)p[k] << (8 * k);
                q[r] = w;
            }
            c[r] = lane < BG ? left_carry(f, rowc_base + (size_t)row * B + lane) : 0u;
        }
    };
    load_chunk(y0, cq, cc);
    for (int yc = y0; yc < y1; yc += CH) {
        const bool more = yc + CH < y1;
        if (more) load_chunk(yc + CH, nq, nc);
#pragma unroll
        for (int r = 0; r < CH; ++r) {
            const int y = yc + r;
            if (y < y1) {
                // bins of the lane's pixels; 256 (no bin) past the frame
                uint32_t q[CPL];
#pragma unroll
                for (int c = 0; c < CPL; ++c)
                    q[c] = c < nvalid ? (((cq[r] >> (8 * c)) & 0xFFu) * (uint32_t)B) >> 8 : 256u;
                IH_GLOBAL uint32_t* orow = out + (size_t)b_lo * plane + (size_t)y * W + xl;
#pragma unroll
                for (int t = 0; t < BG; ++t) {
                    const uint32_t b = (uint32_t)(b_lo + t);
                    uint32_t h[CPL], s = 0;
#pragma unroll
                    for (int c = 0; c < CPL; ++c) {
                        h[c] = q[c] == b ? 1u : 0u;
                        s += h[c];
                    }
                    uint32_t below = 0;
#pragma unroll
                    for (int k = 0; k < kBits; ++k)
                        below += lanes_below(__builtin_amdgcn_ballot_w64(((s >> k) & 1u) != 0)) << k;
                    uint32_t run = (uint32_t)__builtin_amdgcn_readlane((int)cc[r], t) + below;
#pragma unroll
                    for (int c = 0; c < CPL; ++c) {
                        run += h[c];
                        V[t][c] += run;
                    }
                    IH_GLOBAL uint32_t* o = orow + (size_t)t * plane;
                    if (vec) {
                        store_run<CPL>(o, V[t]);
                    } else {
#pragma unroll
                        for (int c = 0; c < CPL; ++c)
                            if (c < nvalid) o[c] = V[t][c];
                    }
                }
            }
        }
        if (more) {
#pragma unroll
            for (int r = 0; r < CH; ++r) {
                cq[r] = nq[r];
                cc[r] = nc[r];
            }
        }
    }
}

template <int BG, int CPL>
__global__ __launch_bounds__(kWave * kWavesPerBlock)
void tile_bm_kernel(FrameArgs f)
{
    const int64_t item = (int64_t)blockIdx.x * kWavesPerBlock + wave_in_block();
    if (item >= tile_bm_items_of(f.g, BG)) return;                     // whole wave leaves together
    tile_bm_body<BG, CPL>(f, item);
}

// Many bin-major frames with the same bin group BG and columns per lane CPL:
// one wave per item over the job table (a job per frame, `begin` its first
// item).
template <int BG, int CPL>
__global__ __launch_bounds__(kWave * kWavesPerBlock)
void tile_bm_batch_kernel(const FrameArgs* __restrict__ frames, const Job* __restrict__ jobs, int32_t njobs,
                          int64_t nitems)
{
    const int64_t item = (int64_t)blockIdx.x * kWavesPerBlock + wave_in_block();
    if (item >= nitems) return;                                        // whole wave leaves together
    const Job jb = cload(jobs, find_job(cmem(jobs), njobs, item));
    const FrameArgs f = cload(frames, jb.frame);
    tile_bm_body<BG, CPL>(f, item - jb.begin);
}

// ---------------------------------------------------------------------------
// Write reference: the tile pass's store stream with nothing else
// ---------------------------------------------------------------------------
// Same work items, lanes and store order as the tile pass for B <= 64 (one
// bin per lane, kWave / B segments of TX columns per wave, TY-row bands), but
// no loads and no arithmetic: each entry gets its row index.  Measures what
// the device's write path reaches in the tile pass's geometry.
template <int TX>
__global__ __launch_bounds__(kWave * kWavesPerBlock)
void write_reference_kernel(uint32_t* out_, int32_t H, int32_t W, int32_t B, int32_t TY, int32_t nJG, int32_t S)
{
    IH_GLOBAL uint32_t* out = gmem(out_);
    const int64_t item = (int64_t)blockIdx.x * kWavesPerBlock + wave_in_block();
    const int nTY = (H + TY - 1) / TY;
    if (item >= (int64_t)nTY * nJG) return;
    const int i = (int)(item / nJG), jg = (int)(item - (int64_t)i * nJG);
    const int lane = threadIdx.x % kWave;
    const int s = lane / B, b = lane - s * B;
    const int x0 = (jg * S + s) * TX;
    if (s >= S || x0 >= W) return;
    const int ncols = min(TX, W - x0);
    const int y0 = i * TY, y1 = min(H, y0 + TY);
    for (int y = y0; y < y1; ++y) {
        IH_GLOBAL uint32_t* orow = out + ((size_t)y * W + x0) * B + b;
#pragma unroll
        for (int k = 0; k < TX; ++k)
            if (k < ncols) orow[(size_t)k * B] = (uint32_t)y;
    }
}

hipError_t launch_write_reference(uint32_t* out, int32_t H, int32_t W, int32_t B, int32_t TX, int32_t TY,
                                  hipStream_t stream)
{
    const int32_t S = kWave / B;
    const int32_t nTX = (W + TX - 1) / TX, nJG = (nTX + S - 1) / S;
    const int64_t items = (int64_t)((H + TY - 1) / TY) * nJG;
    const unsigned blocks = (unsigned)((items + kWavesPerBlock - 1) / kWavesPerBlock);
    const dim3 grid(blocks), block(kWave * kWavesPerBlock);
    if (TX == 32)
        hipLaunchKernelGGL(write_reference_kernel<32>, grid, block, 0, stream, out, H, W, B, TY, nJG, S);
    else if (TX == 64)
        hipLaunchKernelGGL(write_reference_kernel<64>, grid, block, 0, stream, out, H, W, B, TY, nJG, S);
    else
        hipLaunchKernelGGL(write_reference_kernel<128>, grid, block, 0, stream, out, H, W, B, TY, nJG, S);
    return hipGetLastError();
}

// A bin table passed by value as a kernel argument, written to device memory.
struct LutArg {
    uint32_t w[64];
};
__global__ __launch_bounds__(kWave)
void lut_store_kernel(LutArg a, uint32_t* dst)
{
    dst[threadIdx.x] = a.w[threadIdx.x];
}

// ---------------------------------------------------------------------------
// host side: launches (geometry and tile choice live in ih_geom.cpp, the
// tile kernels in ih_tile_*.hip)
// ---------------------------------------------------------------------------
// The count kernel of a tile width and schedule (single-frame or batched form).
static const void* count_fn(int TX, bool fused, bool batched)
{
    if (batched) {
        if (fused)
            return TX == 32 ? reinterpret_cast<const void*>(&count_batch_kernel<32, true>)
                 : TX == 128 ? reinterpret_cast<const void*>(&count_batch_kernel<128, true>)
                             : reinterpret_cast<const void*>(&count_batch_kernel<64, true>);
        return TX == 32 ? reinterpret_cast<const void*>(&count_batch_kernel<32, false>)
             : TX == 128 ? reinterpret_cast<const void*>(&count_batch_kernel<128, false>)
                         : reinterpret_cast<const void*>(&count_batch_kernel<64, false>);
    }
    if (fused)
        return TX == 32 ? reinterpret_cast<const void*>(&count_kernel<32, true>)
             : TX == 128 ? reinterpret_cast<const void*>(&count_kernel<128, true>)
                         : reinterpret_cast<const void*>(&count_kernel<64, true>);
    return TX == 32 ? reinterpret_cast<const void*>(&count_kernel<32, false>)
         : TX == 128 ? reinterpret_cast<const void*>(&count_kernel<128, false>)
                     : reinterpret_cast<const void*>(&count_kernel<64, false>);
}

hipError_t preload_kernels()
{
    std::vector<const void*> fns = {
        reinterpret_cast<const void*>(&count_kernel<32, false>), reinterpret_cast<const void*>(&count_kernel<64, false>),
        reinterpret_cast<const void*>(&count_kernel<128, false>), reinterpret_cast<const void*>(&count_kernel<32, true>),
        reinterpret_cast<const void*>(&count_kernel<64, true>), reinterpret_cast<const void*>(&count_kernel<128, true>),
        reinterpret_cast<const void*>(&count_batch_kernel<32, false>),
        reinterpret_cast<const void*>(&count_batch_kernel<64, false>),
        reinterpret_cast<const void*>(&count_batch_kernel<128, false>),
        reinterpret_cast<const void*>(&count_batch_kernel<32, true>),
        reinterpret_cast<const void*>(&count_batch_kernel<64, true>),
        reinterpret_cast<const void*>(&count_batch_kernel<128, true>),
        reinterpret_cast<const void*>(&scan_kernel<1>), reinterpret_cast<const void*>(&scan_kernel<kScanParts>),
        reinterpret_cast<const void*>(&scan_batch_kernel<1>),
        reinterpret_cast<const void*>(&scan_batch_kernel<kScanParts>),
        reinterpret_cast<const void*>(&query_kernel<false>), reinterpret_cast<const void*>(&query_kernel<true>),
        reinterpret_cast<const void*>(&lut_store_kernel)};
    // one kernel of every tile-pass source (each source is one code object)
    const TileVariant vs[] = {{1, 64, 64, false, false, false}, {1, 64, 64, false, true, false},
                              {1, 64, 64, true, false, false}, {1, 64, 64, true, true, false},
                              {1, 64, 0, false, false, true}};
    for (const TileVariant& v : vs) {
        const TileFns f = tile_fns(v);
        fns.push_back(f.single);
        fns.push_back(f.batch);
    }
    for (const void* fn : fns) {
        hipFuncAttributes attr;
        hipError_t e = hipFuncGetAttributes(&attr, fn);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

int64_t scan_blocks(const Geom& g)
{
    const int64_t per = scan_per_block(g.nTY);
    const int nb = corner_bins_per_block(g);
    return ((int64_t)g.W * g.B + per - 1) / per + (g.B + nb - 1) / nb;
}

hipError_t launch_phase(Phase ph, const FrameArgs& f, bool nontemporal, hipStream_t stream)
{
    const Geom& g = f.g;
    switch (ph) {
    case Phase::kAgg: {
        const int32_t row_blocks = count_row_blocks(g);
        const unsigned blocks = (unsigned)row_blocks + (unsigned)count_tile_blocks(g);
        const size_t lds = count_lds(g);
        const void* fn = count_fn(g.TX, g.K != 0, false);
        FrameArgs fa = f;
        int32_t rb = row_blocks;
        void* args[] = {&fa, &rb};
        hipError_t e = hipLaunchKernel(fn, dim3(blocks), dim3(kAggThreads), args, lds, stream);
        if (e != hipSuccess) return e;
        break;
    }
    case Phase::kScan:
        if (g.K || g.PC) break;         // fused or prefix counts: no scan launch
        if (scan_parts(g.nTY) == 1)
            hipLaunchKernelGGL(scan_kernel<1>, dim3((unsigned)scan_blocks(g)), dim3(kScanThreads), 0, stream, f);
        else
            hipLaunchKernelGGL(scan_kernel<kScanParts>, dim3((unsigned)scan_blocks(g)), dim3(kScanThreads), 0,
                               stream, f);
        break;
    case Phase::kTile: {
        const int32_t n_int = interior_groups(g, f.frame, f.out);
        const int32_t parts[2][2] = {{0, n_int}, {n_int, g.nJG - n_int}};
        for (int p = 0; p < 2; ++p) {
            int32_t begin = parts[p][0], count = parts[p][1];
            if (count <= 0) continue;
            const int64_t items = (int64_t)g.nTY * count;
            const unsigned blocks = (unsigned)((items + kWavesPerBlock - 1) / kWavesPerBlock);
            const TileFns fn = tile_fns(tile_variant(g, nontemporal, p == 1, f.lut != nullptr));
            FrameArgs fa = f;
            void* args[] = {&fa, &begin, &count};
            hipError_t e = hipLaunchKernel(fn.single, dim3(blocks), dim3(kWave * kWavesPerBlock),
                                           args, 0, stream);
            if (e != hipSuccess) return e;
        }
        break;
    }
    }
    return hipGetLastError();
}

int32_t count_row_blocks(const Geom& g) { return (g.H + kRowsPerCountBlock - 1) / kRowsPerCountBlock; }

size_t count_lds(const Geom& g)
{
    return std::max(kRowsPerCountBlock * rowcarry_lds_bytes(g), agg_lds_bytes(g.TX, g.B));
}

hipError_t launch_count_batch(int TX, bool fused, const FrameArgs* frames, const Job* jobs, int32_t njobs,
                              int64_t nblocks, size_t lds_bytes, hipStream_t stream)
{
    if (nblocks <= 0) return hipSuccess;
    const void* fn = count_fn(TX, fused, true);
    const FrameArgs* fa = frames;
    const Job* jb = jobs;
    int32_t nj = njobs;
    void* args[] = {&fa, &jb, &nj};
    return hipLaunchKernel(fn, dim3((unsigned)nblocks), dim3(kAggThreads), args, lds_bytes, stream);
}

hipError_t launch_scan_batch(int parts, const FrameArgs* frames, const Job* jobs, int32_t njobs, int64_t nblocks,
                             hipStream_t stream)
{
    if (nblocks <= 0) return hipSuccess;
    const dim3 grid((unsigned)nblocks), block(kScanThreads);
    if (parts == 1)
        hipLaunchKernelGGL(scan_batch_kernel<1>, grid, block, 0, stream, frames, jobs, njobs);
    else
        hipLaunchKernelGGL(scan_batch_kernel<kScanParts>, grid, block, 0, stream, frames, jobs, njobs);
    return hipGetLastError();
}

hipError_t launch_tile_batch(const TileVariant& v, const FrameArgs* frames, const Job* jobs,
                             int32_t njobs, int64_t nitems, int32_t grid, uint32_t* sched, hipStream_t stream)
{
    if (nitems <= 0) return hipSuccess;
    const TileFns fn = tile_fns(v);
    void* args[] = {&frames, &jobs, &njobs, &nitems, &sched};
    hipError_t e = hipLaunchKernel(fn.batch, dim3((unsigned)grid), dim3(kWave * kWavesPerBlock), args, 0, stream);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

int32_t tile_resident_blocks(const TileVariant& v)
{
    const TileFns fn = tile_fns(v);
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 1024;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn.batch, kWave * kWavesPerBlock, 0) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    return cus * per_cu;
}

// Largest power of two up to 16 that divides B: the bins of one bin-major
// work item (more bins per item keep more ballot masks and carries live than
// the scalar registers hold).
int bm_group(int B)
{
    int bg = 16;
    while (B % bg != 0) bg >>= 1;
    return bg;
}

template <int CPL>
static void launch_bm_single(int bg, const FrameArgs& f, unsigned blocks, hipStream_t stream)
{
    const dim3 grid(blocks), block(kWave * kWavesPerBlock);
    switch (bg) {
    case 16: hipLaunchKernelGGL((tile_bm_kernel<16, CPL>), grid, block, 0, stream, f); break;
    case 8: hipLaunchKernelGGL((tile_bm_kernel<8, CPL>), grid, block, 0, stream, f); break;
    case 4: hipLaunchKernelGGL((tile_bm_kernel<4, CPL>), grid, block, 0, stream, f); break;
    case 2: hipLaunchKernelGGL((tile_bm_kernel<2, CPL>), grid, block, 0, stream, f); break;
    default: hipLaunchKernelGGL((tile_bm_kernel<1, CPL>), grid, block, 0, stream, f); break;
    }
}

hipError_t launch_tile_bm(const FrameArgs& f, hipStream_t stream)
{
    const int64_t items = tile_bm_items(f.g);
    const unsigned blocks = (unsigned)((items + kWavesPerBlock - 1) / kWavesPerBlock);
    if (f.g.CPL == 4) launch_bm_single<4>(bm_group(f.g.B), f, blocks, stream);
    else launch_bm_single<1>(bm_group(f.g.B), f, blocks, stream);
    return hipGetLastError();
}

int64_t tile_bm_items(const Geom& g) { return tile_bm_items_of(g, bm_group(g.B)); }

template <int CPL>
static void launch_bm_batch(int bg, const FrameArgs* frames, const Job* jobs, int32_t njobs, int64_t nitems,
                            hipStream_t stream)
{
    const unsigned blocks = (unsigned)((nitems + kWavesPerBlock - 1) / kWavesPerBlock);
    const dim3 grid(blocks), block(kWave * kWavesPerBlock);
    switch (bg) {
    case 16: hipLaunchKernelGGL((tile_bm_batch_kernel<16, CPL>), grid, block, 0, stream, frames, jobs, njobs, nitems); break;
    case 8: hipLaunchKernelGGL((tile_bm_batch_kernel<8, CPL>), grid, block, 0, stream, frames, jobs, njobs, nitems); break;
    case 4: hipLaunchKernelGGL((tile_bm_batch_kernel<4, CPL>), grid, block, 0, stream, frames, jobs, njobs, nitems); break;
    case 2: hipLaunchKernelGGL((tile_bm_batch_kernel<2, CPL>), grid, block, 0, stream, frames, jobs, njobs, nitems); break;
    default: hipLaunchKernelGGL((tile_bm_batch_kernel<1, CPL>), grid, block, 0, stream, frames, jobs, njobs, nitems); break;
    }
}

hipError_t launch_tile_bm_batch(int bg, int cpl, const FrameArgs* frames, const Job* jobs, int32_t njobs,
                                int64_t nitems, hipStream_t stream)
{
    if (nitems <= 0) return hipSuccess;
    if (cpl == 4) launch_bm_batch<4>(bg, frames, jobs, njobs, nitems, stream);
    else launch_bm_batch<1>(bg, frames, jobs, njobs, nitems, stream);
    return hipGetLastError();
}

hipError_t launch_lut_store(const uint8_t* lut_host, uint32_t* dst, hipStream_t stream)
{
    LutArg a;
    memcpy(a.w, lut_host, sizeof a.w);
    hipLaunchKernelGGL(lut_store_kernel, dim3(1), dim3(kWave), 0, stream, a, dst);
    return hipGetLastError();
}

hipError_t launch_query(const uint32_t* ih, int32_t H, int32_t W, int32_t B,
                        const int32_t* rects, int64_t n, uint32_t* hists,
                        uint32_t* bad_count, bool binmajor, hipStream_t stream)
{
    if (n == 0) return hipSuccess;
    const int64_t per = B >= kWave ? 1 : kWave / B;           // rectangles per wave
    const int64_t waves = (n + per - 1) / per;
    const int64_t blocks = (waves + kQueryThreads / kWave - 1) / (kQueryThreads / kWave);
    if (binmajor)
        hipLaunchKernelGGL(query_kernel<true>, dim3((unsigned)blocks), dim3(kQueryThreads), 0, stream,
                           ih, H, W, B, rects, n, hists, bad_count);
    else
        hipLaunchKernelGGL(query_kernel<false>, dim3((unsigned)blocks), dim3(kQueryThreads), 0, stream,
                           ih, H, W, B, rects, n, hists, bad_count);
    return hipGetLastError();
}

}  // namespace ih
