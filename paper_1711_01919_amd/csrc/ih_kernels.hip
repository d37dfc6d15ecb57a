// HIP kernels (gfx950) for the exact integral histogram and its region query.
//
// The integral histogram (Sec. 2.1, Eq. 1) is a 2-D inclusive prefix count
// per bin.  It is computed by reduce-then-scan over TY x TX tiles:
//
//   1. agg_kernel     per tile: bin counts of every tile-row segment, of every
//                     tile column, and of the whole tile (LDS atomics, one
//                     pass over the uint8 pixels).
//   2. scan kernels   exclusive scans of those counts across tiles, giving for
//                     each tile its left carry per row, its top carry per
//                     column, and its top-left corner count.
//   3. tile_kernel    the hot pass: each lane owns BPL bins of one tile
//                     segment; it bins each pixel of the row (binning is fused
//                     here, the one-hot tensor is never stored), scans the row
//                     in-lane, adds the row into TX column accumulators held in
//                     VGPRs, and stores the finished H x W x B entries.
//
// For entry (x, y, b) of a tile whose top-left pixel is (x0, y0):
//   H(x,y,b) = corner(b) + sum_{x0<=x'<=x} top(x',b)
//            + sum_{y0<=y'<=y} left(y',b) + local(x,y,b)
// where top/left/corner count the pixels above / to the left / above-left of
// the tile.  This is the inclusion-exclusion of Eq. 1 over the four regions;
// all arithmetic is exact uint32.
#include "ih_internal.h"

namespace ih {

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Phase 1: per-tile bin counts
// ---------------------------------------------------------------------------
constexpr int kAggThreads = 256;
constexpr int kAggRows = 32;     // rows whose segment counts are held in LDS at once

// Two 16-bit counters per LDS word: row-segment counts are <= TX and column
// counts are <= TY, both far below 2^16, so a carry never crosses halves.
__device__ __forceinline__ void lds_inc16(uint32_t* h, uint32_t e)
{
    atomicAdd(&h[e >> 1], 1u << ((e & 1u) << 4));
}
__device__ __forceinline__ uint32_t lds_get16(const uint32_t* h, uint32_t e)
{
    return (h[e >> 1] >> ((e & 1u) << 4)) & 0xFFFFu;
}

template <int TX>
__global__ __launch_bounds__(kAggThreads)
void agg_kernel(const uint8_t* __restrict__ frame, Geom g,
                uint32_t* __restrict__ rowc, uint32_t* __restrict__ colc,
                uint32_t* __restrict__ corner)
{
    __shared__ uint32_t rowh[kAggRows * 256 / 2];
    __shared__ uint32_t colh[TX * 256 / 2];
    constexpr int kRowsPerPass = kAggThreads / TX;

    const int B = g.B;
    const int tile = blockIdx.x;
    const int i = tile / g.nTX;
    const int j = tile - i * g.nTX;
    const int x0 = j * TX, y0 = i * g.TY;
    const int tw = min(TX, g.W - x0);
    const int th = min(g.TY, g.H - y0);
    const int tid = threadIdx.x;
    const int tr = tid / TX, tx = tid % TX;

    for (int e = tid; e < (TX * B + 1) / 2; e += kAggThreads) colh[e] = 0;

    for (int yc = 0; yc < th; yc += kAggRows) {
        const int rows = min(kAggRows, th - yc);
        for (int e = tid; e < (rows * B + 1) / 2; e += kAggThreads) rowh[e] = 0;
        __syncthreads();                  // also orders the colh clearing before the first chunk
        if (tx < tw) {
            for (int r = tr; r < rows; r += kRowsPerPass) {
                const uint32_t v = frame[(size_t)(y0 + yc + r) * g.W + x0 + tx];
                const uint32_t q = (v * (uint32_t)B) >> 8;
                lds_inc16(rowh, (uint32_t)(r * B) + q);
                lds_inc16(colh, (uint32_t)(tx * B) + q);
            }
        }
        __syncthreads();
        for (int e = tid; e < rows * B; e += kAggThreads) {
            const int r = e / B;
            const int b = e - r * B;
            rowc[((size_t)(y0 + yc + r) * g.nTX + j) * B + b] = lds_get16(rowh, (uint32_t)e);
        }
        __syncthreads();
    }
    for (int e = tid; e < tw * B; e += kAggThreads)
        colc[((size_t)i * g.W + x0) * B + e] = lds_get16(colh, (uint32_t)e);
    for (int b = tid; b < B; b += kAggThreads) {
        uint32_t s = 0;
        for (int x = 0; x < tw; ++x) s += lds_get16(colh, (uint32_t)(x * B + b));
        corner[((size_t)i * g.nTX + j) * B + b] = s;
    }
}

// ---------------------------------------------------------------------------
// Phase 2: exclusive scans of the per-tile counts
// ---------------------------------------------------------------------------
constexpr int kScanThreads = 256;

// Row segments across tile columns, column counts across tile bands, and tile
// totals across bands -- all independent sequences, one thread each.
__global__ __launch_bounds__(kScanThreads)
void scan_a_kernel(Geom g, uint32_t* __restrict__ rowc, uint32_t* __restrict__ colc,
                   uint32_t* __restrict__ corner)
{
    const int64_t B = g.B;
    int64_t t = (int64_t)blockIdx.x * kScanThreads + threadIdx.x;
    const int64_t nrow = (int64_t)g.H * B, ncol = (int64_t)g.W * B, ntot = (int64_t)g.nTX * B;
    uint32_t* p;
    int64_t stride;
    int len;
    if (t < nrow) {
        const int64_t y = t / B, b = t - y * B;
        p = rowc + y * g.nTX * B + b;
        stride = B;
        len = g.nTX;
    } else if ((t -= nrow) < ncol) {
        p = colc + t;
        stride = (int64_t)g.W * B;
        len = g.nTY;
    } else if ((t -= ncol) < ntot) {
        p = corner + t;
        stride = (int64_t)g.nTX * B;
        len = g.nTY;
    } else {
        return;
    }
    uint32_t run = 0;
    for (int k = 0; k < len; ++k) {
        const uint32_t v = p[k * stride];
        p[k * stride] = run;
        run += v;
    }
}

// Band-scanned tile totals across tile columns: corner[i][j][b] becomes the
// count of pixels above and to the left of tile (i, j).
__global__ __launch_bounds__(kScanThreads)
void scan_b_kernel(Geom g, uint32_t* __restrict__ corner)
{
    const int64_t B = g.B;
    const int64_t t = (int64_t)blockIdx.x * kScanThreads + threadIdx.x;
    if (t >= (int64_t)g.nTY * B) return;
    const int64_t i = t / B, b = t - i * B;
    uint32_t* p = corner + i * g.nTX * B + b;
    uint32_t run = 0;
    for (int k = 0; k < g.nTX; ++k) {
        const uint32_t v = p[k * B];
        p[k * B] = run;
        run += v;
    }
}

// ---------------------------------------------------------------------------
// Phase 3: the tile pass (hot loop)
// ---------------------------------------------------------------------------
template <int BPL, bool NT>
__device__ __forceinline__ void store_bins(uint32_t* p, const uint32_t (&v)[BPL])
{
    if constexpr (BPL == 1) {
        if constexpr (NT) __builtin_nontemporal_store(v[0], p);
        else *p = v[0];
    } else if constexpr (BPL == 2) {
        u32x2 w = {v[0], v[1]};
        if constexpr (NT) __builtin_nontemporal_store(w, reinterpret_cast<u32x2*>(p));
        else *reinterpret_cast<u32x2*>(p) = w;
    } else {
        u32x4 w = {v[0], v[1], v[2], v[3]};
        if constexpr (NT) __builtin_nontemporal_store(w, reinterpret_cast<u32x4*>(p));
        else *reinterpret_cast<u32x4*>(p) = w;
    }
}

struct RowArgs {
    const uint8_t* frame;
    uint32_t* out;
    const uint32_t* rowc;
    int32_t W, nTX, B, j, x0, b0, ncols;
    bool vec_ok;
};

// Rows y0..y1-1 of one tile segment.  GUARD=false is the interior path (the
// whole wave has full, aligned segments); GUARD=true handles ragged right
// edges, unaligned frames and partial bin groups with per-step predicates.
template <int BPL, int TX, bool NT, bool GUARD>
__device__ __forceinline__ void tile_rows(const RowArgs& a, int y0, int y1,
                                          const uint32_t (&lo)[BPL], const uint32_t (&wd)[BPL],
                                          const bool (&bvalid)[BPL], uint32_t (&V)[BPL][TX])
{
    for (int y = y0; y < y1; ++y) {
        // Left carry of this row: pixels of row y left of the segment, per bin.
        uint32_t cnt[BPL];
        const uint32_t* rp = a.rowc + ((size_t)y * a.nTX + a.j) * a.B + a.b0;
#pragma unroll
        for (int t = 0; t < BPL; ++t) cnt[t] = bvalid[t] ? rp[t] : 0u;

        uint32_t px[TX / 4];
        const uint8_t* prow = a.frame + (size_t)y * a.W + a.x0;
        if constexpr (!GUARD) {
#pragma unroll
            for (int q = 0; q < TX / 16; ++q) {
                const u32x4 w = *reinterpret_cast<const u32x4*>(prow + 16 * q);
                px[4 * q + 0] = w.x; px[4 * q + 1] = w.y;
                px[4 * q + 2] = w.z; px[4 * q + 3] = w.w;
            }
        } else {
#pragma unroll
            for (int q = 0; q < TX / 4; ++q) px[q] = 0u;
#pragma unroll
            for (int k = 0; k < TX; ++k)
                if (k < a.ncols) px[k / 4] |= (uint32_t)prow[k] << (8 * (k % 4));
        }

        uint32_t* orow = a.out + ((size_t)y * a.W + a.x0) * a.B + a.b0;
#pragma unroll
        for (int k = 0; k < TX; ++k) {
            const uint32_t v = (px[k / 4] >> (8 * (k % 4))) & 0xFFu;
            uint32_t o[BPL];
#pragma unroll
            for (int t = 0; t < BPL; ++t) {
                cnt[t] += (v - lo[t]) < wd[t] ? 1u : 0u;      // in-lane row scan
                V[t][k] += cnt[t];                            // column accumulation
                o[t] = V[t][k];
            }
            if constexpr (!GUARD) {
                store_bins<BPL, NT>(orow + (size_t)k * a.B, o);
            } else if (k < a.ncols) {
                if (a.vec_ok) {
                    store_bins<BPL, NT>(orow + (size_t)k * a.B, o);
                } else {
#pragma unroll
                    for (int t = 0; t < BPL; ++t)
                        if (bvalid[t]) orow[(size_t)k * a.B + t] = o[t];
                }
            }
        }
    }
}

// One wave per work item: tile band i (TY rows) x column group jg (S adjacent
// tile segments).  GUARD=false requires every active segment of every launched
// group to be TX columns wide, the frame and W 16-byte aligned, B % BPL == 0
// and out aligned to 4*BPL bytes; the host launches GUARD=true for the rest.
template <int BPL, int TX, int BC, bool NT, bool GUARD>
__global__ __launch_bounds__(kWave * kWavesPerBlock)
void tile_kernel(const uint8_t* __restrict__ frame, uint32_t* __restrict__ out,
                 const uint32_t* __restrict__ rowc, const uint32_t* __restrict__ colc,
                 const uint32_t* __restrict__ corner, Geom g, int32_t jg_begin, int32_t jg_count)
{
    static_assert(TX % 16 == 0, "pixel rows are loaded 16 bytes at a time");
    constexpr int LC = BC ? (BC + BPL - 1) / BPL : 1;
    const int B = BC ? BC : g.B;
    const int L = BC ? LC : g.L;
    const int S = BC ? kWave / LC : g.S;

    const int lane = threadIdx.x % kWave;
    const int64_t item = (int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    if (item >= (int64_t)g.nTY * jg_count) return;        // whole wave leaves together
    const int i = (int)(item / jg_count);
    const int jg = jg_begin + (int)(item - (int64_t)i * jg_count);
    const int s = lane / L;
    const int b0 = (lane - s * L) * BPL;
    const int j = jg * S + s;
    const bool active = (s < S) && (j < g.nTX) && (b0 < B);
    if (!active) return;
    const int x0 = j * TX;
    const int ncols = GUARD ? min(TX, g.W - x0) : TX;
    const int y0 = i * g.TY;
    const int y1 = min(g.H, y0 + g.TY);

    // Bin b holds the values v with ceil(256 b / B) <= v < ceil(256 (b+1) / B),
    // which is floor(v B / 256) == b.  A lane tests v - lo < width (unsigned).
    uint32_t lo[BPL], wd[BPL];
    bool bvalid[BPL];
#pragma unroll
    for (int t = 0; t < BPL; ++t) {
        const int b = b0 + t;
        bvalid[t] = GUARD ? b < B : true;
        const uint32_t l = (uint32_t)(256 * b + B - 1) / (uint32_t)B;
        const uint32_t h = (uint32_t)(256 * (b + 1) + B - 1) / (uint32_t)B;
        lo[t] = bvalid[t] ? l : 0u;
        wd[t] = bvalid[t] ? h - l : 0u;
    }

    // Column state: corner + running sum of the top carries along the segment.
    uint32_t V[BPL][TX];
    {
        uint32_t acc[BPL];
        const uint32_t* cp = corner + ((size_t)i * g.nTX + j) * B + b0;
        const uint32_t* tp = colc + ((size_t)i * g.W + x0) * B + b0;
#pragma unroll
        for (int t = 0; t < BPL; ++t) acc[t] = bvalid[t] ? cp[t] : 0u;
#pragma unroll
        for (int k = 0; k < TX; ++k) {
#pragma unroll
            for (int t = 0; t < BPL; ++t) {
                if (k < ncols && bvalid[t]) acc[t] += tp[(size_t)k * B + t];
                V[t][k] = acc[t];
            }
        }
    }

    const bool vec_ok = (b0 + BPL <= B) && (B % BPL == 0) &&
                        ((reinterpret_cast<uintptr_t>(out) & (4 * BPL - 1)) == 0);
    RowArgs a{frame, out, rowc, g.W, g.nTX, B, j, x0, b0, ncols, vec_ok};
    tile_rows<BPL, TX, NT, GUARD>(a, y0, y1, lo, wd, bvalid, V);
}

// ---------------------------------------------------------------------------
// Region query (Sec. 2.1, Eq. 2): one thread per (rectangle, bin)
// ---------------------------------------------------------------------------
constexpr int kQueryThreads = 256;

__global__ __launch_bounds__(kQueryThreads)
void query_kernel(const uint32_t* __restrict__ ih, int32_t H, int32_t W, int32_t B,
                  const int32_t* __restrict__ rects, int64_t n,
                  uint32_t* __restrict__ hists, uint32_t* __restrict__ bad)
{
    const int64_t t = (int64_t)blockIdx.x * kQueryThreads + threadIdx.x;
    if (t >= n * B) return;
    const int64_t r = t / B;
    const int b = (int)(t - r * B);
    const int32_t x0 = rects[4 * r + 0], y0 = rects[4 * r + 1];
    const int32_t x1 = rects[4 * r + 2], y1 = rects[4 * r + 3];
    const bool ok = x0 >= 0 && x0 <= x1 && x1 < W && y0 >= 0 && y0 <= y1 && y1 < H;
    uint32_t h = 0;
    if (ok) {
        const size_t rowA = (size_t)y1 * W;               // row y1
        const size_t rowB = (size_t)(y0 - 1) * W;          // row y0-1 (used only when y0 > 0)
        h = ih[(rowA + x1) * B + b];
        if (x0 > 0) h -= ih[(rowA + x0 - 1) * B + b];
        if (y0 > 0) {
            h -= ih[(rowB + x1) * B + b];
            if (x0 > 0) h += ih[(rowB + x0 - 1) * B + b];
        }
    } else if (b == 0 && bad) {
        atomicAdd(bad, 1u);
    }
    hists[t] = h;
}

// ---------------------------------------------------------------------------
// host-side launch helpers
// ---------------------------------------------------------------------------
ScratchLayout scratch_layout(const Geom& g)
{
    ScratchLayout s;
    s.rowc = 0;
    s.colc = s.rowc + (size_t)g.H * g.nTX * g.B;
    s.corner = s.colc + (size_t)g.nTY * g.W * g.B;
    s.words = s.corner + (size_t)g.nTY * g.nTX * g.B;
    return s;
}

static int bins_per_lane(int B) { return B <= 64 ? 1 : (B <= 128 ? 2 : 4); }

Geom make_geom(int32_t H, int32_t W, int32_t B, const TileChoice& t)
{
    Geom g;
    g.H = H; g.W = W; g.B = B;
    g.TX = t.TX; g.TY = t.TY;
    g.nTX = (W + t.TX - 1) / t.TX;
    g.nTY = (H + t.TY - 1) / t.TY;
    g.BPL = bins_per_lane(B);
    g.L = (B + g.BPL - 1) / g.BPL;
    g.S = kWave / g.L;
    g.nJG = (g.nTX + g.S - 1) / g.S;
    return g;
}

bool tile_supported(int32_t B, const TileChoice& t)
{
    const int bpl = bins_per_lane(B);
    if (t.TY < 1 || t.TY > 65535) return false;
    if (bpl == 4) return t.TX == 32;
    return t.TX == 32 || t.TX == 64;
}

TileChoice default_tile(int32_t H, int32_t W, int32_t B)
{
    TileChoice t;
    t.TX = bins_per_lane(B) == 4 ? 32 : 64;
    t.nontemporal = false;
    // Tallest tile (fewest carries) that still gives enough independent waves.
    const Geom g0 = make_geom(H, W, B, TileChoice{t.TX, 1, false});
    int TY = 256;
    while (TY > 16 && (int64_t)((H + TY - 1) / TY) * g0.nJG < 2048) TY /= 2;
    t.TY = TY;
    return t;
}

using TileFn = void (*)(const uint8_t*, uint32_t*, const uint32_t*, const uint32_t*,
                        const uint32_t*, Geom, int32_t, int32_t);

template <int BPL, int TX, bool NT, bool GUARD>
static TileFn pick_b(int B)
{
    if constexpr (BPL == 1) {
        if (B == 16) return tile_kernel<1, TX, 16, NT, GUARD>;
        if (B == 32) return tile_kernel<1, TX, 32, NT, GUARD>;
        if (B == 64) return tile_kernel<1, TX, 64, NT, GUARD>;
        return tile_kernel<1, TX, 0, NT, GUARD>;
    } else if constexpr (BPL == 2) {
        if (B == 128) return tile_kernel<2, TX, 128, NT, GUARD>;
        return tile_kernel<2, TX, 0, NT, GUARD>;
    } else {
        if (B == 256) return tile_kernel<4, TX, 256, NT, GUARD>;
        return tile_kernel<4, TX, 0, NT, GUARD>;
    }
}

template <bool NT, bool GUARD>
static TileFn pick_tile(const Geom& g)
{
    switch (g.BPL) {
    case 1: return g.TX == 32 ? pick_b<1, 32, NT, GUARD>(g.B) : pick_b<1, 64, NT, GUARD>(g.B);
    case 2: return g.TX == 32 ? pick_b<2, 32, NT, GUARD>(g.B) : pick_b<2, 64, NT, GUARD>(g.B);
    default: return pick_b<4, 32, NT, GUARD>(g.B);
    }
}

static TileFn pick_tile(const Geom& g, bool nt, bool guard)
{
    if (nt) return guard ? pick_tile<true, true>(g) : pick_tile<true, false>(g);
    return guard ? pick_tile<false, true>(g) : pick_tile<false, false>(g);
}

// Column groups [0, n) whose active segments are all full and aligned run the
// unguarded kernel; the rest run the guarded one.
int32_t interior_groups(const Geom& g, const uint8_t* frame, const uint32_t* out)
{
    const bool aligned = ((reinterpret_cast<uintptr_t>(frame) & 15) == 0) && (g.W % 16 == 0) &&
                         (g.B % g.BPL == 0) &&
                         ((reinterpret_cast<uintptr_t>(out) & (4 * g.BPL - 1)) == 0);
    if (!aligned) return 0;
    const int32_t full_tiles = g.W / g.TX;
    if (full_tiles == g.nTX) return g.nJG;
    return full_tiles / g.S;
}

static void launch_tiles(const uint8_t* frame, uint32_t* out, const uint32_t* rowc,
                         const uint32_t* colc, const uint32_t* corner, const Geom& g,
                         bool nt, hipStream_t stream)
{
    const int32_t n_int = interior_groups(g, frame, out);
    const int32_t parts[2][2] = {{0, n_int}, {n_int, g.nJG - n_int}};
    for (int p = 0; p < 2; ++p) {
        const int32_t begin = parts[p][0], count = parts[p][1];
        if (count <= 0) continue;
        const int64_t items = (int64_t)g.nTY * count;
        const unsigned blocks = (unsigned)((items + kWavesPerBlock - 1) / kWavesPerBlock);
        TileFn fn = pick_tile(g, nt, p == 1);
        hipLaunchKernelGGL(fn, dim3(blocks), dim3(kWave * kWavesPerBlock), 0, stream,
                           frame, out, rowc, colc, corner, g, begin, count);
    }
}

hipError_t launch_phase(Phase ph, const uint8_t* frame, uint32_t* out, uint32_t* scratch,
                        const Geom& g, bool nontemporal, hipStream_t stream)
{
    const ScratchLayout sl = scratch_layout(g);
    uint32_t* rowc = scratch + sl.rowc;
    uint32_t* colc = scratch + sl.colc;
    uint32_t* corner = scratch + sl.corner;
    switch (ph) {
    case Phase::kAgg: {
        const unsigned ntiles = (unsigned)g.nTX * (unsigned)g.nTY;
        if (g.TX == 32)
            hipLaunchKernelGGL(agg_kernel<32>, dim3(ntiles), dim3(kAggThreads), 0, stream, frame, g, rowc, colc, corner);
        else
            hipLaunchKernelGGL(agg_kernel<64>, dim3(ntiles), dim3(kAggThreads), 0, stream, frame, g, rowc, colc, corner);
        break;
    }
    case Phase::kScan: {
        const int64_t na = (int64_t)g.H * g.B + (int64_t)g.W * g.B + (int64_t)g.nTX * g.B;
        hipLaunchKernelGGL(scan_a_kernel, dim3((unsigned)((na + kScanThreads - 1) / kScanThreads)),
                           dim3(kScanThreads), 0, stream, g, rowc, colc, corner);
        const int64_t nb = (int64_t)g.nTY * g.B;
        hipLaunchKernelGGL(scan_b_kernel, dim3((unsigned)((nb + kScanThreads - 1) / kScanThreads)),
                           dim3(kScanThreads), 0, stream, g, corner);
        break;
    }
    case Phase::kTile:
        launch_tiles(frame, out, rowc, colc, corner, g, nontemporal, stream);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_query(const uint32_t* ih, int32_t H, int32_t W, int32_t B,
                        const int32_t* rects, int64_t n, uint32_t* hists,
                        uint32_t* bad_count, hipStream_t stream)
{
    if (n == 0) return hipSuccess;
    const int64_t nt = n * B;
    hipLaunchKernelGGL(query_kernel, dim3((unsigned)((nt + kQueryThreads - 1) / kQueryThreads)),
                       dim3(kQueryThreads), 0, stream, ih, H, W, B, rects, n, hists, bad_count);
    return hipGetLastError();
}

}  // namespace ih
