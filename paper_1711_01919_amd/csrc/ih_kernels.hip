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
#include "ih_internal.h"

#include <algorithm>
#include <cstring>

namespace ih {

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Every buffer the kernels touch is device (global) memory.  Pointers read
// from a device table carry no address space, and accesses through them would
// compile to flat instructions, which also count against the LDS/scalar
// counter; casting to the global address space keeps them global_*.
#define IH_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ IH_GLOBAL T* gmem(T* p)
{
    return (IH_GLOBAL T*)p;
}

// The frame and job tables of a batched launch are read-only for the whole
// launch and indexed by wave-uniform values; reading them through the
// constant address space lets them come in with scalar loads, so everything
// derived from them (sizes, loop bounds, pointers) stays wave-uniform.
#define IH_CONST __attribute__((address_space(4)))
template <class T>
__device__ __forceinline__ const IH_CONST T* cmem(const T* p)
{
    return (const IH_CONST T*)p;
}
template <class T>
__device__ __forceinline__ T cload(const T* table, int64_t idx)
{
    T v;
    __builtin_memcpy(&v, cmem(table) + idx, sizeof(T));
    return v;
}

// Index of the calling wave within its workgroup.  The value is the same on
// every lane of a wave, and saying so keeps what is derived from it (work
// item, frame, loop bounds) in scalar registers.
__device__ __forceinline__ int wave_in_block()
{
    return __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
}

// Largest job whose `begin` is <= idx (jobs sorted by begin, jobs[0].begin == 0).
// idx is uniform across the caller's wave, so the loads stay scalar.
__device__ __forceinline__ int find_job(const IH_CONST Job* jobs, int32_t njobs, int64_t idx)
{
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].begin <= idx) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

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

// Bin of a pixel value.  A frame either uses the uniform bins floor(v B / 256)
// or a table of 256 bins (non-decreasing, so each bin is one value range),
// which the count kernels stage in LDS, four entries per word.
__device__ __forceinline__ void stage_lut(const FrameArgs& f, uint32_t* lutw, int tid, int nthreads)
{
    if (f.lut)
        for (int e = tid; e < 64; e += nthreads) lutw[e] = reinterpret_cast<const IH_GLOBAL uint32_t*>(gmem(f.lut))[e];
}
__device__ __forceinline__ uint32_t bin_of(const FrameArgs& f, const uint32_t* lutw, uint32_t v, uint32_t B)
{
    return f.lut ? (lutw[v >> 2] >> (8 * (v & 3u))) & 0xFFu : (v * B) >> 8;
}

// Entries of a non-decreasing 256-entry bin table below bin b, i.e. the first
// value of bin b (binary search in nine halving steps).
__device__ __forceinline__ uint32_t lut_count_below(const IH_GLOBAL uint8_t* lut, uint32_t b)
{
    uint32_t pos = 0;
#pragma unroll 1
    for (uint32_t step = 256; step > 0; step >>= 1)
        if (pos + step <= 256 && lut[pos + step - 1] < b) pos += step;
    return pos;
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

__device__ __forceinline__ void rowcarry_body(const FrameArgs& f, int64_t y, uint32_t* lds)
{
    const Geom& g = f.g;
    const int B = g.B, TX = g.TX, bpl = g.BPL;
    const int lane = threadIdx.x % kWave;
    uint32_t run[4] = {0u, 0u, 0u, 0u};
    const IH_GLOBAL uint8_t* prow = gmem(f.frame) + y * g.W;
    // rowc is segment-major, [j][y][b]: a tile wave's rows are contiguous
    IH_GLOBAL uint32_t* out = gmem(f.rowc) + y * B;
    const size_t seg_stride = (size_t)g.H * B;
    // 16-byte chunks never straddle a segment (TX is a multiple of 16)
    const bool vec = ((reinterpret_cast<uintptr_t>(prow) & 15) == 0);
    // the bin table sits after the counters of the largest segment chunk
    uint32_t* lutw = lds + (((kSegChunk < g.nTX ? kSegChunk : g.nTX) * B + 3) / 4);
    stage_lut(f, lutw, lane, kRowThreads);      // visible after the first barrier below
    for (int j0 = 0; j0 < g.nTX; j0 += kSegChunk) {
        const int ns = min(kSegChunk, g.nTX - j0);
        for (int w = lane; w < (ns * B + 3) / 4; w += kRowThreads) lds[w] = 0u;
        wave_sync();
        const int x0 = j0 * TX;
        const int npx = min(ns * TX, g.W - x0);
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
                const uint32_t seg = (uint32_t)((p / TX) * B);
                const uint32_t words[4] = {w[u].x, w[u].y, w[u].z, w[u].w};
#pragma unroll
                for (int k = 0; k < 16; ++k) {
                    if (p + k < npx) {
                        const uint32_t v = (words[k / 4] >> (8 * (k % 4))) & 0xFFu;
                        lds_inc8(lds, seg + bin_of(f, lutw, v, (uint32_t)B));
                    }
                }
            }
        }
        wave_sync();
        for (int s = 0; s < ns; ++s) {
            IH_GLOBAL uint32_t* o = out + (size_t)(j0 + s) * seg_stride;
            for (int t = 0; t < bpl; ++t) {
                const int b = lane * bpl + t;
                if (b < B) {
                    o[b] = run[t];
                    run[t] += lds_get8(lds, (uint32_t)(s * B + b));
                }
            }
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
// (16-bit LDS counters, <= TY pixels each), written to colc[i][x][b], and the
// tile's total per bin, written to corner[i][j][b].

// Two 16-bit counters per LDS word: column counts are <= TY <= 65535, so a
// carry never crosses halves.
__device__ __forceinline__ void lds_inc16(uint32_t* h, uint32_t e)
{
    atomicAdd(&h[e >> 1], 1u << ((e & 1u) << 4));
}
__device__ __forceinline__ uint32_t lds_get16(const uint32_t* h, uint32_t e)
{
    return (h[e >> 1] >> ((e & 1u) << 4)) & 0xFFFFu;
}

template <int TX>
__device__ __forceinline__ void agg_body(const FrameArgs& f, int64_t tile, uint32_t* colh, uint32_t* lutw)
{
    constexpr int kRowsPerPass = kAggThreads / TX;
    const Geom& g = f.g;
    const int B = g.B;
    const int i = (int)(tile / g.nTX);
    const int j = (int)(tile - (int64_t)i * g.nTX);
    const int x0 = j * TX, y0 = i * g.TY;
    const int tw = min(TX, g.W - x0);
    const int th = min(g.TY, g.H - y0);
    const int tid = threadIdx.x;
    const int tr = tid / TX, tx = tid % TX;

    for (int e = tid; e < (TX * B + 1) / 2; e += kAggThreads) colh[e] = 0;
    stage_lut(f, lutw, tid, kAggThreads);
    __syncthreads();
    if (tx < tw) {
        const IH_GLOBAL uint8_t* p = gmem(f.frame) + (size_t)y0 * g.W + x0 + tx;
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
                    lds_inc16(colh, (uint32_t)(tx * B) + bin_of(f, lutw, v[u], (uint32_t)B));
        }
    }
    __syncthreads();
    for (int e = tid; e < tw * B; e += kAggThreads)
        gmem(f.colc)[((size_t)i * g.W + x0) * B + e] = lds_get16(colh, (uint32_t)e);
    for (int b = tid; b < B; b += kAggThreads) {
        uint32_t s = 0;
        for (int x = 0; x < tw; ++x) s += lds_get16(colh, (uint32_t)(x * B + b));
        gmem(f.corner)[((size_t)i * g.nTX + j) * B + b] = s;
    }
}

// Phase 1 of a single frame in one launch: blocks [0, row_blocks) hold four
// row-carry waves each (rows 4 b .. 4 b + 3), the other blocks one tile of
// column counts each; both kinds run side by side and use the dynamic LDS
// buffer by role.  The batched form does the same per frame: a job's jg_begin
// holds its frame's row-block count, followed by the frame's tile blocks.
constexpr int kRowsPerCountBlock = kAggThreads / kWave;

__host__ __device__ inline size_t agg_lds_bytes(int TX, int B)
{
    return ((size_t)TX * B + 1) / 2 * 4 + 256;
}

template <int TX>
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
    uint32_t* colh = lds;
    agg_body<TX>(f, (int64_t)blockIdx.x - row_blocks, colh, colh + ((size_t)TX * f.g.B + 1) / 2);
}

template <int TX>
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
    uint32_t* colh = lds;
    agg_body<TX>(f, local - jb.jg_begin, colh, colh + ((size_t)TX * f.g.B + 1) / 2);
}

// ---------------------------------------------------------------------------
// Phase 2: exclusive scans of the per-tile counts
// ---------------------------------------------------------------------------
// Exclusive scan of p[0], p[stride], ... p[(len-1)*stride] in place, starting
// from `run`.  Loads of a chunk are issued before its stores so that many are
// in flight at once.
__device__ __forceinline__ void scan_seq(IH_GLOBAL uint32_t* p, int64_t stride, int len, uint32_t run)
{
    constexpr int C = 16;
    int k = 0;
    for (; k + C <= len; k += C) {
        uint32_t v[C];
#pragma unroll
        for (int u = 0; u < C; ++u) v[u] = p[(k + u) * stride];
#pragma unroll
        for (int u = 0; u < C; ++u) { p[(k + u) * stride] = run; run += v[u]; }
    }
    for (; k < len; ++k) {
        const uint32_t v = p[k * stride];
        p[k * stride] = run;
        run += v;
    }
}

__device__ __forceinline__ uint32_t sum_seq(const IH_GLOBAL uint32_t* p, int64_t stride, int len)
{
    constexpr int C = 16;
    uint32_t s = 0;
    int k = 0;
    for (; k + C <= len; k += C) {
        uint32_t v[C];
#pragma unroll
        for (int u = 0; u < C; ++u) v[u] = p[(k + u) * stride];
#pragma unroll
        for (int u = 0; u < C; ++u) s += v[u];
    }
    for (; k < len; ++k) s += p[k * stride];
    return s;
}

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
template <int P>
__device__ __forceinline__ void scan_seq_parts(IH_GLOBAL uint32_t* p, int64_t stride, int len, bool active,
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
                p[(int64_t)(lo + u) * stride] = run;
                run += v[u];
            }
    } else {
        scan_seq(p + (int64_t)lo * stride, stride, hi - lo, run);
    }
}

// Column counts across tile bands and tile totals across bands --
// independent sequences of length nTY; the frame's blocks take the column
// sequences first, then the tile-total ones, so that each block holds one
// kind.  `blk` is the block's index within the frame's scan blocks.
template <int P>
__device__ __forceinline__ void scan_a_body(const FrameArgs& f, int64_t blk, uint32_t* sums)
{
    const Geom& g = f.g;
    const int64_t B = g.B;
    constexpr int per = kScanThreads / P;
    const int64_t ncol = (int64_t)g.W * B, ntot = (int64_t)g.nTX * B;
    const int64_t col_blocks = (ncol + per - 1) / per;
    const bool is_col = blk < col_blocks;                    // uniform over the block
    const int64_t t = (is_col ? blk : blk - col_blocks) * per + (int)threadIdx.x % per;
    IH_GLOBAL uint32_t* base = is_col ? gmem(f.colc) : gmem(f.corner);
    const int64_t stride = (is_col ? (int64_t)g.W : (int64_t)g.nTX) * B;
    scan_seq_parts<P>(base + t, stride, g.nTY, t < (is_col ? ncol : ntot), sums);
}

// Band-scanned tile totals across tile columns (sequences of length nTX):
// corner[i][j][b] becomes the count of pixels above and to the left of tile
// (i, j).
template <int P>
__device__ __forceinline__ void scan_b_body(const FrameArgs& f, int64_t blk, uint32_t* sums)
{
    const Geom& g = f.g;
    const int64_t B = g.B;
    constexpr int per = kScanThreads / P;
    const int64_t t = blk * per + (int)threadIdx.x % per;
    const bool active = t < (int64_t)g.nTY * B;
    const int64_t i = t / B, b = t - i * B;
    scan_seq_parts<P>(gmem(f.corner) + i * g.nTX * B + b, B, g.nTX, active, sums);
}

template <int P>
__global__ __launch_bounds__(kScanThreads)
void scan_a_kernel(FrameArgs f)
{
    __shared__ uint32_t sums[P == 1 ? 1 : kScanThreads];
    scan_a_body<P>(f, blockIdx.x, sums);
}

template <int P>
__global__ __launch_bounds__(kScanThreads)
void scan_b_kernel(FrameArgs f)
{
    __shared__ uint32_t sums[P == 1 ? 1 : kScanThreads];
    scan_b_body<P>(f, blockIdx.x, sums);
}

template <int P>
__global__ __launch_bounds__(kScanThreads)
void scan_a_batch_kernel(const FrameArgs* __restrict__ frames, const Job* __restrict__ jobs, int32_t njobs)
{
    __shared__ uint32_t sums[P == 1 ? 1 : kScanThreads];
    const Job jb = cload(jobs, find_job(cmem(jobs), njobs, blockIdx.x));
    const FrameArgs f = cload(frames, jb.frame);
    scan_a_body<P>(f, (int64_t)blockIdx.x - jb.begin, sums);
}

template <int P>
__global__ __launch_bounds__(kScanThreads)
void scan_b_batch_kernel(const FrameArgs* __restrict__ frames, const Job* __restrict__ jobs, int32_t njobs)
{
    __shared__ uint32_t sums[P == 1 ? 1 : kScanThreads];
    const Job jb = cload(jobs, find_job(cmem(jobs), njobs, blockIdx.x));
    const FrameArgs f = cload(frames, jb.frame);
    scan_b_body<P>(f, (int64_t)blockIdx.x - jb.begin, sums);
}

// ---------------------------------------------------------------------------
// Phase 3: the tile pass (hot loop)
// ---------------------------------------------------------------------------
template <int BPL, bool NT>
__device__ __forceinline__ void store_bins(IH_GLOBAL uint32_t* p, const uint32_t (&v)[BPL])
{
    if constexpr (BPL == 1) {
        if constexpr (NT) __builtin_nontemporal_store(v[0], p);
        else *p = v[0];
    } else if constexpr (BPL == 2) {
        u32x2 w = {v[0], v[1]};
        if constexpr (NT) __builtin_nontemporal_store(w, reinterpret_cast<IH_GLOBAL u32x2*>(p));
        else *reinterpret_cast<IH_GLOBAL u32x2*>(p) = w;
    } else {
        u32x4 w = {v[0], v[1], v[2], v[3]};
        if constexpr (NT) __builtin_nontemporal_store(w, reinterpret_cast<IH_GLOBAL u32x4*>(p));
        else *reinterpret_cast<IH_GLOBAL u32x4*>(p) = w;
    }
}

// Pixels of row y of a tile segment (TX bytes, packed four per dword).
template <int TX, bool GUARD, bool UNIFORM>
__device__ __forceinline__ void load_px(const FrameArgs& f, int y, int x0, int ncols, uint32_t (&px)[TX / 4])
{
    const IH_GLOBAL uint8_t* prow = gmem(f.frame) + (size_t)y * f.g.W + x0;
    if constexpr (!GUARD && UNIFORM) {
        // One segment per wave: every lane reads the same pixels, so read
        // them once with scalar loads (their wait never involves the stores).
        const IH_CONST uint8_t* crow = cmem(f.frame) + (size_t)y * f.g.W + x0;
#pragma unroll
        for (int q = 0; q < TX / 16; ++q) {
            const u32x4 w = *reinterpret_cast<const IH_CONST u32x4*>(crow + 16 * q);
            px[4 * q + 0] = w.x; px[4 * q + 1] = w.y;
            px[4 * q + 2] = w.z; px[4 * q + 3] = w.w;
        }
    } else if constexpr (!GUARD) {
#pragma unroll
        for (int q = 0; q < TX / 16; ++q) {
            const u32x4 w = *reinterpret_cast<const IH_GLOBAL u32x4*>(prow + 16 * q);
            px[4 * q + 0] = w.x; px[4 * q + 1] = w.y;
            px[4 * q + 2] = w.z; px[4 * q + 3] = w.w;
        }
    } else {
#pragma unroll
        for (int q = 0; q < TX / 4; ++q) px[q] = 0u;
#pragma unroll
        for (int k = 0; k < TX; ++k)
            if (k < ncols) px[k / 4] |= (uint32_t)prow[k] << (8 * (k % 4));
    }
}

// Left carries of CH consecutive rows y, y+1, ... of segment j (rows past the
// band clamped to its last row): CH x B contiguous uint32 in the segment-major
// rowc, read as one burst.
template <int BPL, int CH>
__device__ __forceinline__ void load_carries(const FrameArgs& f, int y, int y_last, int j, int b0, int B,
                                             const bool (&bvalid)[BPL], uint32_t (&cb)[CH][BPL])
{
    const IH_GLOBAL uint32_t* rp = gmem(f.rowc) + (size_t)j * f.g.H * B + b0;
#pragma unroll
    for (int q = 0; q < CH; ++q) {
        const IH_GLOBAL uint32_t* r = rp + (size_t)min(y + q, y_last) * B;
#pragma unroll
        for (int t = 0; t < BPL; ++t) cb[q][t] = bvalid[t] ? r[t] : 0u;
    }
}

// One wave, one work item: tile band i (TY rows) x column group jg (S adjacent
// tile segments).  GUARD=false requires all S segments of the group to exist
// and be TX columns wide, the frame and W 16-byte aligned, B % BPL == 0 and
// out aligned to 4*BPL bytes; the host routes everything else to GUARD=true.
template <int BPL, int TX, int BC, bool NT, bool GUARD, bool TABLE>
__device__ __forceinline__ void tile_body(const FrameArgs& f, int i, int jg, int lane)
{
    static_assert(TX % 16 == 0, "pixel rows are loaded 16 bytes at a time");
    constexpr int LC = BC ? (BC + BPL - 1) / BPL : 1;
    constexpr bool UNIFORM = BC != 0 && kWave / LC == 1;      // one segment per wave
    const Geom& g = f.g;
    const int B = BC ? BC : g.B;
    const int L = BC ? LC : g.L;
    const int S = BC ? kWave / LC : g.S;

    const int s = lane / L;
    const int b0 = (lane - s * L) * BPL;
    const int j = jg * S + s;
    if (!((s < S) && (j < g.nTX) && (b0 < B))) return;      // idle lane
    const int x0 = j * TX;
    const int ncols = GUARD ? min(TX, g.W - x0) : TX;
    const int y0 = i * g.TY;
    const int y1 = min(g.H, y0 + g.TY);

    // Bin b holds the values v in [lo, lo + width).  Uniform bins: v with
    // ceil(256 b / B) <= v < ceil(256 (b+1) / B), which is floor(v B / 256)
    // == b.  A bin table: lo = #{v : lut[v] < b}, lo + width = #{v : lut[v]
    // <= b} (the table never decreases).  A lane tests v - lo < width
    // (unsigned); an empty bin has width 0.
    uint32_t lo[BPL], wd[BPL];
    bool bvalid[BPL];
#pragma unroll
    for (int t = 0; t < BPL; ++t) bvalid[t] = GUARD ? b0 + t < B : true;
    if constexpr (TABLE) {
        const IH_GLOBAL uint8_t* lt = gmem(f.lut);
#pragma unroll
        for (int t = 0; t < BPL; ++t) {
            const uint32_t l = lut_count_below(lt, (uint32_t)(b0 + t));
            const uint32_t h = lut_count_below(lt, (uint32_t)(b0 + t + 1));
            lo[t] = bvalid[t] ? l : 0u;
            wd[t] = bvalid[t] ? h - l : 0u;
        }
    } else {
#pragma unroll
        for (int t = 0; t < BPL; ++t) {
            const int b = b0 + t;
            const uint32_t l = (uint32_t)(256 * b + B - 1) / (uint32_t)B;
            const uint32_t h = (uint32_t)(256 * (b + 1) + B - 1) / (uint32_t)B;
            lo[t] = bvalid[t] ? l : 0u;
            wd[t] = bvalid[t] ? h - l : 0u;
        }
    }

    // Column state: corner + running sum of the top carries along the segment.
    uint32_t V[BPL][TX];
    {
        uint32_t acc[BPL];
        const IH_GLOBAL uint32_t* cp = gmem(f.corner) + ((size_t)i * g.nTX + j) * B + b0;
        const IH_GLOBAL uint32_t* tp = gmem(f.colc) + ((size_t)i * g.W + x0) * B + b0;
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
                        ((reinterpret_cast<uintptr_t>(f.out) & (4 * BPL - 1)) == 0);

    auto row_pass = [&](int y, const uint32_t (&px)[TX / 4], const uint32_t (&c0)[BPL]) {
        IH_GLOBAL uint32_t* orow = gmem(f.out) + ((size_t)y * g.W + x0) * B + b0;
        uint32_t cnt[BPL];
#pragma unroll
        for (int t = 0; t < BPL; ++t) cnt[t] = c0[t];
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
                store_bins<BPL, NT>(orow + (size_t)k * B, o);
            } else if (k < ncols) {
                if (vec_ok) {
                    store_bins<BPL, NT>(orow + (size_t)k * B, o);
                } else {
#pragma unroll
                    for (int t = 0; t < BPL; ++t)
                        if (bvalid[t]) orow[(size_t)k * B + t] = o[t];
                }
            }
        }
    };
    // Reads beside the write stream cost DRAM time per read burst, so the
    // left carries come CH rows at a time (one contiguous burst from the
    // segment-major rowc), loaded a chunk ahead into nb and handed to cb,
    // which shifts down one row per row.  Pixels of row y+1 are loaded before
    // the stores of row y (two register sets alternate): loads and stores
    // share one in-order completion counter on this architecture, so a load
    // issued after a row's stores could only be waited for behind them.
    // Rows past the band are clamped, so every wave runs the same control flow.
    // Several segments per wave (B < 64, compile-time B, whole segments):
    // the pixels of a chunk of rows for all of the wave's segments come in
    // one wave-wide load too, and each lane fetches its segment's bytes of a
    // row from the lane holding them (ds_bpermute).  Piece p (16 bytes) of a
    // chunk is row r, 16-byte column c, segment s with p = (r * PPR + c) * SC
    // + s, held by lane p.
    constexpr int SC = kWave / LC;
    constexpr int PPR = TX / 16;
    constexpr bool CHUNK_PX = !GUARD && !UNIFORM && BC != 0 && SC * PPR <= kWave;
    constexpr int CH = CHUNK_PX ? (8 / BPL < kWave / (SC * PPR) ? 8 / BPL : kWave / (SC * PPR)) : 8 / BPL;
    uint32_t cb[CH][BPL], nb[CH][BPL];
    if constexpr (CHUNK_PX) {
        static_assert(CH * SC * PPR <= kWave, "a pixel chunk must fit one wave-wide load");
        auto load_chunk_px = [&](int yc, u32x4& dst) {
            const int p = lane < CH * SC * PPR ? lane : 0;
            const int ps = p % SC, pc_ = (p / SC) % PPR, pr = p / (SC * PPR);
            const int row = min(yc + pr, y1 - 1);
            const int px0 = (jg * SC + ps) * TX + 16 * pc_;
            dst = *reinterpret_cast<const IH_GLOBAL u32x4*>(gmem(f.frame) + (size_t)row * g.W + px0);
        };
        u32x4 pc, pn;
        load_carries<BPL, CH>(f, y0, y1 - 1, j, b0, B, bvalid, cb);
        load_chunk_px(y0, pc);
        __builtin_amdgcn_s_waitcnt(0);
        for (int yc = y0; yc < y1; yc += CH) {
            const bool more = yc + CH < y1;
            if (more) {
                load_carries<BPL, CH>(f, yc + CH, y1 - 1, j, b0, B, bvalid, nb);
                load_chunk_px(yc + CH, pn);
            }
#pragma unroll 1
            for (int r = 0; r < CH; ++r) {
                const int y = yc + r;
                uint32_t px[TX / 4];
#pragma unroll
                for (int q = 0; q < TX / 4; ++q) {
                    const int src = (r * PPR + q / 4) * SC + s;
                    px[q] = (uint32_t)__builtin_amdgcn_ds_bpermute(src * 4, (int)pc[q % 4]);
                }
                if (y < y1) row_pass(y, px, cb[0]);
#pragma unroll
                for (int q = 0; q + 1 < CH; ++q)
#pragma unroll
                    for (int t = 0; t < BPL; ++t) cb[q][t] = cb[q + 1][t];
            }
            if (more) {
#pragma unroll
                for (int q = 0; q < CH; ++q)
#pragma unroll
                    for (int t = 0; t < BPL; ++t) cb[q][t] = nb[q][t];
                pc = pn;
            }
        }
        return;
    }
    uint32_t pxa[TX / 4], pxb[TX / 4];
    load_carries<BPL, CH>(f, y0, y1 - 1, j, b0, B, bvalid, cb);
    load_px<TX, GUARD, UNIFORM>(f, y0, x0, ncols, pxa);
    // Drain everything once per work item, so that inside the loop the
    // compiler's counter bookkeeping sees only the in-loop prefetches.
    __builtin_amdgcn_s_waitcnt(0);
    for (int yc = y0; yc < y1; yc += CH) {
        if (yc + CH < y1) load_carries<BPL, CH>(f, yc + CH, y1 - 1, j, b0, B, bvalid, nb);
#pragma unroll 1
        for (int r = 0; r < CH; r += 2) {
            const int y = yc + r;
            load_px<TX, GUARD, UNIFORM>(f, min(y + 1, y1 - 1), x0, ncols, pxb);
            __builtin_amdgcn_sched_barrier(0);        // keep the prefetch ahead of the stores
            if (y < y1) row_pass(y, pxa, cb[0]);
#pragma unroll
            for (int q = 0; q + 1 < CH; ++q)
#pragma unroll
                for (int t = 0; t < BPL; ++t) cb[q][t] = cb[q + 1][t];
            load_px<TX, GUARD, UNIFORM>(f, min(y + 2, y1 - 1), x0, ncols, pxa);
            __builtin_amdgcn_sched_barrier(0);
            if (y + 1 < y1) row_pass(y + 1, pxb, cb[0]);
#pragma unroll
            for (int q = 0; q + 1 < CH; ++q)
#pragma unroll
                for (int t = 0; t < BPL; ++t) cb[q][t] = cb[q + 1][t];
        }
#pragma unroll
        for (int q = 0; q < CH; ++q)
#pragma unroll
            for (int t = 0; t < BPL; ++t) cb[q][t] = nb[q][t];
    }
}

template <int BPL, int TX, int BC, bool NT, bool GUARD, bool TABLE>
__global__ __launch_bounds__(kWave * kWavesPerBlock)
void tile_kernel(FrameArgs f, int32_t jg_begin, int32_t jg_count)
{
    const int64_t item = (int64_t)blockIdx.x * kWavesPerBlock + wave_in_block();
    if (item >= (int64_t)f.g.nTY * jg_count) return;      // whole wave leaves together
    const int i = (int)(item / jg_count);
    const int jg = jg_begin + (int)(item - (int64_t)i * jg_count);
    tile_body<BPL, TX, BC, NT, GUARD, TABLE>(f, i, jg, threadIdx.x % kWave);
}

// Persistent form: each wave strides over the work items of all jobs.
template <int BPL, int TX, int BC, bool NT, bool GUARD, bool TABLE>
__global__ __launch_bounds__(kWave * kWavesPerBlock)
void tile_batch_kernel(const FrameArgs* __restrict__ frames, const Job* __restrict__ jobs,
                       int32_t njobs, int64_t nitems)
{
    const int64_t stride = (int64_t)gridDim.x * kWavesPerBlock;
    for (int64_t item = (int64_t)blockIdx.x * kWavesPerBlock + wave_in_block(); item < nitems;
         item += stride) {
        const Job jb = cload(jobs, find_job(cmem(jobs), njobs, item));
        const int64_t local = item - jb.begin;
        const int i = (int)(local / jb.jg_count);
        const int jg = jb.jg_begin + (int)(local - (int64_t)i * jb.jg_count);
        const FrameArgs f = cload(frames, jb.frame);
        tile_body<BPL, TX, BC, NT, GUARD, TABLE>(f, i, jg, threadIdx.x % kWave);
    }
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
// Entry (x, y, b) at (b * H + y) * W + x.  One wave per (tile band, 64-column
// segment, group of BG <= 16 bins, BG a power of two dividing B); lane l owns column
// x0 + l.  For a row and a bin the in-row prefix across the segment is a
// ballot of the lanes whose pixel falls in the bin and a count of the set
// bits below each lane (mbcnt), plus the left carry of the row; the column
// accumulators V[t] start from the corner and the lane prefix of the top
// carries.  Stores are 256 contiguous bytes per bin and row.  The carry
// phases are the same as for the H x W x B layout with 64-column tiles.
__device__ __forceinline__ uint32_t wave_inclusive_sum(uint32_t v, int lane)
{
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t u = (uint32_t)__builtin_amdgcn_ds_bpermute((lane >= d ? lane - d : lane) * 4, (int)v);
        v += lane >= d ? u : 0u;
    }
    return v;
}

// Items of a frame: nTY * nTX * (B / BG), one wave each.
template <int BG>
__device__ __forceinline__ void tile_bm_body(const FrameArgs& f, int64_t item)
{
    const Geom& g = f.g;
    const int B = g.B, H = g.H, W = g.W;
    const int n_groups = B / BG;
    const int lane = threadIdx.x % kWave;
    const int grp = (int)(item % n_groups);
    const int64_t tile = item / n_groups;
    const int i = (int)(tile / g.nTX), j = (int)(tile % g.nTX);
    const int x0 = j * kWave, x = x0 + lane;
    const bool valid = x < W;
    const int y0 = i * g.TY, y1 = min(H, y0 + g.TY);
    const int b_lo = grp * BG;

    uint32_t V[BG];
    {
        const IH_GLOBAL uint32_t* cp = gmem(f.corner) + ((size_t)i * g.nTX + j) * B + b_lo;
        const IH_GLOBAL uint32_t* tp = gmem(f.colc) + ((size_t)i * W + x) * B + b_lo;
        const uint32_t corner = lane < BG ? cp[lane] : 0u;     // lane t: corner of bin b_lo + t
#pragma unroll
        for (int t = 0; t < BG; ++t) {
            const uint32_t c = valid ? tp[t] : 0u;
            V[t] = (uint32_t)__builtin_amdgcn_readlane((int)corner, t) + wave_inclusive_sum(c, lane);
        }
    }
    const IH_GLOBAL uint8_t* frame = gmem(f.frame);
    const IH_GLOBAL uint32_t* rowc = gmem(f.rowc) + (size_t)j * H * B + b_lo;
    IH_GLOBAL uint32_t* out = gmem(f.out);
    const size_t plane = (size_t)H * W;
    // Pixels (binned) and left carries come 8 rows at a time, a chunk ahead:
    // lane t holds the carry of bin b_lo + t; rows past the band are clamped.
    constexpr int CH = 8;
    uint32_t cq[CH], cc[CH], nq[CH], nc[CH];
    auto load_chunk = [&](int yc, uint32_t (&q)[CH], uint32_t (&c)[CH]) {
#pragma unroll
        for (int r = 0; r < CH; ++r) {
            const int row = min(yc + r, y1 - 1);
            const uint32_t v = valid ? frame[(size_t)row * W + x] : 0u;
            q[r] = valid ? (v * (uint32_t)B) >> 8 : 0xFFFFu;
            c[r] = lane < BG ? rowc[(size_t)row * B + lane] : 0u;
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
                IH_GLOBAL uint32_t* orow = out + (size_t)b_lo * plane + (size_t)y * W + x;
#pragma unroll
                for (int t = 0; t < BG; ++t) {
                    const bool hit = cq[r] == (uint32_t)(b_lo + t);
                    const uint64_t m = __builtin_amdgcn_ballot_w64(hit);
                    const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                    V[t] += (uint32_t)__builtin_amdgcn_readlane((int)cc[r], t) + below + (hit ? 1u : 0u);
                    if (valid) orow[(size_t)t * plane] = V[t];
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

template <int BG>
__global__ __launch_bounds__(kWave * kWavesPerBlock)
void tile_bm_kernel(FrameArgs f)
{
    const int64_t item = (int64_t)blockIdx.x * kWavesPerBlock + wave_in_block();
    if (item >= (int64_t)f.g.nTY * f.g.nTX * (f.g.B / BG)) return;     // whole wave leaves together
    tile_bm_body<BG>(f, item);
}

// Many bin-major frames with the same bin group BG: one wave per item over
// the job table (a job per frame, `begin` its first item).
template <int BG>
__global__ __launch_bounds__(kWave * kWavesPerBlock)
void tile_bm_batch_kernel(const FrameArgs* __restrict__ frames, const Job* __restrict__ jobs, int32_t njobs,
                          int64_t nitems)
{
    const int64_t item = (int64_t)blockIdx.x * kWavesPerBlock + wave_in_block();
    if (item >= nitems) return;                                        // whole wave leaves together
    const Job jb = cload(jobs, find_job(cmem(jobs), njobs, item));
    const FrameArgs f = cload(frames, jb.frame);
    tile_bm_body<BG>(f, item - jb.begin);
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
// host side: kernel table and launches (geometry and tile choice live in
// ih_geom.cpp)
// ---------------------------------------------------------------------------
// Table of compiled tile kernels: single-frame and batched entry per variant.
struct TileFns {
    const void* single;
    const void* batch;
};

template <int BPL, int TX, int BC, bool NT, bool GUARD, bool TABLE = false>
static TileFns fns_of()
{
    return TileFns{reinterpret_cast<const void*>(&tile_kernel<BPL, TX, BC, NT, GUARD, TABLE>),
                   reinterpret_cast<const void*>(&tile_batch_kernel<BPL, TX, BC, NT, GUARD, TABLE>)};
}

// Frames binned by a table: runtime B and regular stores only.
template <bool GUARD>
static TileFns pick_table(const TileVariant& v)
{
    switch (v.bpl) {
    case 1: return v.tx == 32 ? fns_of<1, 32, 0, false, GUARD, true>() : fns_of<1, 64, 0, false, GUARD, true>();
    case 2: return v.tx == 32 ? fns_of<2, 32, 0, false, GUARD, true>() : fns_of<2, 64, 0, false, GUARD, true>();
    default: return fns_of<4, 32, 0, false, GUARD, true>();
    }
}

template <int BPL, int TX, bool NT, bool GUARD>
static TileFns pick_bc(int bc)
{
    if constexpr (BPL == 1) {
        if (bc == 16) return fns_of<1, TX, 16, NT, GUARD>();
        if (bc == 32) return fns_of<1, TX, 32, NT, GUARD>();
        if (bc == 64) return fns_of<1, TX, 64, NT, GUARD>();
        return fns_of<1, TX, 0, NT, GUARD>();
    } else if constexpr (BPL == 2) {
        if (bc == 128) return fns_of<2, TX, 128, NT, GUARD>();
        return fns_of<2, TX, 0, NT, GUARD>();
    } else {
        if (bc == 256) return fns_of<4, TX, 256, NT, GUARD>();
        return fns_of<4, TX, 0, NT, GUARD>();
    }
}

template <bool NT, bool GUARD>
static TileFns pick_v(const TileVariant& v)
{
    switch (v.bpl) {
    case 1:
        if (v.tx == 128) return fns_of<1, 128, 64, NT, GUARD>();      // B == 64 only
        return v.tx == 32 ? pick_bc<1, 32, NT, GUARD>(v.bc) : pick_bc<1, 64, NT, GUARD>(v.bc);
    case 2: return v.tx == 32 ? pick_bc<2, 32, NT, GUARD>(v.bc) : pick_bc<2, 64, NT, GUARD>(v.bc);
    default: return pick_bc<4, 32, NT, GUARD>(v.bc);
    }
}

static TileFns tile_fns(const TileVariant& v)
{
    if (v.table) return v.guard ? pick_table<true>(v) : pick_table<false>(v);
    if (v.nt) return v.guard ? pick_v<true, true>(v) : pick_v<true, false>(v);
    return v.guard ? pick_v<false, true>(v) : pick_v<false, false>(v);
}


int64_t scan_a_blocks(const Geom& g)
{
    const int64_t per = scan_per_block(g.nTY);
    return ((int64_t)g.W * g.B + per - 1) / per + ((int64_t)g.nTX * g.B + per - 1) / per;
}

int64_t scan_b_blocks(const Geom& g)
{
    const int64_t per = scan_per_block(g.nTX);
    return ((int64_t)g.nTY * g.B + per - 1) / per;
}

hipError_t launch_phase(Phase ph, const FrameArgs& f, bool nontemporal, hipStream_t stream)
{
    const Geom& g = f.g;
    switch (ph) {
    case Phase::kAgg: {
        const int32_t row_blocks = count_row_blocks(g);
        const unsigned blocks = (unsigned)row_blocks + (unsigned)g.nTX * (unsigned)g.nTY;
        const size_t lds = count_lds(g);
        if (g.TX == 32)
            hipLaunchKernelGGL(count_kernel<32>, dim3(blocks), dim3(kAggThreads), (unsigned)lds, stream, f, row_blocks);
        else if (g.TX == 128)
            hipLaunchKernelGGL(count_kernel<128>, dim3(blocks), dim3(kAggThreads), (unsigned)lds, stream, f, row_blocks);
        else
            hipLaunchKernelGGL(count_kernel<64>, dim3(blocks), dim3(kAggThreads), (unsigned)lds, stream, f, row_blocks);
        break;
    }
    case Phase::kScan:
        if (scan_parts(g.nTY) == 1)
            hipLaunchKernelGGL(scan_a_kernel<1>, dim3((unsigned)scan_a_blocks(g)), dim3(kScanThreads), 0, stream, f);
        else
            hipLaunchKernelGGL(scan_a_kernel<kScanParts>, dim3((unsigned)scan_a_blocks(g)), dim3(kScanThreads), 0,
                               stream, f);
        if (scan_parts(g.nTX) == 1)
            hipLaunchKernelGGL(scan_b_kernel<1>, dim3((unsigned)scan_b_blocks(g)), dim3(kScanThreads), 0, stream, f);
        else
            hipLaunchKernelGGL(scan_b_kernel<kScanParts>, dim3((unsigned)scan_b_blocks(g)), dim3(kScanThreads), 0,
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

hipError_t launch_count_batch(int TX, const FrameArgs* frames, const Job* jobs, int32_t njobs,
                              int64_t nblocks, size_t lds_bytes, hipStream_t stream)
{
    if (nblocks <= 0) return hipSuccess;
    const dim3 grid((unsigned)nblocks), block(kAggThreads);
    if (TX == 32)
        hipLaunchKernelGGL(count_batch_kernel<32>, grid, block, (unsigned)lds_bytes, stream, frames, jobs, njobs);
    else if (TX == 128)
        hipLaunchKernelGGL(count_batch_kernel<128>, grid, block, (unsigned)lds_bytes, stream, frames, jobs, njobs);
    else
        hipLaunchKernelGGL(count_batch_kernel<64>, grid, block, (unsigned)lds_bytes, stream, frames, jobs, njobs);
    return hipGetLastError();
}

hipError_t launch_scan_a_batch(int parts, const FrameArgs* frames, const Job* jobs, int32_t njobs,
                               int64_t nblocks, hipStream_t stream)
{
    if (nblocks <= 0) return hipSuccess;
    const dim3 grid((unsigned)nblocks), block(kScanThreads);
    if (parts == 1)
        hipLaunchKernelGGL(scan_a_batch_kernel<1>, grid, block, 0, stream, frames, jobs, njobs);
    else
        hipLaunchKernelGGL(scan_a_batch_kernel<kScanParts>, grid, block, 0, stream, frames, jobs, njobs);
    return hipGetLastError();
}

hipError_t launch_scan_b_batch(int parts, const FrameArgs* frames, const Job* jobs, int32_t njobs,
                               int64_t nblocks, hipStream_t stream)
{
    if (nblocks <= 0) return hipSuccess;
    const dim3 grid((unsigned)nblocks), block(kScanThreads);
    if (parts == 1)
        hipLaunchKernelGGL(scan_b_batch_kernel<1>, grid, block, 0, stream, frames, jobs, njobs);
    else
        hipLaunchKernelGGL(scan_b_batch_kernel<kScanParts>, grid, block, 0, stream, frames, jobs, njobs);
    return hipGetLastError();
}

hipError_t launch_tile_batch(const TileVariant& v, const FrameArgs* frames, const Job* jobs,
                             int32_t njobs, int64_t nitems, int32_t grid, hipStream_t stream)
{
    if (nitems <= 0) return hipSuccess;
    const TileFns fn = tile_fns(v);
    void* args[] = {&frames, &jobs, &njobs, &nitems};
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

hipError_t launch_tile_bm(const FrameArgs& f, hipStream_t stream)
{
    const Geom& g = f.g;
    const int bg = bm_group(g.B);
    const int64_t items = (int64_t)g.nTY * g.nTX * (g.B / bg);
    const unsigned blocks = (unsigned)((items + kWavesPerBlock - 1) / kWavesPerBlock);
    const dim3 grid(blocks), block(kWave * kWavesPerBlock);
    switch (bg) {
    case 16: hipLaunchKernelGGL(tile_bm_kernel<16>, grid, block, 0, stream, f); break;
    case 8: hipLaunchKernelGGL(tile_bm_kernel<8>, grid, block, 0, stream, f); break;
    case 4: hipLaunchKernelGGL(tile_bm_kernel<4>, grid, block, 0, stream, f); break;
    case 2: hipLaunchKernelGGL(tile_bm_kernel<2>, grid, block, 0, stream, f); break;
    default: hipLaunchKernelGGL(tile_bm_kernel<1>, grid, block, 0, stream, f); break;
    }
    return hipGetLastError();
}

int64_t tile_bm_items(const Geom& g) { return (int64_t)g.nTY * g.nTX * (g.B / bm_group(g.B)); }

hipError_t launch_tile_bm_batch(int bg, const FrameArgs* frames, const Job* jobs, int32_t njobs, int64_t nitems,
                                hipStream_t stream)
{
    if (nitems <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)((nitems + kWavesPerBlock - 1) / kWavesPerBlock);
    const dim3 grid(blocks), block(kWave * kWavesPerBlock);
    switch (bg) {
    case 16: hipLaunchKernelGGL(tile_bm_batch_kernel<16>, grid, block, 0, stream, frames, jobs, njobs, nitems); break;
    case 8: hipLaunchKernelGGL(tile_bm_batch_kernel<8>, grid, block, 0, stream, frames, jobs, njobs, nitems); break;
    case 4: hipLaunchKernelGGL(tile_bm_batch_kernel<4>, grid, block, 0, stream, frames, jobs, njobs, nitems); break;
    case 2: hipLaunchKernelGGL(tile_bm_batch_kernel<2>, grid, block, 0, stream, frames, jobs, njobs, nitems); break;
    default: hipLaunchKernelGGL(tile_bm_batch_kernel<1>, grid, block, 0, stream, frames, jobs, njobs, nitems); break;
    }
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
