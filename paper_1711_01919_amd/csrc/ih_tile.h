// The tile pass (hot loop) of the integral histogram: binning fused with
// the in-lane row scan, VGPR column accumulators and the output stores, as a
// device function with single-frame and persistent batched kernels around it,
// and the tables that name each compiled variant.  Each tile_*.hip source
// instantiates one part of the variants, so they compile in parallel.
#pragma once

#include "ih_device.h"
#include "ih_tile_fns.h"

namespace ih {

// s_waitcnt operand that waits for the LDS/scalar-memory counter to reach zero
// and leaves the vector-memory and export counters unconstrained (gfx9
// encoding: vmcnt in bits 3:0 and 15:14, expcnt in 6:4, lgkmcnt in 11:8).
constexpr int kWaitLgkm0 = 0xC07F;

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
        // A whole segment whose row starts on a four-byte boundary: dword
        // loads.  Otherwise (the frame's right edge, or rows that are not
        // word-aligned) byte loads of the pixels inside the frame.
        if (ncols == TX && (reinterpret_cast<uintptr_t>(prow) & 3) == 0) {
#pragma unroll
            for (int q = 0; q < TX / 4; ++q) px[q] = reinterpret_cast<const IH_GLOBAL uint32_t*>(prow)[q];
        } else {
#pragma unroll
            for (int q = 0; q < TX / 4; ++q) px[q] = 0u;
#pragma unroll
            for (int k = 0; k < TX; ++k)
                if (k < ncols) px[k / 4] |= (uint32_t)prow[k] << (8 * (k % 4));
        }
    }
}

// Left carries of CH consecutive rows y, y+1, ... of segment j (rows past the
// band clamped to its last row): CH x B contiguous entries (uint16, or uint32
// for frames wider than 65536) in the segment-major rowc, read as one burst.
template <int BPL, int CH>
__device__ __forceinline__ void load_carries(const FrameArgs& f, int y, int y_last, int j, int b0, int B,
                                             const bool (&bvalid)[BPL], uint32_t (&cb)[CH][BPL])
{
    const size_t base = (size_t)j * f.g.H * B + b0;
    if (f.g.RC16) {
        const IH_GLOBAL uint16_t* rp = gmem(reinterpret_cast<const uint16_t*>(f.rowc)) + base;
#pragma unroll
        for (int q = 0; q < CH; ++q) {
            const IH_GLOBAL uint16_t* r = rp + (size_t)min(y + q, y_last) * B;
#pragma unroll
            for (int t = 0; t < BPL; ++t) cb[q][t] = bvalid[t] ? (uint32_t)r[t] : 0u;
        }
    } else {
        const IH_GLOBAL uint32_t* rp = gmem(f.rowc) + base;
#pragma unroll
        for (int q = 0; q < CH; ++q) {
            const IH_GLOBAL uint32_t* r = rp + (size_t)min(y + q, y_last) * B;
#pragma unroll
            for (int t = 0; t < BPL; ++t) cb[q][t] = bvalid[t] ? r[t] : 0u;
        }
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

    // A table that decreases somewhere (a bin need not be one range of
    // values): every pixel of a row is binned through the table, staged in
    // this wave's LDS, before the lanes test their bins (q == b).
    __shared__ uint32_t lut_lds[kWavesPerBlock][kWave];
    uint32_t* lutw = nullptr;
    if constexpr (TABLE) {
        if (f.lut_general) {
            lutw = lut_lds[wave_in_block()];
            lutw[lane] = reinterpret_cast<const IH_GLOBAL uint32_t*>(gmem(f.lut))[lane];
            __builtin_amdgcn_s_waitcnt(0);
            __builtin_amdgcn_wave_barrier();
        }
    }
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
    // == b.  A non-decreasing bin table: lo = #{v : lut[v] < b}, lo + width =
    // #{v : lut[v] <= b}.  A lane tests v - lo < width (unsigned); an empty
    // bin has width 0.  Any other table: v is the pixel's bin, lo = b, width 1.
    uint32_t lo[BPL], wd[BPL];
    bool bvalid[BPL];
#pragma unroll
    for (int t = 0; t < BPL; ++t) bvalid[t] = GUARD ? b0 + t < B : true;
    if constexpr (TABLE) {
        const IH_GLOBAL uint8_t* lt = gmem(f.lut);
#pragma unroll
        for (int t = 0; t < BPL; ++t) {
            uint32_t l = (uint32_t)(b0 + t), h = l + 1;
            if (!lutw) {
                l = lut_count_below(lt, (uint32_t)(b0 + t));
                h = lut_count_below(lt, (uint32_t)(b0 + t + 1));
            }
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

    // Left carries and pixels, a chunk of rows at a time (see below); the
    // first chunk's loads go out before the column state's, so that every
    // load the work item needs before its first store is in flight at once.
    // Several segments per wave (B < 64, compile-time B, whole segments):
    // the pixels of a chunk of rows for all of the wave's segments come in
    // one wave-wide load, and each lane fetches its segment's bytes of a row
    // from the lane holding them (ds_bpermute).  Piece p (16 bytes) of a
    // chunk is row r, 16-byte column c, segment s with p = (r * PPR + c) * SC
    // + s, held by lane p.
    constexpr int SC = kWave / LC;
    constexpr int PPR = TX / 16;
    constexpr bool CHUNK_PX = !GUARD && !UNIFORM && BC != 0 && SC * PPR <= kWave;
    constexpr int CH = CHUNK_PX ? (8 / BPL < kWave / (SC * PPR) ? 8 / BPL : kWave / (SC * PPR)) : 8 / BPL;
    uint32_t cb[CH][BPL], nb[CH][BPL];
    auto load_chunk_px = [&](int yc, u32x4& dst) {
        const int p = lane < CH * SC * PPR ? lane : 0;
        const int ps = p % SC, pc_ = (p / SC) % PPR, pr = p / (SC * PPR);
        const int row = min(yc + pr, y1 - 1);
        const int px0 = (jg * SC + ps) * TX + 16 * pc_;
        dst = *reinterpret_cast<const IH_GLOBAL u32x4*>(gmem(f.frame) + (size_t)row * g.W + px0);
    };
    u32x4 pc, pn;
    uint32_t pxa[TX / 4], pxb[TX / 4];
    load_carries<BPL, CH>(f, y0, y1 - 1, j, b0, B, bvalid, cb);
    if constexpr (CHUNK_PX) {
        static_assert(CH * SC * PPR <= kWave, "a pixel chunk must fit one wave-wide load");
        load_chunk_px(y0, pc);
    } else {
        load_px<TX, GUARD, UNIFORM>(f, y0, x0, ncols, pxa);
    }

    // Column state: corner + running sum of the top carries along the segment.
    // Reduce-then-scan: the scans left tile (i, j)'s corner count and band
    // i's top carries.  Prefix counts: the top carries are stored as they
    // are; the corner is the sum of the tile-column totals left of tile j.
    // Fused: tile band i is band k of carry band I.  Its corner is the sum,
    // over the carry bands above, of their pixels left of the tile column,
    // plus the pixels of carry band I's first k tile bands left of it
    // (snapshot k - 1); a column's top carry is its count above carry band I
    // plus the same snapshot's count.  The top carries are loaded into V
    // first and the corner terms after them; masked-off terms read a valid
    // address and add zero, so no load waits behind a branch.
    uint32_t V[BPL][TX];
    {
        uint32_t acc[BPL];
        const IH_GLOBAL uint32_t* corner = gmem(f.corner);
        const IH_GLOBAL uint32_t* colc = gmem(f.colc);
        size_t tofs;
        const IH_GLOBAL uint32_t* tq = nullptr;
        const int K = g.K, I = K ? i / K : 0, k_in = i - I * K;
        if (g.PC || K == 0) {
            tofs = ((size_t)i * g.W + x0) * B + b0;
        } else {
            tofs = (((size_t)I * K + K - 1) * g.W + x0) * B + b0;
            if (k_in > 0) tq = colc + (((size_t)I * K + k_in - 1) * g.W + x0) * B + b0;
        }
        if (g.CC16) {
            const IH_GLOBAL uint16_t* c16 = gmem(reinterpret_cast<const uint16_t*>(f.colc));
#pragma unroll
            for (int k = 0; k < TX; ++k)
#pragma unroll
                for (int t = 0; t < BPL; ++t) {
                    const bool ok = k < ncols && bvalid[t];
                    const uint32_t v = *(ok ? c16 + tofs + (size_t)k * B + t : c16);
                    V[t][k] = ok ? v : 0u;
                }
        } else {
#pragma unroll
            for (int k = 0; k < TX; ++k)
#pragma unroll
                for (int t = 0; t < BPL; ++t) {
                    const bool ok = k < ncols && bvalid[t];
                    const uint32_t v = *(ok ? colc + tofs + (size_t)k * B + t : colc);
                    V[t][k] = ok ? v : 0u;
                }
        }
        if (tq) {
#pragma unroll
            for (int k = 0; k < TX; ++k)
#pragma unroll
                for (int t = 0; t < BPL; ++t) {
                    const bool ok = k < ncols && bvalid[t];
                    const uint32_t v = *(ok ? tq + (size_t)k * B + t : colc);
                    V[t][k] += ok ? v : 0u;
                }
        }
#pragma unroll
        for (int t = 0; t < BPL; ++t) acc[t] = 0u;
        if (g.PC) {
            // the totals of the tile columns to the left, LB columns of loads
            // in flight together
            constexpr int LB = TX * BPL <= 32 ? 16 : 8;
            const IH_GLOBAL uint32_t* cp = corner + (size_t)i * g.nTX * B + b0;
            for (int jp = 0; jp < j; jp += LB) {
                uint32_t v[LB][BPL];
#pragma unroll
                for (int u = 0; u < LB; ++u)
#pragma unroll
                    for (int t = 0; t < BPL; ++t) {
                        const bool ok = jp + u < j && bvalid[t];
                        v[u][t] = *(ok ? cp + (size_t)(jp + u) * B + t : corner);
                        v[u][t] = ok ? v[u][t] : 0u;
                    }
                // all of the chunk's loads issue before any of them is waited for
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int u = 0; u < LB; ++u)
#pragma unroll
                    for (int t = 0; t < BPL; ++t) acc[t] += v[u][t];
            }
        } else if (K == 0) {
            const IH_GLOBAL uint32_t* cp = corner + ((size_t)i * g.nTX + j) * B + b0;
#pragma unroll
            for (int t = 0; t < BPL; ++t) acc[t] = bvalid[t] ? cp[t] : 0u;
        } else {
            const size_t band_words = (size_t)K * g.nTX * B;
            const IH_GLOBAL uint32_t* cq = corner + ((size_t)(K - 1) * g.nTX + j) * B + b0;
#pragma unroll 4
            for (int ip = 0; ip < I; ++ip)
#pragma unroll
                for (int t = 0; t < BPL; ++t)
                    if (bvalid[t]) acc[t] += cq[(size_t)ip * band_words + t];
            if (k_in > 0) {
                const IH_GLOBAL uint32_t* cp = corner + (((size_t)I * K + k_in - 1) * g.nTX + j) * B + b0;
#pragma unroll
                for (int t = 0; t < BPL; ++t)
                    if (bvalid[t]) acc[t] += cp[t];
            }
        }
#pragma unroll
        for (int k = 0; k < TX; ++k)
#pragma unroll
            for (int t = 0; t < BPL; ++t) {
                acc[t] += V[t][k];
                V[t][k] = acc[t];
            }
    }

    const bool vec_ok = (b0 + BPL <= B) && (B % BPL == 0) &&
                        ((reinterpret_cast<uintptr_t>(f.out) & (4 * BPL - 1)) == 0);

    auto row_pass = [&](int y, const uint32_t (&px_in)[TX / 4], const uint32_t (&c0)[BPL]) {
        IH_GLOBAL uint32_t* orow = gmem(f.out) + ((size_t)y * g.W + x0) * B + b0;
        uint32_t px[TX / 4];
#pragma unroll
        for (int q = 0; q < TX / 4; ++q) px[q] = px_in[q];
        if constexpr (TABLE) {
            if (lutw) {
                // bin every pixel of the row through the table
#pragma unroll
                for (int q = 0; q < TX / 4; ++q) {
                    uint32_t w = 0;
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const uint32_t v = (px[q] >> (8 * e)) & 0xFFu;
                        w |= ((lutw[v >> 2] >> (8 * (v & 3u))) & 0xFFu) << (8 * e);
                    }
                    px[q] = w;
                }
            }
        }
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
    if constexpr (CHUNK_PX) {
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
    // Scalar loads (the pixels of one-segment waves) may return out of order,
    // so a wait for one of them is a wait for all: the row being started
    // waits for its own pixels (loaded a row earlier) before the next row's
    // loads go out, and the compiler then needs no wait that would cover
    // those.
    auto wait_scalar = [&]() {
        if constexpr (UNIFORM && !GUARD) {
            __builtin_amdgcn_sched_barrier(0);
            __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
            __builtin_amdgcn_sched_barrier(0);
        }
    };
    // Drain everything once per work item, so that inside the loop the
    // compiler's counter bookkeeping sees only the in-loop prefetches.
    __builtin_amdgcn_s_waitcnt(0);
    for (int yc = y0; yc < y1; yc += CH) {
        if (yc + CH < y1) load_carries<BPL, CH>(f, yc + CH, y1 - 1, j, b0, B, bvalid, nb);
#pragma unroll 1
        for (int r = 0; r < CH; r += 2) {
            const int y = yc + r;
            wait_scalar();
            load_px<TX, GUARD, UNIFORM>(f, min(y + 1, y1 - 1), x0, ncols, pxb);
            __builtin_amdgcn_sched_barrier(0);        // keep the prefetch ahead of the stores
            if (y < y1) row_pass(y, pxa, cb[0]);
#pragma unroll
            for (int q = 0; q + 1 < CH; ++q)
#pragma unroll
                for (int t = 0; t < BPL; ++t) cb[q][t] = cb[q + 1][t];
            wait_scalar();
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

// Persistent form over the work items of all jobs.  With a scheduling
// counter (sched: next item, waves finished; both zero at launch) each wave
// takes the next item from the counter when it finishes one, so waves that
// drew small items take more of them (the job table lists the largest items
// first); the last wave to finish resets both words for the next launch.
// Without one, each wave strides over the items.
template <int BPL, int TX, int BC, bool NT, bool GUARD, bool TABLE>
__global__ __launch_bounds__(kWave * kWavesPerBlock)
void tile_batch_kernel(const FrameArgs* __restrict__ frames, const Job* __restrict__ jobs,
                       int32_t njobs, int64_t nitems, uint32_t* sched)
{
    auto run = [&](int64_t item) {
        const Job jb = cload(jobs, find_job(cmem(jobs), njobs, item));
        const int64_t local = item - jb.begin;
        const int i = (int)(local / jb.jg_count);
        const int jg = jb.jg_begin + (int)(local - (int64_t)i * jb.jg_count);
        const FrameArgs f = cload(frames, jb.frame);
        tile_body<BPL, TX, BC, NT, GUARD, TABLE>(f, i, jg, threadIdx.x % kWave);
    };
    if (sched) {
        const bool leader = threadIdx.x % kWave == 0;
        for (;;) {
            uint32_t got = 0;
            if (leader) got = atomicAdd(&sched[0], 1u);
            const int64_t item = (int64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)got);
            if (item >= nitems) break;                        // whole wave leaves together
            run(item);
        }
        if (leader && atomicAdd(&sched[1], 1u) == gridDim.x * (uint32_t)kWavesPerBlock - 1u) {
            // every wave has taken its last item: nobody reads the counter again in this launch
            atomicExch(&sched[0], 0u);
            atomicExch(&sched[1], 0u);
        }
        return;
    }
    const int64_t stride = (int64_t)gridDim.x * kWavesPerBlock;
    for (int64_t item = (int64_t)blockIdx.x * kWavesPerBlock + wave_in_block(); item < nitems; item += stride)
        run(item);
}

template <int BPL, int TX, int BC, bool NT, bool GUARD, bool TABLE = false>
TileFns fns_of()
{
    return TileFns{reinterpret_cast<const void*>(&tile_kernel<BPL, TX, BC, NT, GUARD, TABLE>),
                   reinterpret_cast<const void*>(&tile_batch_kernel<BPL, TX, BC, NT, GUARD, TABLE>)};
}

// Frames binned by a table: runtime B and regular stores only.
template <bool GUARD>
TileFns pick_table(const TileVariant& v)
{
    switch (v.bpl) {
    case 1: return v.tx == 32 ? fns_of<1, 32, 0, false, GUARD, true>() : fns_of<1, 64, 0, false, GUARD, true>();
    case 2: return v.tx == 32 ? fns_of<2, 32, 0, false, GUARD, true>() : fns_of<2, 64, 0, false, GUARD, true>();
    default: return fns_of<4, 32, 0, false, GUARD, true>();
    }
}

template <int BPL, int TX, bool NT, bool GUARD>
TileFns pick_bc(int bc)
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
TileFns pick_v(const TileVariant& v)
{
    switch (v.bpl) {
    case 1:
        if (v.tx == 128) return fns_of<1, 128, 64, NT, GUARD>();      // B == 64 only
        return v.tx == 32 ? pick_bc<1, 32, NT, GUARD>(v.bc) : pick_bc<1, 64, NT, GUARD>(v.bc);
    case 2: return v.tx == 32 ? pick_bc<2, 32, NT, GUARD>(v.bc) : pick_bc<2, 64, NT, GUARD>(v.bc);
    default: return pick_bc<4, 32, NT, GUARD>(v.bc);
    }
}


}  // namespace ih
