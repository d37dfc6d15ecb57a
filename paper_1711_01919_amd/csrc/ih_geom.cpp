// Host-side geometry of the tile decomposition: scratch layout, frame
// arguments, supported tiles and the single-frame tile heuristic, and the
// choice of compiled tile-kernel variant.  No device code.
#include "ih_internal.h"

namespace ih {

ScratchLayout scratch_layout(const Geom& g)
{
    ScratchLayout s;
    const size_t bands = g.K ? (size_t)g.nS * g.K : (size_t)g.nTY;
    s.cnt = 0;
    s.rowc = kCounterWords;
    const size_t rowc_entries = (size_t)g.H * g.nTX * g.B;
    const size_t rowc_words = g.RC16 ? (rowc_entries + 1) / 2 : rowc_entries;
    s.colc = s.rowc + (rowc_words + 63) / 64 * 64;
    const size_t colc_entries = bands * g.W * g.B;
    const size_t colc_words = g.CC16 ? (colc_entries + 1) / 2 : colc_entries;
    s.corner = s.colc + (colc_words + 63) / 64 * 64;
    s.words = s.corner + bands * g.nTX * g.B;
    return s;
}

FrameArgs frame_args(const uint8_t* frame, uint32_t* out, uint32_t* scratch, const Geom& g,
                     const uint8_t* lut, bool lut_general)
{
    const ScratchLayout sl = scratch_layout(g);
    return FrameArgs{frame, out, scratch + sl.rowc, scratch + sl.colc, scratch + sl.corner, scratch + sl.cnt,
                     lut, lut && lut_general ? 1 : 0, g};
}

bool lut_is_general(const uint8_t* lut_host)
{
    for (int v = 1; v < 256; ++v)
        if (lut_host[v] < lut_host[v - 1]) return true;
    return false;
}

bool fused_supported(const Geom& g)
{
    return g.K >= 1 && (int64_t)g.nTX + g.nS <= kCounterWords && (int64_t)g.K * g.TY <= 65535;
}

bool prefix_supported(const Geom& g)
{
    return g.PC == 1 && g.K == 0 && g.H <= 65536 && g.nTX <= kMaxPrefixTileColumns;
}

int32_t fused_bands(int32_t nTY, int32_t max_bands)
{
    return (nTY + max_bands - 1) / max_bands;
}

int64_t count_tile_blocks(const Geom& g) { return (int64_t)g.nTX * (g.K ? g.nS : g.nTY); }

int bins_per_lane(int B) { return B <= 64 ? 1 : (B <= 128 ? 2 : 4); }

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
    g.PC = t.prefix ? 1 : 0;
    g.CPL = t.bm_cpl;
    g.RC16 = W <= 65536 ? 1 : 0;
    g.K = t.K > 0 && !t.prefix ? t.K : 0;
    g.CC16 = g.K == 0 && H <= 65536 ? 1 : 0;
    g.nS = g.K ? (g.nTY + g.K - 1) / g.K : 0;
    return g;
}

bool tile_supported(int32_t B, const TileChoice& t)
{
    const int bpl = bins_per_lane(B);
    if (t.TY < 1 || t.TY > 65535) return false;
    if (bpl == 4) return t.TX == 32;
    if (bpl == 2) return t.TX == 32 || t.TX == 64;
    // 128 columns of accumulators fit the register file only with one
    // segment per wave and compile-time B
    return t.TX == 32 || t.TX == 64 || (t.TX == 128 && B == 64);
}

int32_t even_band_height(int32_t H, int32_t TY)
{
    const int32_t n = (H + TY - 1) / TY;
    return (H + n - 1) / n;
}

TileChoice default_tile(int32_t H, int32_t W, int32_t B)
{
    TileChoice t;
    t.nontemporal = false;
    // Frames up to 1920 x 1080 with B <= 64: measured one-frame sweeps (ten
    // shapes from 640 x 480 to 1920 x 1080, B = 16 to 64) favour 32-column
    // tiles and fewer, taller bands than the rule below (1920 x 1080 B=32:
    // 70.0 us at 32 x 64 against 88.6 us at 64 x 16; B=64: 126 against 132 us
    // at 64 x 32; 640 x 480 B=64: 28.4 against 32.3 us), as long as a band's
    // work items stay below about 640 KB of output (1920 x 1080 B=64 at
    // 32 x 128: 146 us) and leave some 450 of them.
    if (bins_per_lane(B) == 1 && (int64_t)H * W <= kMidFramePixels) {
        // non-temporal stores: 1-6% faster on every such frame measured
        // (640 x 480 B=32 19.3 against 20.6 us, 1920 x 1080 B=16 47.1 against
        // 49.6 us)
        t.nontemporal = true;
        t.TX = 32;
        const Geom g0 = make_geom(H, W, B, TileChoice{32, 1, false});
        const int64_t row_bytes = (int64_t)g0.S * 32 * B * 4;      // a work item's output per row
        auto bands = [&](int ty) { return (H + ty - 1) / ty; };
        int TY = 512;
        while (TY > 8 && ((int64_t)bands(TY) * g0.nJG < kMidFrameWaves || row_bytes * TY > kMidFrameItemBytes))
            TY /= 2;
        t.TY = TY;
        t.prefix = bands(TY) <= kMaxPrefixBands && (int64_t)H * W * bands(TY) / 2 <= kMidPrefixPixels;
        t.TY = even_band_height(H, t.TY);
        if (t.prefix && !prefix_supported(make_geom(H, W, B, t))) t.prefix = false;
        return t;
    }
    // Tallest tile (fewest carries) that still gives enough independent
    // waves (one per work item in a single-frame launch).  Frames above
    // 1920 x 1080 and up to 3840 x 2160 with B <= 128 take non-temporal
    // stores and at least about
    // 480 waves (3840 x 2160 B=16 / 32 / 64 / 128: 140 / 214 / 413 / 785 us
    // against 147 / 237 / 451 / 860 us with regular stores and about 1000
    // waves); larger ones about 1000 waves and regular stores (7680 x 4320
    // B=16 took 774 us with non-temporal stores against 492 us).  B=64 takes
    // 128-column tiles, and beyond 3840 x 2160 bands of at most 256 rows
    // (7680 x 4320 B=64: 1.66 ms at 128 x 256 against 2.16 ms at 64 x 512;
    // 8192 x 8192 B=64: 3.18 against 3.48 ms).
    const bool upto4k = bins_per_lane(B) <= 2 && (int64_t)H * W > kMidFramePixels && (int64_t)H * W <= k4KFramePixels;
    const int64_t min_waves = upto4k ? kMinWaves4K : kMinWaves;
    auto waves = [&](int tx, int ty) {
        return (int64_t)((H + ty - 1) / ty) * make_geom(H, W, B, TileChoice{tx, 1, false}).nJG;
    };
    t.TX = bins_per_lane(B) == 4 ? 32 : 64;
    if (B == 64 && waves(128, 16) >= min_waves) t.TX = 128;
    int TY = (t.TX == 128 && !upto4k) ? 256 : 512;
    while (TY > 16 && waves(t.TX, TY) < min_waves) TY /= 2;
    t.TY = TY;
    t.nontemporal = upto4k && waves(t.TX, TY) >= min_waves;
    // Small frames (too few waves even at 16 rows): 32-column tiles for
    // parallelism and the prefix-count schedule (two launches, no scans;
    // 640 x 480 B=32: 25.0 against 29.0 us per frame under reduce-then-scan
    // with 8-row bands).  Its count blocks read about bands / 2 frames' worth
    // of pixels, so bands start at 8 rows and grow until there are at most
    // kMaxPrefixBands of them and that stays within kPrefixCountPixels
    // (1920 x 1080 B=16: 32-row bands, 70.6 us against 107 us at 8 rows and
    // 150 us under reduce-then-scan).
    if (waves(t.TX, TY) < min_waves) {
        t.TX = 32;
        t.TY = 8;
        t.nontemporal = false;
        auto bands = [&](int ty) { return (H + ty - 1) / ty; };
        while (t.TY < 64 && (bands(t.TY) > kMaxPrefixBands || (int64_t)H * W * bands(t.TY) / 2 > kPrefixCountPixels))
            t.TY *= 2;
        t.prefix = (H + t.TY - 1) / t.TY <= kMaxPrefixBands;
        if (!t.prefix) t.TY = 8;
    }
    t.TY = even_band_height(H, t.TY);
    if (t.prefix && !prefix_supported(make_geom(H, W, B, t))) t.prefix = false;
    return t;
}

void binmajor_tiles(const BinmajorShape* frames, size_t n, TileChoice* tiles)
{
    auto items = [&](int cpl, int ty) {
        int64_t it = 0;
        for (size_t k = 0; k < n; ++k) {
            int bg = 16;
            while (frames[k].B % bg != 0) bg >>= 1;
            it += (int64_t)((frames[k].H + ty - 1) / ty) * bm_segments(frames[k].W, cpl) * (frames[k].B / bg);
        }
        return it;
    };
    const int cpl = items(4, 64) >= kBmItemsWide ? 4 : 1;
    const int64_t target = cpl == 4 ? kBmItemsWide : kBmItemsNarrow;
    int ty = 512;
    while (ty > 8 && items(cpl, ty) < target) ty /= 2;
    for (size_t k = 0; k < n; ++k) {
        tiles[k] = TileChoice{64, even_band_height(frames[k].H, ty), false};
        tiles[k].bm_cpl = cpl;
    }
}

TileChoice binmajor_tile(int32_t H, int32_t W, int32_t B)
{
    const BinmajorShape f{H, W, B};
    TileChoice t;
    binmajor_tiles(&f, 1, &t);
    return t;
}

int32_t interior_groups(const Geom& g, const uint8_t* frame, const uint32_t* out)
{
    const bool aligned = ((reinterpret_cast<uintptr_t>(frame) & 15) == 0) && (g.W % 16 == 0) &&
                         (g.B % g.BPL == 0) &&
                         ((reinterpret_cast<uintptr_t>(out) & (4 * g.BPL - 1)) == 0);
    if (!aligned) return 0;
    // Only groups whose S segments are all whole tiles: the unguarded kernel
    // may load pixels of every segment of its group.
    return (g.W / g.TX) / g.S;
}

bool TileVariant::operator<(const TileVariant& o) const
{
    if (bpl != o.bpl) return bpl < o.bpl;
    if (tx != o.tx) return tx < o.tx;
    if (bc != o.bc) return bc < o.bc;
    if (nt != o.nt) return nt < o.nt;
    if (guard != o.guard) return guard < o.guard;
    return table < o.table;
}
bool TileVariant::operator==(const TileVariant& o) const
{
    return bpl == o.bpl && tx == o.tx && bc == o.bc && nt == o.nt && guard == o.guard && table == o.table;
}

// Bin counts with a specialised kernel (compile-time B); others use runtime B.
static int32_t const_bins(int bpl, int B)
{
    if (bpl == 1 && (B == 16 || B == 32 || B == 64)) return B;
    if (bpl == 2 && B == 128) return B;
    if (bpl == 4 && B == 256) return B;
    return 0;
}

TileVariant tile_variant(const Geom& g, bool nontemporal, bool guard, bool table)
{
    if (table) return TileVariant{g.BPL, g.TX, 0, false, guard, true};
    return TileVariant{g.BPL, g.TX, const_bins(g.BPL, g.B), nontemporal, guard, false};
}

}  // namespace ih
