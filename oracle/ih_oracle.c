/*
 * Integral-histogram ORACLE -- test infrastructure, not product code.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * load this library.  It shares no source, header, table or helper with the
 * HIP implementation, and the HIP implementation never calls it.
 *
 * Plain, slow, sequential C.  Every function below follows a passage of
 * "Fast Integral Histogram Computations on GPU for Real-Time Video
 * Analytics" (Poostchi et al.), cited in its comment:
 *
 *   ihref_Q                   binning function Q of Sec. 2.1 (text of Eq. 1)
 *   ihref_integral_histogram  Eq. 1, evaluated with the sequential recursion
 *                             of Sec. 2.2, Algorithm 1
 *   ihref_integral_histogram_lut  Eq. 1 / Algorithm 1 with Q given as a table
 *                             (bins of arbitrary edges: the paper states Q as
 *                             membership of I(r,c) in bin b without fixing
 *                             the bins, Sec. 2.1)
 *   ihref_integral_histogram_binmajor  Eq. 1 per bin plane as running sums
 *                             along rows, then down columns, stored b x h x w
 *                             (the paper's layout, Sec. 3.1)
 *   ihref_integral_rows       the same recursion continued over a block of
 *                             rows, for frames whose tensor does not fit RAM
 *   ihref_row_by_definition   one row of Eq. 1, summed directly (columns
 *                             first, then rows) -- no recursion
 *   ihref_entry               one entry of Eq. 1 as the literal double sum
 *   ihref_region_histogram    Eq. 2, four-corner region query
 *   ihref_rect_count          a region's histogram by direct counting
 *
 * Conventions (readings of points the paper leaves open):
 *   - layout: the tensor is H x W x B with the bin index innermost,
 *     entry (x, y, b) at offset (y*W + x)*B + b;  x is the column in [0,W),
 *     y the row in [0,H);
 *   - Q(v) = floor(v*B/256) for a uint8 value v and 1 <= B <= 256;
 *   - the sums of Eq. 1 are inclusive; H at index -1 is 0;
 *   - counts are uint32 ("4 byte integers", Sec. 4.6); callers keep H*W below
 *     2^32, so no entry can overflow;
 *   - a query rectangle {x0,y0,x1,y1} has inclusive corners, and Eq. 2 is
 *     applied with r- = x0-1, c- = y0-1 (zero at -1), in modular uint32
 *     arithmetic.
 *
 * The test suite shows that its pins catch plausible mistakes by compiling
 * copies of this file with one mistake patched in; this file itself holds
 * none and has no switch for them.
 */
#include <stdint.h>
#include <stddef.h>
#include <string.h>
#include <stdlib.h>

/* Sec. 2.1: Q(I(r,c), b) is 1 when the value I(r,c) lies in bin b.  The paper
 * gives no bin edges; the bins here split [0,256) uniformly by
 * floor(v*B/256), so bin b holds the values v with 256*b <= v*B < 256*(b+1). */
uint32_t ihref_Q(uint32_t v, uint32_t B)
{
    return (v * B) >> 8;
}

static uint32_t at(const uint32_t* Ht, int64_t W, int64_t B, int64_t x, int64_t y, int64_t b)
{
    /* H at index -1 (row or column) is zero: Algorithm 1 starts from H <- 0
     * and its recursion reads the neighbours at x-1 and y-1. */
    if (x < 0 || y < 0) return 0u;
    return Ht[(y * W + x) * B + b];
}

/*
 * Sec. 2.2, Algorithm 1 (sequential integral histogram), which evaluates
 * Eq. 1:  H(x,y,b) = H(x-1,y,b) + H(x,y-1,b) - H(x-1,y-1,b) + Q(I(x,y),b).
 *
 * The paper loops over bins outermost and stores b x h x w; the bins are
 * independent of each other (Sec. 3.2), so here the bin loop sits innermost,
 * which visits the H x W x B layout in memory order and yields the same
 * values.  Rows run top to bottom and columns left to right, as in the
 * listing, so every neighbour read has already been written.
 *
 * Returns 0 on success, -1 on bad arguments.
 */
int ihref_integral_histogram(const uint8_t* I, int64_t H, int64_t W, int64_t B, uint32_t* out)
{
    if (!I || !out || H <= 0 || W <= 0 || B < 1 || B > 256) return -1;
    for (int64_t y = 0; y < H; ++y) {
        for (int64_t x = 0; x < W; ++x) {
            const uint32_t q = ihref_Q(I[y * W + x], (uint32_t)B);
            for (int64_t b = 0; b < B; ++b) {
                uint32_t h = at(out, W, B, x - 1, y, b)
                           + at(out, W, B, x, y - 1, b)
                           - at(out, W, B, x - 1, y - 1, b);
                if (q == (uint32_t)b) h += 1u;
                out[(y * W + x) * B + b] = h;
            }
        }
    }
    return 0;
}

/*
 * Eq. 1 stored bin-major, b x h x w, as the paper lays the tensor out
 * (Sec. 3.1, Fig. 2): entry (x, y, b) at (b*H + y)*W + x.  Each bin plane
 * takes the double sum of Eq. 1 as two running sums: along every row first
 * (the sum over columns c <= x of the bin indicator), then down every column
 * of those row sums (the sum over rows r <= y).
 * Returns 0 on success, -1 on bad arguments.
 */
int ihref_integral_histogram_binmajor(const uint8_t* I, int64_t H, int64_t W, int64_t B, uint32_t* out)
{
    if (!I || !out || H <= 0 || W <= 0 || B < 1 || B > 256) return -1;
    for (int64_t b = 0; b < B; ++b) {
        uint32_t* P = out + b * H * W;
        for (int64_t y = 0; y < H; ++y) {
            uint32_t run = 0;
            for (int64_t x = 0; x < W; ++x) {
                run += ihref_Q(I[y * W + x], (uint32_t)B) == (uint32_t)b ? 1u : 0u;
                P[y * W + x] = run;
            }
        }
        for (int64_t y = 1; y < H; ++y)
            for (int64_t x = 0; x < W; ++x)
                P[y * W + x] += P[(y - 1) * W + x];
    }
    return 0;
}

/*
 * Sec. 2.2, Algorithm 1 again, with the membership test Q(I(x,y), b) of Eq. 1
 * read from a table: the pixel of value v counts in bin lut[v] (lut holds 256
 * entries, each below B).  Any table is accepted; tables whose entries never
 * decrease give bins that are contiguous value ranges with arbitrary edges.
 * Returns 0 on success, -1 on bad arguments.
 */
int ihref_integral_histogram_lut(const uint8_t* I, int64_t H, int64_t W, int64_t B, const uint8_t* lut,
                                 uint32_t* out)
{
    if (!I || !out || !lut || H <= 0 || W <= 0 || B < 1 || B > 256) return -1;
    for (int v = 0; v < 256; ++v)
        if ((int64_t)lut[v] >= B) return -1;
    for (int64_t y = 0; y < H; ++y) {
        for (int64_t x = 0; x < W; ++x) {
            const uint32_t q = lut[I[y * W + x]];
            for (int64_t b = 0; b < B; ++b) {
                uint32_t h = at(out, W, B, x - 1, y, b) + at(out, W, B, x, y - 1, b)
                           - at(out, W, B, x - 1, y - 1, b);
                if (q == (uint32_t)b) h += 1u;
                out[(y * W + x) * B + b] = h;
            }
        }
    }
    return 0;
}

/*
 * Algorithm 1 continued over rows [y_begin, y_end) only, for tensors too large
 * to hold at once.  prev_row holds H(., y_begin-1, .) as W*B entries (ignored,
 * and may be NULL, when y_begin == 0).  out_rows receives (y_end-y_begin)*W*B
 * entries, row after row.  The caller passes the last produced row as
 * prev_row of the next block.
 */
int ihref_integral_rows(const uint8_t* I, int64_t H, int64_t W, int64_t B,
                        int64_t y_begin, int64_t y_end,
                        const uint32_t* prev_row, uint32_t* out_rows)
{
    if (!I || !out_rows || H <= 0 || W <= 0 || B < 1 || B > 256) return -1;
    if (y_begin < 0 || y_end > H || y_begin >= y_end) return -1;
    if (y_begin > 0 && !prev_row) return -1;
    const int64_t rowlen = W * B;
    for (int64_t y = y_begin; y < y_end; ++y) {
        uint32_t* cur = out_rows + (y - y_begin) * rowlen;
        const uint32_t* up = (y == y_begin) ? (y_begin > 0 ? prev_row : NULL)
                                            : out_rows + (y - y_begin - 1) * rowlen;
        for (int64_t x = 0; x < W; ++x) {
            const uint32_t q = ihref_Q(I[y * W + x], (uint32_t)B);
            for (int64_t b = 0; b < B; ++b) {
                const uint32_t left = x > 0 ? cur[(x - 1) * B + b] : 0u;
                const uint32_t above = up ? up[x * B + b] : 0u;
                const uint32_t corner = (up && x > 0) ? up[(x - 1) * B + b] : 0u;
                cur[x * B + b] = left + above - corner + (q == (uint32_t)b ? 1u : 0u);
            }
        }
    }
    return 0;
}

/*
 * Row y of Eq. 1 summed directly, without the recursion:
 *   H(x,y,b) = sum_{x'<=x} ( sum_{y'<=y} Q(I(x',y'), b) ).
 * The inner sum is a per-column count over rows 0..y; the outer sum runs over
 * columns.  Costs O(W*(y+1) + W*B); row_out receives W*B entries.
 */
int ihref_row_by_definition(const uint8_t* I, int64_t H, int64_t W, int64_t B,
                            int64_t y, uint32_t* row_out)
{
    if (!I || !row_out || H <= 0 || W <= 0 || B < 1 || B > 256 || y < 0 || y >= H) return -1;
    uint32_t* colcount = (uint32_t*)calloc((size_t)(W * B), sizeof(uint32_t));
    if (!colcount) return -1;
    for (int64_t yy = 0; yy <= y; ++yy)
        for (int64_t x = 0; x < W; ++x)
            colcount[x * B + ihref_Q(I[yy * W + x], (uint32_t)B)] += 1u;
    for (int64_t b = 0; b < B; ++b) {
        uint32_t s = 0;
        for (int64_t x = 0; x < W; ++x) {
            s += colcount[x * B + b];
            row_out[x * B + b] = s;
        }
    }
    free(colcount);
    return 0;
}

/* One entry of Eq. 1 as the literal double sum over the rectangle from the
 * top-left corner to (x, y).  O((x+1)*(y+1)). */
uint32_t ihref_entry(const uint8_t* I, int64_t W, int64_t B, int64_t x, int64_t y, int64_t b)
{
    uint32_t s = 0;
    for (int64_t r = 0; r <= y; ++r)
        for (int64_t c = 0; c <= x; ++c)
            s += (ihref_Q(I[r * W + c], (uint32_t)B) == (uint32_t)b) ? 1u : 0u;
    return s;
}

/*
 * Sec. 2.1, Eq. 2:  h(R,b) = H(r+,c+,b) - H(r-,c+,b) - H(r+,c-,b) + H(r-,c-,b).
 * rects holds n records {x0,y0,x1,y1} (int32, inclusive corners); the corners
 * used are (x1,y1), (x0-1,y1), (x1,y0-1), (x0-1,y0-1), with H = 0 at index -1.
 * hists receives n*B entries.  Returns the index+1 of the first invalid
 * rectangle (nothing written for it or after it), or 0 when all are valid.
 */
int64_t ihref_region_histogram(const uint32_t* Ht, int64_t H, int64_t W, int64_t B,
                               const int32_t* rects, int64_t n, uint32_t* hists)
{
    for (int64_t i = 0; i < n; ++i) {
        const int64_t x0 = rects[4 * i + 0], y0 = rects[4 * i + 1];
        const int64_t x1 = rects[4 * i + 2], y1 = rects[4 * i + 3];
        if (x0 < 0 || y0 < 0 || x1 < x0 || y1 < y0 || x1 >= W || y1 >= H) return i + 1;
        for (int64_t b = 0; b < B; ++b) {
            const uint32_t h = at(Ht, W, B, x1, y1, b) - at(Ht, W, B, x0 - 1, y1, b)
                             - at(Ht, W, B, x1, y0 - 1, b) + at(Ht, W, B, x0 - 1, y0 - 1, b);
            hists[i * B + b] = h;
        }
    }
    return 0;
}

/* The histogram of one rectangle by counting its pixels: the quantity Eq. 2
 * is meant to return, computed without the integral histogram. */
int ihref_rect_count(const uint8_t* I, int64_t H, int64_t W, int64_t B,
                     int32_t x0, int32_t y0, int32_t x1, int32_t y1, uint32_t* hist)
{
    if (x0 < 0 || y0 < 0 || x1 < x0 || y1 < y0 || x1 >= W || y1 >= H) return -1;
    memset(hist, 0, (size_t)B * sizeof(uint32_t));
    for (int64_t r = y0; r <= y1; ++r)
        for (int64_t c = x0; c <= x1; ++c)
            hist[ihref_Q(I[r * W + c], (uint32_t)B)] += 1u;
    return 0;
}
