"""Pins for the CPU oracle: checks against what the paper and the mathematics
fix, none of which re-types the oracle's own recursion.

  - brute force of Eq. 1 (the double sum) on every tiny frame shape;
  - invariants: per-pixel bin sum (x+1)(y+1), last entry = full-frame
    histogram, 2-D backward difference = one-hot of the binned frame,
    monotone in x and y;
  - closed forms: constant frame, B=1, frames binned by column only or row only;
  - the textbook route cumsum(cumsum(one-hot)) on a full 640x480 frame;
  - hand-worked fixtures under tests/golden/;
  - Eq. 2 against direct pixel counting and the area invariant;
  - table binning: brute force with the table's one-hot, the uniform table
    equals Q, empty bins stay zero;
  - bin-major storage: brute force per bin plane;
  - planted mistakes: every copy of the oracle with one plausible mistake
    patched in must fail a pin.
"""
import json
from pathlib import Path

import numpy as np
import pytest

import oracle

GOLDEN = Path(__file__).resolve().parent / "golden"


def onehot_numpy(I, B):
    """One-hot of the binned frame, written independently in numpy: bin b holds
    the values v with 256*b <= v*B < 256*(b+1)."""
    v = I.astype(np.int64)[..., None]
    b = np.arange(B, dtype=np.int64)
    return ((v * B >= 256 * b) & (v * B < 256 * (b + 1))).astype(np.uint32)


def onehot_lut_numpy(I, B, lut):
    """One-hot of a frame binned through a 256-entry table, in numpy."""
    q = np.asarray(lut, dtype=np.int64)[I.astype(np.int64)]
    return (q[..., None] == np.arange(B)).astype(np.uint32)


def random_monotone_lut(rng, B):
    """Non-decreasing table over [0, 256) with values in [0, B): bin edges
    drawn at random, so some bins may be empty."""
    edges = np.sort(rng.integers(0, 257, size=B - 1))
    return np.searchsorted(edges, np.arange(256), side="right").astype(np.uint8)


def brute_eq1(I, B, oh=None):
    oh = onehot_numpy(I, B) if oh is None else oh
    H, W = I.shape
    out = np.zeros((H, W, B), dtype=np.uint32)
    for y in range(H):
        for x in range(W):
            out[y, x] = oh[: y + 1, : x + 1].sum(axis=(0, 1))
    return out


# ---------------------------------------------------------------------------
# the pin suite as a function, so the planted-mistake test can reuse it
# ---------------------------------------------------------------------------
def pin_failures(orc, quick=False):
    fails = []
    rng = np.random.default_rng(1234)

    # binning (Sec. 2.1 reading): bins are contiguous value intervals whose
    # sizes differ by at most one; powers of two take the top bits
    for B in (1, 2, 3, 5, 7, 16, 32, 100, 128, 255, 256):
        q = np.array([orc.Q(v, B) for v in range(256)])
        if q.min() != 0 or q.max() != B - 1 or np.any(np.diff(q) < 0) or np.any(np.diff(q) > 1):
            fails.append(f"Q-range-B{B}")
            continue
        sizes = np.bincount(q, minlength=B)
        if sizes.max() - sizes.min() > 1 or sizes.min() < 1:
            fails.append(f"Q-sizes-B{B}")
        if B & (B - 1) == 0:
            shift = 8 - (B.bit_length() - 1)
            if not np.array_equal(q, np.arange(256) >> shift):
                fails.append(f"Q-pow2-B{B}")
    g = json.loads((GOLDEN / "bin_edges_b3.json").read_text())
    q3 = np.array([orc.Q(v, 3) for v in range(256)])
    if list(np.flatnonzero(np.diff(q3)) + 1) != g["first_value_of_bin"][1:] or \
            list(np.bincount(q3)) != g["bin_sizes"]:
        fails.append("Q-golden-B3")

    # hand-worked fixture
    g = json.loads((GOLDEN / "hand_3x4_b2.json").read_text())
    I = np.array(g["frame_rows"], dtype=np.uint8)
    IH = orc.integral_histogram(I, g["B"])
    if not (np.array_equal(IH[..., 0], np.array(g["H_bin0_rows"])) and
            np.array_equal(IH[..., 1], np.array(g["H_bin1_rows"]))):
        fails.append("golden-eq1")
    if not np.array_equal(orc.region_histogram(IH, np.array(g["rects"])), np.array(g["hists"])):
        fails.append("golden-eq2")
    for r, h in zip(g["rects"], g["hists"]):
        if not np.array_equal(orc.rect_count(I, g["B"], r), np.array(h)):
            fails.append("golden-count")
            break

    # brute force of Eq. 1 on every tiny shape
    sides = range(1, 6) if quick else range(1, 10)
    for B in (1, 2, 3, 5, 7, 16, 32, 256):
        for H in sides:
            for W in sides:
                I = rng.integers(0, 256, size=(H, W), dtype=np.uint8)
                if not np.array_equal(orc.integral_histogram(I, B), brute_eq1(I, B)):
                    fails.append(f"brute-{H}x{W}-B{B}")
                    break
            else:
                continue
            break

    # invariants on ragged mid-size frames
    for (H, W, B) in ((37, 53, 3), (29, 64, 16), (17, 31, 256), (40, 40, 1), (8, 70, 128)):
        I = rng.integers(0, 256, size=(H, W), dtype=np.uint8)
        IH = orc.integral_histogram(I, B).astype(np.int64)
        xy = (np.arange(H)[:, None] + 1) * (np.arange(W)[None, :] + 1)
        if not np.array_equal(IH.sum(axis=2), xy):
            fails.append(f"inv-sum-{H}x{W}-B{B}")
        if not np.array_equal(IH[-1, -1], onehot_numpy(I, B).sum(axis=(0, 1))):
            fails.append(f"inv-last-{H}x{W}-B{B}")
        P = np.pad(IH, ((1, 0), (1, 0), (0, 0)))
        diff = P[1:, 1:] - P[:-1, 1:] - P[1:, :-1] + P[:-1, :-1]
        if not np.array_equal(diff, onehot_numpy(I, B)):
            fails.append(f"inv-diff-{H}x{W}-B{B}")
        if np.any(np.diff(IH, axis=0) < 0) or np.any(np.diff(IH, axis=1) < 0):
            fails.append(f"inv-monotone-{H}x{W}-B{B}")

    # closed forms
    H, W = 13, 21
    xy = (np.arange(H)[:, None] + 1) * (np.arange(W)[None, :] + 1)
    for c in (0, 1, 127, 128, 200, 255):
        for B in (1, 4, 7, 64, 256):
            IH = orc.integral_histogram(np.full((H, W), c, np.uint8), B)
            want = np.zeros((H, W, B), np.uint32)
            want[..., (c * B) // 256] = xy
            if not np.array_equal(IH, want):
                fails.append(f"closed-const-{c}-B{B}")
    I = rng.integers(0, 256, size=(H, W), dtype=np.uint8)
    if not np.array_equal(orc.integral_histogram(I, 1)[..., 0], xy):
        fails.append("closed-B1")
    B = 8
    colvals = rng.integers(0, 256, size=W, dtype=np.uint8)
    I = np.broadcast_to(colvals[None, :], (H, W)).copy()
    ohc = onehot_numpy(colvals[None, :], B)[0]                     # (W, B)
    want = (np.arange(H)[:, None, None] + 1) * np.cumsum(ohc, axis=0)[None]
    if not np.array_equal(orc.integral_histogram(I, B), want):
        fails.append("closed-column-only")
    rowvals = rng.integers(0, 256, size=H, dtype=np.uint8)
    I = np.broadcast_to(rowvals[:, None], (H, W)).copy()
    ohr = onehot_numpy(rowvals[:, None], B)[:, 0]                  # (H, B)
    want = (np.arange(W)[None, :, None] + 1) * np.cumsum(ohr, axis=0)[:, None, :]
    if not np.array_equal(orc.integral_histogram(I, B), want):
        fails.append("closed-row-only")

    # row-block continuation, row-by-definition and single entries agree
    # with the brute force on a ragged frame
    H, W, B = 23, 19, 5
    I = rng.integers(0, 256, size=(H, W), dtype=np.uint8)
    ref = brute_eq1(I, B)
    for rows in (1, 4, 7, 23):
        blocks = np.concatenate([blk for _, blk in orc.iter_row_blocks(I, B, rows)])
        if not np.array_equal(blocks, ref):
            fails.append(f"rows-{rows}")
    for y in (0, 1, 11, 22):
        if not np.array_equal(orc.row_by_definition(I, B, y), ref[y]):
            fails.append(f"rowdef-{y}")
    for (x, y, b) in ((0, 0, 0), (18, 22, 4), (5, 9, 2), (0, 22, 1), (18, 0, 3)):
        if orc.entry(I, B, x, y, b) != ref[y, x, b]:
            fails.append(f"entry-{x}-{y}-{b}")

    # bin-major storage (the paper's order): brute force per bin plane
    for (H, W, B) in ((1, 1, 1), (4, 7, 3), (9, 5, 16), (7, 8, 256)):
        I = rng.integers(0, 256, size=(H, W), dtype=np.uint8)
        if not np.array_equal(orc.integral_histogram_binmajor(I, B), np.moveaxis(brute_eq1(I, B), 2, 0)):
            fails.append(f"binmajor-brute-{H}x{W}-B{B}")

    # table binning (bins with arbitrary edges, and arbitrary tables): brute
    # force with the table's one-hot, the uniform table equals Q, invariants
    for (H, W, B) in ((1, 1, 1), (3, 7, 3), (9, 4, 16), (6, 6, 7), (5, 9, 256)):
        for monotone in (True, False):
            lut = random_monotone_lut(rng, B) if monotone else rng.integers(0, B, size=256).astype(np.uint8)
            I = rng.integers(0, 256, size=(H, W), dtype=np.uint8)
            got = orc.integral_histogram_lut(I, B, lut)
            if not np.array_equal(got, brute_eq1(I, B, onehot_lut_numpy(I, B, lut))):
                fails.append(f"lut-brute-{H}x{W}-B{B}-{monotone}")
    for B in (2, 5, 64):
        I = rng.integers(0, 256, size=(17, 23), dtype=np.uint8)
        qtable = ((np.arange(256) * B) >> 8).astype(np.uint8)
        if not np.array_equal(orc.integral_histogram_lut(I, B, qtable), brute_eq1(I, B)):
            fails.append(f"lut-uniform-B{B}")
    lut = np.zeros(256, np.uint8)
    lut[200:] = 3                                                  # bins 1, 2 empty
    I = rng.integers(0, 256, size=(11, 13), dtype=np.uint8)
    got = orc.integral_histogram_lut(I, 4, lut).astype(np.int64)
    xy = (np.arange(11)[:, None] + 1) * (np.arange(13)[None, :] + 1)
    if not (np.array_equal(got.sum(axis=2), xy) and not got[..., 1:3].any()
            and got[-1, -1, 3] == int((I >= 200).sum())):
        fails.append("lut-empty-bins")

    # Eq. 2 against direct counting in numpy and the area invariant
    for (H, W, B) in ((31, 47, 16), (9, 5, 3), (1, 1, 2), (1, 33, 7), (40, 1, 256)):
        I = rng.integers(0, 256, size=(H, W), dtype=np.uint8)
        IH = orc.integral_histogram(I, B)
        xs = np.sort(rng.integers(0, W, size=(60, 2)), axis=1)
        ys = np.sort(rng.integers(0, H, size=(60, 2)), axis=1)
        rects = np.stack([xs[:, 0], ys[:, 0], xs[:, 1], ys[:, 1]], axis=1)
        rects = np.concatenate([rects, [[0, 0, W - 1, H - 1], [W - 1, H - 1, W - 1, H - 1],
                                        [0, 0, 0, 0], [0, H - 1, W - 1, H - 1],
                                        [W - 1, 0, W - 1, H - 1]]]).astype(np.int32)
        got = orc.region_histogram(IH, rects)
        oh = onehot_numpy(I, B)
        for r, h in zip(rects, got):
            x0, y0, x1, y1 = r
            want = oh[y0:y1 + 1, x0:x1 + 1].sum(axis=(0, 1))
            if not np.array_equal(h, want):
                fails.append(f"eq2-{H}x{W}-B{B}")
                break
            if not np.array_equal(orc.rect_count(I, B, r), want):
                fails.append(f"count-{H}x{W}-B{B}")
                break
        area = (rects[:, 2] - rects[:, 0] + 1) * (rects[:, 3] - rects[:, 1] + 1)
        if not np.array_equal(got.sum(axis=1).astype(np.int64), area):
            fails.append(f"eq2-area-{H}x{W}-B{B}")
        if not np.array_equal(got[-5], IH[-1, -1]):
            fails.append(f"eq2-full-{H}x{W}-B{B}")
    return fails


def test_pins_hold(orc):
    assert pin_failures(orc) == []


def test_textbook_cumsum_full_frame(orc):
    """Eq. 1 is a 2-D inclusive prefix sum of the one-hot tensor; numpy's
    cumsum along rows then columns is an independent route to it."""
    rng = np.random.default_rng(7)
    I = rng.integers(0, 256, size=(480, 640), dtype=np.uint8)
    for B in (32, 3):
        want = np.cumsum(np.cumsum(onehot_numpy(I, B), axis=0, dtype=np.uint32), axis=1, dtype=np.uint32)
        assert np.array_equal(orc.integral_histogram(I, B), want)


def test_row_blocks_match_full_frame(orc):
    rng = np.random.default_rng(8)
    I = rng.integers(0, 256, size=(270, 481), dtype=np.uint8)
    full = orc.integral_histogram(I, 64)
    for y0, blk in orc.iter_row_blocks(I, 64, 100):
        assert np.array_equal(blk, full[y0:y0 + blk.shape[0]])


def test_rejects_bad_arguments(orc):
    I = np.zeros((4, 4), np.uint8)
    for B in (0, 257, -1):
        with pytest.raises(ValueError):
            orc.integral_histogram(I, B)
    IH = orc.integral_histogram(I, 4)
    for r in ([0, 0, 4, 0], [-1, 0, 1, 1], [2, 0, 1, 1], [0, 3, 0, 2], [0, 0, 0, 4]):
        with pytest.raises(ValueError):
            orc.region_histogram(IH, np.array([r]))


# Plausible mistakes, each planted into a copy of ih_oracle.c as a textual
# patch inside one function: (function, text as written, text with the mistake).
MISTAKES = {
    "rounding-binning": ("ihref_Q", "return (v * B) >> 8;", "return (v * B + 128u) >> 8;"),
    "corner-dropped": ("ihref_integral_histogram",
                       "+ at(out, W, B, x, y - 1, b)\n                           - at(out, W, B, x - 1, y - 1, b);",
                       "+ at(out, W, B, x, y - 1, b);"),
    "corner-sign": ("ihref_integral_histogram", "- at(out, W, B, x - 1, y - 1, b);",
                    "+ at(out, W, B, x - 1, y - 1, b);"),
    "first-column-pixel-lost": ("ihref_integral_histogram", "if (q == (uint32_t)b) h += 1u;",
                                "if (q == (uint32_t)b && x > 0) h += 1u;"),
    "query-corner-off-by-one": ("ihref_region_histogram",
                                "- at(Ht, W, B, x1, y0 - 1, b) + at(Ht, W, B, x0 - 1, y0 - 1, b);",
                                "- at(Ht, W, B, x1, y0, b) + at(Ht, W, B, x0 - 1, y0, b);"),
    "rows-corner-dropped": ("ihref_integral_rows",
                            "const uint32_t corner = (up && x > 0) ? up[(x - 1) * B + b] : 0u;",
                            "const uint32_t corner = 0u;"),
    "rowdef-row-left-out": ("ihref_row_by_definition", "for (int64_t yy = 0; yy <= y; ++yy)",
                            "for (int64_t yy = 0; yy < y; ++yy)"),
    "count-column-left-out": ("ihref_rect_count", "for (int64_t c = x0; c <= x1; ++c)",
                              "for (int64_t c = x0; c < x1; ++c)"),
    "table-neighbour-entry": ("ihref_integral_histogram_lut", "const uint32_t q = lut[I[y * W + x]];",
                              "const uint32_t q = lut[I[y * W + x] ^ 1u];"),
    "binmajor-row-dropped": ("ihref_integral_histogram_binmajor", "for (int64_t y = 1; y < H; ++y)",
                             "for (int64_t y = 2; y < H; ++y)"),
    "binmajor-run-not-reset": ("ihref_integral_histogram_binmajor",
                               "uint32_t run = 0;\n            for (int64_t x = 0; x < W; ++x) {",
                               "uint32_t run = y > 0 ? P[y * W - 1] : 0u;\n            for (int64_t x = 0; x < W; ++x) {"),
    "entry-column-left-out": ("ihref_entry", "for (int64_t c = 0; c <= x; ++c)", "for (int64_t c = 0; c < x; ++c)"),
    "table-corner-sign": ("ihref_integral_histogram_lut", "- at(out, W, B, x - 1, y - 1, b);",
                          "+ at(out, W, B, x - 1, y - 1, b);"),
}


def function_span(src: str, name: str):
    """[start, end) of the body of the C function `name` in src."""
    import re
    m = re.search(r"^[a-z_0-9 ]*\b" + name + r"\(", src, re.M)
    assert m, name
    end = src.index("\n}\n", m.start()) + 3
    return m.start(), end


def planted_source(name: str) -> str:
    func, old, new = MISTAKES[name]
    src = oracle.SRC.read_text()
    a, b = function_span(src, func)
    body = src[a:b]
    assert body.count(old) == 1, (name, body.count(old))
    return src[:a] + body.replace(old, new) + src[b:]


@pytest.mark.parametrize("name", sorted(MISTAKES))
def test_planted_mistakes_are_caught(tmp_path, name):
    """Each plausible mistake (a rounding binning, a dropped or sign-flipped
    corner term, a lost pixel, an off-by-one corner in Eq. 2, a dropped row or
    column, a wrong table entry), planted into a copy of the oracle, must fail
    at least one pin."""
    src = tmp_path / f"{name}.c"
    src.write_text(planted_source(name))
    lib = oracle.compile_oracle(tmp_path / f"{name}.so", source=src)
    fails = pin_failures(oracle.Oracle(lib), quick=True)
    assert fails, f"planted mistake {name} passed every pin"
