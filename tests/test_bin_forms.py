"""CPU checks of two pieces of integer arithmetic in the count kernels: a
shortcut for the uniform binning Q(v) = floor(v B / 256) (Sec. 2.1, Eq. 1;
the reading of Q for uint8 values), and the layout of their LDS counters.

  - For B = 2^k with k >= 1 the counting loops take the bin of byte c of a
    loaded 32-bit word with one shift and mask, (w >> (8 c + 8 - k)) & (B - 1).
    It must equal floor(v B / 256) for every value in every byte position,
    whatever the other three bytes hold, and its shift must stay below 32.
  - A tile's column counters are 32-bit words where TX (B + 1) <= 64 * 65,
    else two 16-bit halves per word, with one pad word per column.  A model
    of that layout, incremented through the word index and shift the count
    blocks use and read back the way they read it, must give each column's
    count of each bin, also at the largest column count (65535 rows), with
    no word overflowing.

No kernel is launched."""
import numpy as np
import pytest

WIDE_COL_WORDS = 64 * 65


@pytest.mark.parametrize("k", range(1, 9))
def test_power_of_two_bins_are_one_field_extract(k):
    B = 1 << k
    bs = 8 - k
    v = np.arange(256, dtype=np.uint64)
    want = (v * B) >> 8
    rng = np.random.default_rng(k)
    for c in range(4):
        assert 8 * c + bs <= 31
        # the value in byte c, random values in the other three bytes
        other = rng.integers(0, 2**32, size=256, dtype=np.uint64) & ~np.uint64(0xFF << (8 * c))
        w = other | (v << np.uint64(8 * c))
        got = (w >> np.uint64(8 * c + bs)) & np.uint64(B - 1)
        assert np.array_equal(got, want), (B, c)


def test_bins_other_than_powers_of_two_keep_the_product():
    # B = 1 and the B that are not powers of two take floor(v B / 256) as written:
    # the shift form would need a shift of 8 (B = 1) or has no mask form.
    for B in range(1, 257):
        if B >= 2 and B & (B - 1) == 0:
            continue
        v = np.arange(256)
        q = (v * B) >> 8
        assert q.min() == 0 and q.max() == B - 1 if B > 1 else q.max() == 0
        # every bin is a run of consecutive values, sizes differing by at most one
        sizes = np.bincount(q, minlength=B)
        assert sizes.sum() == 256 and sizes.max() - sizes.min() <= 1


@pytest.mark.parametrize("TX,B", [(32, 16), (32, 64), (32, 128), (32, 200), (32, 256), (64, 32), (64, 64),
                                  (64, 100), (64, 128), (128, 64)])
def test_counter_forms_count_every_bin(TX, B):
    # a model of one tile's LDS counters: word x * cw + (b >> sh), increment
    # 1 << ((b & sh) * 16); reading back a counter gives the column's count
    wide = TX * (B + 1) <= WIDE_COL_WORDS
    sh = 0 if wide else 1
    cw = B + 1 if wide else (B + 1) // 2 + 1
    rng = np.random.default_rng(TX * 1000 + B)
    rows = 65535 if TX == 32 and B == 16 else 777        # one case at the largest column count
    bins = (rng.integers(0, 256, size=(rows, TX)) * B) >> 8
    bins[:, 0] = B - 1                                     # a column with every pixel in the last bin
    words = np.zeros(TX * cw, dtype=np.uint64)
    x = np.broadcast_to(np.arange(TX), bins.shape).ravel()
    b = bins.ravel()
    np.add.at(words, x * cw + (b >> sh), np.left_shift(1, (b & sh) * 16).astype(np.uint64))
    assert words.max() < 2**32                             # no word overflows
    xs, bs_ = np.meshgrid(np.arange(TX), np.arange(B), indexing="ij")
    w = words[xs * cw + (bs_ >> sh)]
    got = w if wide else (w >> ((bs_ & 1) * 16).astype(np.uint64)) & np.uint64(0xFFFF)
    want = np.stack([np.bincount(bins[:, c], minlength=B) for c in range(TX)])
    assert np.array_equal(got, want)
    # a column's words end before the next column's: one pad word each
    assert ((B - 1) >> sh) < cw - 1
