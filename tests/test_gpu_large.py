"""Full-size parity on frames whose tensors do not fit a host-side oracle run
at once: the 8192x8192 mixture frame with B=128 (2^33 entries, 34 GB) and an
8192x8192 frame with B=64 (exactly 2^32 entries, the 32-bit index boundary).

Every entry is compared with the oracle: its recursion runs block of rows
after block of rows (integral_rows, carrying the last row), and each block
of the device tensor is downloaded when its turn comes.  On top of that,
rows summed directly from Eq. 1 (row_by_definition), rectangles counted
pixel by pixel, and properties that hold at any size: the bins of each pixel
sum to (x+1)(y+1), and the last entry is the frame's histogram.  Tolerance 0
everywhere."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ihb():
    from paper_1711_01919_amd import binding
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return binding


def bin_sum_invariant(ih, H, W, chunk_rows=64):
    """sum_b H(x,y,b) == (x+1)(y+1) for every pixel, computed on the device."""
    xs = torch.arange(1, W + 1, device="cuda", dtype=torch.int64)
    for y0 in range(0, H, chunk_rows):
        y1 = min(H, y0 + chunk_rows)
        # every count here is below 2^31, so the int32 view reads it unchanged
        s = ih[y0:y1].view(torch.int32).sum(dim=2, dtype=torch.int64)
        want = torch.arange(y0 + 1, y1 + 1, device="cuda", dtype=torch.int64)[:, None] * xs[None, :]
        if not bool(torch.equal(s, want)):
            bad = (s != want).nonzero()[0].tolist()
            return False, (y0 + bad[0], bad[1])
    return True, None


def check_rows(orc, ih, I, B, rows):
    for y in rows:
        got = ih[y].cpu().numpy()
        want = orc.row_by_definition(I, B, y)
        assert np.array_equal(got, want), f"row {y} differs"


@pytest.mark.timeout(600)
def test_mixture_frame_8192_b128(ihb, orc, rows_compare):
    from paper_1711_01919_amd import synth
    I, B, rects = synth.mixture_frame()
    H, W = I.shape
    f = torch.from_numpy(I).cuda()
    ih = ihb.compute(f, B)
    torch.cuda.synchronize()
    diff = rows_compare(orc, ih, I, B)
    assert diff is None, f"first difference (y, x, b, got, want) = {diff}"
    ok, where = bin_sum_invariant(ih, H, W)
    assert ok, f"bin-sum invariant fails at (y, x) = {where}"
    rng = np.random.default_rng(5)
    rows = [0, 1, 255, 256, 4095, 4096, H - 1] + [int(r) for r in rng.integers(0, H, 3)]
    check_rows(orc, ih, I, B, rows)
    assert np.array_equal(ih[H - 1, W - 1].cpu().numpy(), np.bincount(((I.astype(np.int64) * B) >> 8).ravel(),
                                                                        minlength=B).astype(np.uint32))
    # all 1e6 rectangles on the device; area invariant for all, direct counts for a sample
    rd = torch.from_numpy(rects).cuda()
    bad = torch.zeros(1, dtype=torch.uint32, device="cuda")
    hists = ihb.query_device(ih, rd, bad_count=bad)
    torch.cuda.synchronize()
    assert int(bad.item()) == 0
    area = ((rd[:, 2] - rd[:, 0] + 1).to(torch.int64) * (rd[:, 3] - rd[:, 1] + 1).to(torch.int64))
    hs = hists.view(torch.int32).sum(dim=1, dtype=torch.int64)
    assert bool(torch.equal(hs, area))
    small = np.argsort((rects[:, 2] - rects[:, 0] + 1) * (rects[:, 3] - rects[:, 1] + 1))
    sample = np.concatenate([small[:40], rng.integers(0, len(rects), 20)])
    got = hists.cpu().numpy()
    for r in sample:
        assert np.array_equal(got[r], orc.rect_count(I, B, rects[r])), int(r)
    del ih, hists
    torch.cuda.empty_cache()


@pytest.mark.timeout(600)
def test_index_boundary_2_32_entries(ihb, orc, rows_compare):
    """8192 x 8192 x 64 = 2^32 entries: offsets past 2^32 elements' worth of
    bytes and the very last entry must land where they belong."""
    rng = np.random.default_rng(9)
    H = W = 8192
    B = 64
    I = rng.integers(0, 256, size=(H, W), dtype=np.uint8)
    f = torch.from_numpy(I).cuda()
    ih = ihb.compute(f, B)
    torch.cuda.synchronize()
    diff = rows_compare(orc, ih, I, B)
    assert diff is None, f"first difference (y, x, b, got, want) = {diff}"
    ok, where = bin_sum_invariant(ih, H, W)
    assert ok, f"bin-sum invariant fails at (y, x) = {where}"
    check_rows(orc, ih, I, B, [0, 4095, 4096, 8190, H - 1])
    del ih
    torch.cuda.empty_cache()


@pytest.mark.parametrize("B", [16, 64, 128])
def test_single_4k_frames(ihb, orc, rows_compare, B):
    """One 3840x2160 frame through ih_compute (non-temporal stores; 64-column
    tiles, 128-column at B=64); every entry against the oracle."""
    rng = np.random.default_rng(20 + B)
    I = rng.integers(0, 256, size=(2160, 3840), dtype=np.uint8)
    out = ihb.compute(torch.from_numpy(I).cuda(), B)
    torch.cuda.synchronize()
    diff = rows_compare(orc, out, I, B)
    assert diff is None, diff
    del out
    torch.cuda.empty_cache()


def test_batched_large_frames(ihb, orc, rows_compare):
    """Two 3840x2160 frames of different bin counts in one batched plan, with
    the autotuner on; every entry against the oracle."""
    rng = np.random.default_rng(10)
    frames = [rng.integers(0, 256, size=(2160, 3840), dtype=np.uint8) for _ in range(2)]
    bins = [128, 16]
    d = [torch.from_numpy(x).cuda() for x in frames]
    outs = [torch.empty((2160, 3840, b), dtype=torch.uint32, device="cuda") for b in bins]
    plan = ihb.BatchPlan(d, outs, bins, autotune=True)
    plan.launch()
    torch.cuda.synchronize()
    for k in range(2):
        diff = rows_compare(orc, outs[k], frames[k], bins[k])
        assert diff is None, (k, diff)
        ok, where = bin_sum_invariant(outs[k], 2160, 3840)
        assert ok, (k, where)
    plan.close()
