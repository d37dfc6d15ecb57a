"""The bin-major layout (b x h x w, the paper's own, Sec. 3.1): every bin is a
contiguous H x W plane.  Bit-exact against the oracle's Algorithm 1 in the
paper's order (tolerance 0), and the same numbers as ih_compute's H x W x B
result with the axes moved."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ihb():
    from paper_1711_01919_amd import binding
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return binding


@pytest.mark.parametrize("B", [1, 3, 16, 32, 48, 64, 128, 256])
@pytest.mark.parametrize("shape", [(1, 1), (17, 31), (65, 129), (97, 203), (480, 640)])
def test_binmajor_equals_oracle(ihb, orc, B, shape):
    H, W = shape
    rng = np.random.default_rng(B * 131 + H * 7 + W)
    I = rng.integers(0, 256, size=(H, W), dtype=np.uint8)
    out = ihb.compute_binmajor(torch.from_numpy(I).cuda(), B)
    assert tuple(out.shape) == (B, H, W)
    assert np.array_equal(out.cpu().numpy(), orc.integral_histogram_binmajor(I, B))


def test_binmajor_is_hwb_with_axes_moved(ihb):
    rng = np.random.default_rng(60)
    for (H, W, B) in ((1080, 1920, 64), (300, 257, 100)):
        f = torch.from_numpy(rng.integers(0, 256, size=(H, W), dtype=np.uint8)).cuda()
        a = ihb.compute_binmajor(f, B)
        b = ihb.compute(f, B)
        torch.cuda.synchronize()
        assert bool(torch.equal(a.view(torch.int32), b.view(torch.int32).permute(2, 0, 1).contiguous()))


def random_rects(rng, H, W, n):
    xs = np.sort(rng.integers(0, W, size=(n, 2)), axis=1)
    ys = np.sort(rng.integers(0, H, size=(n, 2)), axis=1)
    edge = [[0, 0, W - 1, H - 1], [0, 0, 0, 0], [W - 1, H - 1, W - 1, H - 1], [W - 1, 0, W - 1, H - 1],
            [0, H - 1, W - 1, H - 1], [0, 0, 0, H - 1]]
    return np.concatenate([np.stack([xs[:, 0], ys[:, 0], xs[:, 1], ys[:, 1]], axis=1), edge]).astype(np.int32)


@pytest.mark.parametrize("B", [1, 7, 32, 64, 100, 256])
@pytest.mark.parametrize("shape", [(1, 1), (97, 203), (130, 67)])
def test_binmajor_query_equals_oracle(ihb, orc, B, shape):
    """Eq. 2 on the bin-major tensor: the oracle's four-corner query on its own
    integral histogram, for random, whole-frame, single-pixel and edge
    rectangles; B below and above one wave of bins."""
    H, W = shape
    rng = np.random.default_rng(700 + B + H)
    I = rng.integers(0, 256, size=(H, W), dtype=np.uint8)
    rects = random_rects(rng, H, W, 300)
    bm = ihb.compute_binmajor(torch.from_numpy(I).cuda(), B)
    got = ihb.query_binmajor(bm, rects)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), orc.region_histogram(orc.integral_histogram(I, B), rects))


def test_binmajor_query_device_counts_bad_rects(ihb, orc):
    rng = np.random.default_rng(71)
    H, W, B = 57, 91, 7
    I = rng.integers(0, 256, size=(H, W), dtype=np.uint8)
    good = random_rects(rng, H, W, 20)
    bad = np.array([[0, 0, W, 0], [-1, 0, 0, 0], [5, 0, 4, 0], [0, 0, 0, H]], np.int32)
    mixed = np.concatenate([good[:3], bad, good[3:]])
    bm = ihb.compute_binmajor(torch.from_numpy(I).cuda(), B)
    cnt = torch.zeros(1, dtype=torch.uint32, device="cuda")
    got = ihb.query_binmajor_device(bm, torch.from_numpy(mixed).cuda(), bad_count=cnt)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    assert int(cnt.item()) == 4
    assert np.array_equal(got[3:7], np.zeros((4, B), np.uint32))
    ref = orc.region_histogram(orc.integral_histogram(I, B), good)
    assert np.array_equal(np.concatenate([got[:3], got[7:]]), ref)
    with pytest.raises(ihb.IHError):
        ihb.query_binmajor(bm, bad[:1])


def test_binmajor_query_matches_hwb_query_at_1080p(ihb):
    """At the bench frame size the two layouts answer the same 2000 rectangles
    identically (the H x W x B query is itself pinned against the oracle)."""
    rng = np.random.default_rng(72)
    H, W, B = 1080, 1920, 64
    f = torch.from_numpy(rng.integers(0, 256, size=(H, W), dtype=np.uint8)).cuda()
    rects = random_rects(rng, H, W, 2000)
    a = ihb.query_binmajor(ihb.compute_binmajor(f, B), rects)
    b = ihb.query(ihb.compute(f, B), rects)
    torch.cuda.synchronize()
    assert bool(torch.equal(a.view(torch.int32), b.view(torch.int32)))
