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
