"""GPU parity: the HIP path (through the C ABI) against the CPU oracle, bit
for bit.  Integer results, so the tolerance is zero everywhere."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ihb():
    from paper_1711_01919_amd import binding
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return binding


def gpu_ih(ihb, I, B):
    f = torch.from_numpy(np.ascontiguousarray(I)).cuda()
    out = ihb.compute(f, B)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def frames_of(kind, H, W, rng):
    if kind == "uniform":
        return rng.integers(0, 256, size=(H, W), dtype=np.uint8)
    if kind == "const":
        return np.full((H, W), 200, np.uint8)
    if kind == "checker":
        return (((np.arange(H)[:, None] + np.arange(W)[None, :]) % 2) * 255).astype(np.uint8)
    if kind == "gradient":
        return ((np.arange(H)[:, None] * 7 + np.arange(W)[None, :] * 3) % 256).astype(np.uint8)
    raise ValueError(kind)


SHAPES = [(1, 1), (1, 77), (93, 1), (17, 31), (64, 64), (65, 129), (479, 641), (480, 640)]
BINS = [1, 3, 16, 32, 64, 100, 128, 200, 256]


@pytest.mark.parametrize("H,W", SHAPES)
@pytest.mark.parametrize("B", BINS)
def test_uniform_frames(ihb, orc, H, W, B):
    rng = np.random.default_rng(H * 1000 + W * 7 + B)
    I = frames_of("uniform", H, W, rng)
    assert np.array_equal(gpu_ih(ihb, I, B), orc.integral_histogram(I, B)), (H, W, B)


@pytest.mark.parametrize("kind", ["const", "checker", "gradient"])
@pytest.mark.parametrize("B", [1, 2, 32, 64, 128, 256])
def test_structured_frames(ihb, orc, kind, B):
    I = frames_of(kind, 271, 333, None)
    assert np.array_equal(gpu_ih(ihb, I, B), orc.integral_histogram(I, B))


@pytest.mark.parametrize("H,W,B", [(1081, 1919, 64), (1080, 1920, 64), (720, 1280, 16), (240, 320, 128)])
def test_video_sizes(ihb, orc, H, W, B):
    rng = np.random.default_rng(11)
    I = frames_of("uniform", H, W, rng)
    assert np.array_equal(gpu_ih(ihb, I, B), orc.integral_histogram(I, B))


@pytest.mark.parametrize("H,W,B", [(2, 65536, 1), (3, 65536, 5), (2, 65537, 1), (3, 70001, 3), (1, 131072, 2)])
def test_wide_frames_left_carry_widths(ihb, orc, H, W, B):
    """Left carries are kept as uint16 up to 65536 columns (the largest, at the
    last segment of a B=1 frame, is 65536 - TX) and as uint32 beyond: every
    single-frame form equals the oracle on both sides of the boundary."""
    rng = np.random.default_rng(H * 7 + W + B)
    I = rng.integers(0, 256, size=(H, W), dtype=np.uint8)
    if B == 1:
        I[:] = 200                          # every pixel in the one bin: carries as large as they get
    want = orc.integral_histogram(I, B)
    f = torch.from_numpy(I).cuda()
    assert np.array_equal(ihb.compute(f, B).cpu().numpy(), want)
    bm = ihb.compute_binmajor(f, B)
    assert np.array_equal(bm.permute(1, 2, 0).contiguous().cpu().numpy(), want)
    lut = ((np.arange(256) * B) >> 8).astype(np.uint8)
    assert np.array_equal(ihb.compute_lut(f, B, lut).cpu().numpy(), want)


@pytest.mark.parametrize("H,W,B", [(65536, 8, 1), (65537, 8, 1), (70001, 24, 3)])
def test_tall_frames_column_carry_widths(ihb, orc, H, W, B):
    """Column carries are kept as uint16 up to 65536 rows (the largest top
    carry, above the last band of a B=1 frame, is below 65536) and as uint32
    beyond: the single-frame forms and a reduce-then-scan plan equal the
    oracle on both sides of the boundary."""
    rng = np.random.default_rng(H + W * 13 + B)
    I = rng.integers(0, 256, size=(H, W), dtype=np.uint8)
    if B == 1:
        I[:] = 77                           # every pixel in the one bin: carries as large as they get
    want = orc.integral_histogram(I, B)
    f = torch.from_numpy(I).cuda()
    assert np.array_equal(ihb.compute(f, B).cpu().numpy(), want)
    bm = ihb.compute_binmajor(f, B)
    assert np.array_equal(bm.permute(1, 2, 0).contiguous().cpu().numpy(), want)
    out = torch.empty((H, W, B), dtype=torch.uint32, device="cuda")
    plan = ihb.BatchPlan([f], [out], [B], tile=(32, 64), carry_bands=0)
    plan.launch()
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), want)
    plan.close()


def test_unaligned_frame_and_output(ihb, orc):
    """Frame and output views that start off a 16-byte boundary take the
    guarded kernel and must give the same bits."""
    rng = np.random.default_rng(12)
    H, W, B = 130, 256, 32
    I = frames_of("uniform", H, W, rng)
    buf = torch.zeros(H * W + 3, dtype=torch.uint8, device="cuda")
    buf[3:] = torch.from_numpy(I.reshape(-1)).cuda()
    f = buf[3:].view(H, W)
    obuf = torch.zeros(H * W * B + 1, dtype=torch.uint32, device="cuda")
    out = obuf[1:].view(H, W, B)
    ihb.compute(f, B, out=out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), orc.integral_histogram(I, B))
    assert int(obuf[0].item()) == 0


def test_plain_frame_config(ihb, orc):
    """640x480, B=32 (seed 0) with its 1000 rectangle queries."""
    from paper_1711_01919_amd import synth
    I, B, rects = synth.plain_frame()
    f = torch.from_numpy(I).cuda()
    ih = ihb.compute(f, B)
    hists = ihb.query(ih, rects)
    rd = torch.from_numpy(rects).cuda()
    hists_d = ihb.query_device(ih, rd)
    torch.cuda.synchronize()
    ref = orc.integral_histogram(I, B)
    assert np.array_equal(ih.cpu().numpy(), ref)
    want = orc.region_histogram(ref, rects)
    assert np.array_equal(hists.cpu().numpy(), want)
    assert np.array_equal(hists_d.cpu().numpy(), want)


def test_query_degenerate_and_bad_rects(ihb, orc):
    rng = np.random.default_rng(13)
    H, W, B = 57, 91, 7
    I = frames_of("uniform", H, W, rng)
    ref = orc.integral_histogram(I, B)
    rects = np.array([[0, 0, W - 1, H - 1], [0, 0, 0, 0], [W - 1, H - 1, W - 1, H - 1], [3, 0, 3, H - 1],
                      [0, 5, W - 1, 5], [10, 20, 40, 50]], np.int32)
    ih = ihb.compute(torch.from_numpy(I).cuda(), B)
    got = ihb.query(ih, rects)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), orc.region_histogram(ref, rects))
    bad = np.array([[0, 0, W, 0], [-1, 0, 0, 0], [5, 0, 4, 0], [0, 0, 0, H]], np.int32)
    mixed = np.concatenate([rects[:2], bad, rects[2:]])
    cnt = torch.zeros(1, dtype=torch.uint32, device="cuda")
    gotd = ihb.query_device(ih, torch.from_numpy(mixed).cuda(), bad_count=cnt)
    torch.cuda.synchronize()
    gotd = gotd.cpu().numpy()
    assert int(cnt.item()) == 4
    assert np.array_equal(gotd[2:6], np.zeros((4, B), np.uint32))
    assert np.array_equal(np.concatenate([gotd[:2], gotd[6:]]), orc.region_histogram(ref, rects))
    with pytest.raises(ihb.IHError):
        ihb.query(ih, bad[:1])


def test_repeat_calls_identical(ihb, orc):
    """Same input, many calls and two streams: identical bits each time."""
    rng = np.random.default_rng(14)
    I = frames_of("uniform", 300, 500, rng)
    f = torch.from_numpy(I).cuda()
    ref = orc.integral_histogram(I, 64)
    s2 = torch.cuda.Stream()
    outs = []
    for k in range(6):
        st = s2 if k % 2 else torch.cuda.current_stream()
        with torch.cuda.stream(st):
            outs.append(ihb.compute(f, 64, stream=st))
    torch.cuda.synchronize()
    for o in outs:
        assert np.array_equal(o.cpu().numpy(), ref)


def test_scratch_reuse_and_tables_in_stream_order(ihb, orc):
    """One stream, no synchronisation between calls: frames whose carries need
    more and then less scratch (the stream's buffer is replaced once earlier
    work has drained), and table-binned frames with different tables back to
    back (each call's table is stored in stream order).  Every output equals
    the oracle."""
    rng = np.random.default_rng(15)
    shapes = [(64, 96, 16), (700, 900, 64), (33, 47, 7), (480, 640, 32), (65, 129, 256), (300, 257, 100)]
    frames, luts, refs = [], [], []
    for k, (H, W, B) in enumerate(shapes):
        I = rng.integers(0, 256, size=(H, W), dtype=np.uint8)
        lut = None
        if k % 2:
            edges = np.sort(rng.integers(0, 257, size=B - 1))
            lut = np.searchsorted(edges, np.arange(256), side="right").astype(np.uint8)
        frames.append(I)
        luts.append(lut)
        refs.append(orc.integral_histogram(I, B) if lut is None else orc.integral_histogram_lut(I, B, lut))
    dev = [torch.from_numpy(I).cuda() for I in frames]
    outs = [torch.empty((H, W, B), dtype=torch.uint32, device="cuda") for H, W, B in shapes]
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    for rep in range(2):
        for o in outs:
            o.fill_(0xA5A5A5A5)
        torch.cuda.synchronize()
        for f, o, (H, W, B), lut in zip(dev, outs, shapes, luts):
            if lut is None:
                ihb.compute(f, B, out=o, stream=s)
            else:
                ihb.compute_lut(f, B, lut, out=o, stream=s)
        s.synchronize()
        for k, o in enumerate(outs):
            assert np.array_equal(o.cpu().numpy(), refs[k]), (rep, k, shapes[k])


def test_errors_leave_output_untouched(ihb):
    f = torch.zeros((8, 8), dtype=torch.uint8, device="cuda")
    out = torch.full((8 * 8 * 4,), 0xDEADBEEF, dtype=torch.uint32, device="cuda").view(8, 8, 4)
    for B in (0, 257):
        st = ihb.compute_raw(f.data_ptr(), 8, 8, B, out.data_ptr())
        assert st == 1
    torch.cuda.synchronize()
    assert bool((out == 0xDEADBEEF).all())
