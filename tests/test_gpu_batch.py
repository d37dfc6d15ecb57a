"""Batched form: one launch per phase over many frames, replayed from a
hipGraph.  Every frame must equal the oracle bit for bit, for every tile the
autotuner may pick, across graph replays, and equal the single-frame path."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ihb():
    from paper_1711_01919_amd import binding
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return binding


def to_dev(frames, bins):
    fr = [torch.from_numpy(np.ascontiguousarray(f)).cuda() for f in frames]
    outs = [torch.full((f.shape[0], f.shape[1], b), 0xA5A5A5A5, dtype=torch.uint32, device="cuda")
            for f, b in zip(frames, bins)]
    return fr, outs


def test_uneven_batch_small(ihb, orc):
    """256 frames of five resolutions (scaled down 8x) and four bin counts."""
    from paper_1711_01919_amd import synth
    ub = synth.uneven_batch(scale=8)
    fr, outs = to_dev(ub.frames, ub.bins)
    plan = ihb.BatchPlan(fr, outs, ub.bins)
    info = plan.info()
    assert info["frames"] == 256 and info["graph"]
    plan.launch()
    torch.cuda.synchronize()
    for k, (f, b) in enumerate(zip(ub.frames, ub.bins)):
        assert np.array_equal(outs[k].cpu().numpy(), orc.integral_histogram(f, b)), k
    plan.close()


CANDIDATES = [(tx, ty, nt) for tx in (32, 64, 128) for ty in (16, 32, 64, 128, 256) for nt in (0, 1)]


@pytest.mark.parametrize("tx,ty,nt", CANDIDATES)
def test_every_tile_candidate(ihb, orc, tx, ty, nt):
    """Each tile shape and store flavour the autotuner can choose."""
    rng = np.random.default_rng(tx * 1000 + ty + nt)
    shapes = [(300, 257, 64), (128, 640, 32), (97, 130, 128), (64, 192, 16), (50, 70, 3), (1, 64, 7)]
    if tx == 128:                                       # B = 64 only: whole, ragged and narrow frames
        shapes = [(300, 257, 64), (33, 384, 64), (17, 130, 64), (1, 64, 64), (5, 1, 64)]
    if tx == 32:
        shapes.append((70, 96, 256))
    frames = [rng.integers(0, 256, size=(h, w), dtype=np.uint8) for h, w, _ in shapes]
    bins = [b for _, _, b in shapes]
    fr, outs = to_dev(frames, bins)
    plan = ihb.BatchPlan(fr, outs, bins, tile=(tx, ty), nontemporal=nt)
    for k in range(len(frames)):
        assert plan.frame_tile(k) == (tx, ty, bool(nt))
    plan.launch()
    torch.cuda.synchronize()
    for k, (f, b) in enumerate(zip(frames, bins)):
        assert np.array_equal(outs[k].cpu().numpy(), orc.integral_histogram(f, b)), (k, f.shape, b)
    plan.close()


FUSED = [(tx, ty, k) for tx in (32, 64, 128) for ty in (8, 16, 64) for k in (1, 2, 3, 16)]


@pytest.mark.parametrize("tx,ty,k", FUSED)
def test_fused_carry_schedule(ihb, orc, tx, ty, k):
    """The fused carry schedule (the count launch scans the carries itself:
    the last block of a tile column and of a carry band do the scans) on
    ragged frames of several bin counts, K tile bands per carry band clamped
    to each frame's band count, launched three times so that the arrival
    counters are seen to reset."""
    rng = np.random.default_rng(tx * 10007 + ty * 101 + k)
    shapes = [(300, 257, 64), (128, 640, 32), (97, 130, 128), (64, 192, 16), (50, 70, 3), (1, 64, 7), (17, 1, 5)]
    if tx == 128:
        shapes = [(300, 257, 64), (33, 384, 64), (17, 130, 64), (1, 64, 64), (5, 1, 64)]
    if tx == 32:
        shapes.append((70, 96, 256))
    frames = [rng.integers(0, 256, size=(h, w), dtype=np.uint8) for h, w, _ in shapes]
    bins = [b for _, _, b in shapes]
    refs = [orc.integral_histogram(f, b) for f, b in zip(frames, bins)]
    fr, outs = to_dev(frames, bins)
    plan = ihb.BatchPlan(fr, outs, bins, tile=(tx, ty), carry_bands=k)
    info = plan.info()
    for j, (h, w, b) in enumerate(shapes):
        sc = plan.frame_schedule(j)
        assert sc["tile"] == (tx, ty) and sc["carry_bands"] == min(k, -(-h // ty)), (j, sc)
    # the scans ran in the count launch: no scan launches at all
    assert info["kernel_launches"] == len({tx}) + info["tile_launches"], info
    for rep in range(3):
        for o in outs:
            o.fill_(0xA5A5A5A5)
        torch.cuda.synchronize()
        plan.launch()
        torch.cuda.synchronize()
        for j in range(len(frames)):
            assert np.array_equal(outs[j].cpu().numpy(), refs[j]), (rep, j, shapes[j])
    plan.close()


PREFIX = [(tx, ty) for tx in (32, 64, 128) for ty in (1, 8, 16, 64)]


@pytest.mark.parametrize("tx,ty", PREFIX)
def test_prefix_count_schedule(ihb, orc, tx, ty):
    """The prefix-count schedule (each count block counts every row above its
    band; the tile pass adds up the tile-column totals to its left; no scan
    launch) on ragged frames of several bin counts, launched twice."""
    rng = np.random.default_rng(tx * 7919 + ty)
    shapes = [(300, 257, 64), (128, 640, 32), (97, 130, 128), (64, 192, 16), (50, 70, 3), (1, 64, 7), (17, 1, 5)]
    if tx == 128:
        shapes = [(300, 257, 64), (33, 384, 64), (17, 130, 64), (1, 64, 64), (5, 1, 64)]
    if tx == 32:
        shapes.append((70, 96, 256))
    frames = [rng.integers(0, 256, size=(h, w), dtype=np.uint8) for h, w, _ in shapes]
    bins = [b for _, _, b in shapes]
    refs = [orc.integral_histogram(f, b) for f, b in zip(frames, bins)]
    fr, outs = to_dev(frames, bins)
    plan = ihb.BatchPlan(fr, outs, bins, tile=(tx, ty), carry_bands=-2)
    info = plan.info()
    for j in range(len(shapes)):
        sc = plan.frame_schedule(j)
        assert sc["tile"] == (tx, ty) and sc["carry_bands"] == -2, (j, sc)
    assert info["kernel_launches"] == 1 + info["tile_launches"], info       # no scan launches
    for rep in range(2):
        for o in outs:
            o.fill_(0xA5A5A5A5)
        torch.cuda.synchronize()
        plan.launch()
        torch.cuda.synchronize()
        for j in range(len(frames)):
            assert np.array_equal(outs[j].cpu().numpy(), refs[j]), (rep, j, shapes[j])
    plan.close()


def test_three_schedules_in_one_launch(ihb, orc):
    """In one plan a frame too tall for prefix counts (more than 65536 rows)
    keeps reduce-then-scan while the others take prefix counts, all in the
    same count and tile launches; then the same frames under the fused
    schedule.  Every frame equals the oracle."""
    rng = np.random.default_rng(80)
    shapes = [(70000, 3, 4), (200, 300, 32), (64, 64, 16), (480, 640, 32)]
    frames = [rng.integers(0, 256, size=(h, w), dtype=np.uint8) for h, w, _ in shapes]
    bins = [b for _, _, b in shapes]
    fr, outs = to_dev(frames, bins)
    plans = [ihb.BatchPlan(fr, outs, bins, tile=(32, 8), carry_bands=-2),
             ihb.BatchPlan(fr, outs, bins, tile=(32, 8), carry_bands=3)]
    assert plans[0].frame_schedule(0)["carry_bands"] == 0
    assert all(plans[0].frame_schedule(j)["carry_bands"] == -2 for j in (1, 2, 3))
    refs = [orc.integral_histogram(f, b) for f, b in zip(frames, bins)]
    for plan in plans:
        for o in outs:
            o.fill_(0xA5A5A5A5)
        plan.launch()
        torch.cuda.synchronize()
        for j in range(len(frames)):
            assert np.array_equal(outs[j].cpu().numpy(), refs[j]), j
        plan.close()


@pytest.mark.parametrize("branches", [2, 3, 4])
def test_tile_branches(ihb, orc, branches):
    """Tile-pass launches of several kernel variants spread over graph
    branches: graph launches, ungraphed launches and profiled launches (one
    graph per phase) all equal the oracle, launch after launch, with eager
    work on the stream between them."""
    rng = np.random.default_rng(90 + branches)
    shapes = [(300, 257, 64), (128, 640, 32), (97, 130, 128), (64, 192, 16), (50, 70, 3), (70, 96, 256),
              (240, 320, 64), (33, 384, 16)]
    frames = [rng.integers(0, 256, size=(h, w), dtype=np.uint8) for h, w, _ in shapes]
    bins = [b for _, _, b in shapes]
    refs = [orc.integral_histogram(f, b) for f, b in zip(frames, bins)]
    fr, outs = to_dev(frames, bins)
    for use_graph in (True, False):
        plan = ihb.BatchPlan(fr, outs, bins, use_graph=use_graph, tile_branches=branches)
        assert plan.info()["tile_launches"] >= 3
        for rep in range(3):
            for o in outs:
                o.fill_(0xA5A5A5A5)
            if rep == 2:
                ihb.profile_enable(True)
            plan.launch()
            if rep == 2:
                ph = ihb.profile_read()
                ihb.profile_enable(False)
                assert ph["tile_ms"] > 0
            torch.cuda.synchronize()
            for j in range(len(frames)):
                assert np.array_equal(outs[j].cpu().numpy(), refs[j]), (use_graph, rep, j, shapes[j])
        plan.close()


def test_fused_and_reduce_then_scan_frames_in_one_launch(ihb, orc):
    """A frame too wide for the fused schedule's arrival counters keeps
    reduce-then-scan while the others take the fused one; all share the count
    and tile launches."""
    rng = np.random.default_rng(78)
    shapes = [(3, 140000, 4), (200, 300, 32), (64, 64, 16)]
    frames = [rng.integers(0, 256, size=(h, w), dtype=np.uint8) for h, w, _ in shapes]
    bins = [b for _, _, b in shapes]
    fr, outs = to_dev(frames, bins)
    plan = ihb.BatchPlan(fr, outs, bins, tile=(32, 8), carry_bands=4)
    assert plan.frame_schedule(0)["carry_bands"] == 0
    assert plan.frame_schedule(1)["carry_bands"] == 4 and plan.frame_schedule(2)["carry_bands"] == 4
    for rep in range(2):
        plan.launch()
        torch.cuda.synchronize()
        for j, (f, b) in enumerate(zip(frames, bins)):
            assert np.array_equal(outs[j].cpu().numpy(), orc.integral_histogram(f, b)), (rep, j)
    plan.close()


def test_fused_schedule_pipelined_and_profiled(ihb, orc):
    rng = np.random.default_rng(79)
    shapes = [(240, 320, 64), (97, 203, 32), (360, 640, 16), (61, 64, 128), (480, 640, 64)]
    frames = [rng.integers(0, 256, size=(h, w), dtype=np.uint8) for h, w, _ in shapes]
    bins = [b for _, _, b in shapes]
    refs = [orc.integral_histogram(f, b) for f, b in zip(frames, bins)]
    fr, outs = to_dev(frames, bins)
    for group_bytes, use_graph in ((0, False), (1 << 20, True), (1 << 20, False)):
        plan = ihb.BatchPlan(fr, outs, bins, use_graph=use_graph, group_bytes=group_bytes, carry_bands=2)
        for rep in range(2):
            for o in outs:
                o.zero_()
            torch.cuda.synchronize()
            if rep == 1:
                ihb.profile_enable(True)
            plan.launch()
            if rep == 1:
                ph = ihb.profile_read()
                ihb.profile_enable(False)
                assert ph["frames"] == len(frames) and ph["tile_ms"] > 0
            torch.cuda.synchronize()
            for j in range(len(frames)):
                assert np.array_equal(outs[j].cpu().numpy(), refs[j]), (group_bytes, use_graph, rep, j)
        plan.close()


def test_small_and_large_tile_grids(ihb, orc):
    """One batch with tile grids of 1 x 2, 38 x 22 and 138 x 66 tiles: carry
    sequences shorter and longer than one scan chunk, split over the waves of
    a scan block or not."""
    rng = np.random.default_rng(77)
    shapes = [(600, 700, 8), (2200, 2100, 4), (16, 33, 5)]   # grids 38x22, 138x66, 1x2 at 32x16
    frames = [rng.integers(0, 256, size=(h, w), dtype=np.uint8) for h, w, _ in shapes]
    bins = [b for _, _, b in shapes]
    fr, outs = to_dev(frames, bins)
    plan = ihb.BatchPlan(fr, outs, bins, tile=(32, 16))
    plan.launch()
    torch.cuda.synchronize()
    for k, (f, b) in enumerate(zip(frames, bins)):
        assert np.array_equal(outs[k].cpu().numpy(), orc.integral_histogram(f, b)), (k, f.shape, b)
    plan.close()


def test_graph_replays_with_eager_work_between(ihb, orc):
    rng = np.random.default_rng(21)
    frames = [rng.integers(0, 256, size=(240, 320), dtype=np.uint8) for _ in range(5)]
    bins = [16, 32, 64, 128, 32]
    fr, outs = to_dev(frames, bins)
    refs = [orc.integral_histogram(f, b) for f, b in zip(frames, bins)]
    plan = ihb.BatchPlan(fr, outs, bins)
    for rep in range(4):
        for o in outs:
            o.zero_()
        torch.cuda.synchronize()
        plan.launch()
        torch.cuda.synchronize()
        for k in range(len(frames)):
            assert np.array_equal(outs[k].cpu().numpy(), refs[k]), (rep, k)
    plan.close()


def test_profiled_and_ungraphed_launches(ihb, orc):
    rng = np.random.default_rng(22)
    frames = [rng.integers(0, 256, size=(200, 256), dtype=np.uint8) for _ in range(3)]
    bins = [64, 64, 64]
    fr, outs = to_dev(frames, bins)
    for use_graph in (True, False):
        plan = ihb.BatchPlan(fr, outs, bins, use_graph=use_graph)
        ihb.profile_enable(True)
        plan.launch()
        ph = ihb.profile_read()
        ihb.profile_enable(False)
        assert ph["frames"] == 3 and ph["tile_ms"] > 0
        torch.cuda.synchronize()
        for k in range(3):
            assert np.array_equal(outs[k].cpu().numpy(), orc.integral_histogram(frames[k], bins[k]))
        plan.close()


@pytest.mark.parametrize("group_bytes,use_graph", [(1 << 20, True), (1 << 20, False), (1, True), (40 << 20, True)])
def test_pipelined_groups(ihb, orc, group_bytes, use_graph):
    """Frames split into pipeline groups (carries of group g+1 on a second
    stream beside the tile pass of group g): graph replays with eager work
    between them, direct launches, profiled launches, one frame per group
    (group_bytes=1) and uneven groups all give the oracle's bits."""
    rng = np.random.default_rng(24)
    shapes = [(240, 320, 64), (97, 203, 32), (360, 640, 16), (61, 64, 128), (240, 320, 64), (130, 257, 7),
              (480, 640, 64)]
    frames = [rng.integers(0, 256, size=(h, w), dtype=np.uint8) for h, w, _ in shapes]
    bins = [b for _, _, b in shapes]
    refs = [orc.integral_histogram(f, b) for f, b in zip(frames, bins)]
    fr, outs = to_dev(frames, bins)
    plan = ihb.BatchPlan(fr, outs, bins, use_graph=use_graph, group_bytes=group_bytes)
    info = plan.info()
    assert info["graph"] == use_graph
    total = sum(h * w * b * 4 for h, w, b in shapes)
    assert 2 <= info["groups"] <= len(frames)
    if group_bytes == 1:
        assert info["groups"] == len(frames)
    else:
        assert info["groups"] == min(len(frames), -(-total // group_bytes))
    for rep in range(3):
        for o in outs:
            o.zero_()
        torch.cuda.synchronize()
        if rep == 2:
            ihb.profile_enable(True)
        plan.launch()
        if rep == 2:
            ph = ihb.profile_read()
            ihb.profile_enable(False)
            assert ph["frames"] == len(frames) and ph["tile_ms"] > 0 and ph["agg_ms"] > 0
        torch.cuda.synchronize()
        for k in range(len(frames)):
            assert np.array_equal(outs[k].cpu().numpy(), refs[k]), (rep, k)
    plan.close()


def test_pipelined_launch_orders_after_stream_work(ihb, orc):
    """Work enqueued on the launch stream before a pipelined launch (the frame
    upload) is seen by the side stream's carry phases, and work after it sees
    every output."""
    rng = np.random.default_rng(25)
    frames = [rng.integers(0, 256, size=(300, 400), dtype=np.uint8) for _ in range(6)]
    bins = [64] * 6
    fr = [torch.zeros((300, 400), dtype=torch.uint8, device="cuda") for _ in range(6)]
    outs = [torch.empty((300, 400, 64), dtype=torch.uint32, device="cuda") for _ in range(6)]
    s = torch.cuda.Stream()
    plan = ihb.BatchPlan(fr, outs, bins, group_bytes=1 << 20, stream=s)
    host = [torch.from_numpy(f).pin_memory() for f in frames]
    sums = []
    with torch.cuda.stream(s):
        for d, h in zip(fr, host):
            d.copy_(h, non_blocking=True)
        plan.launch(s)
        for o in outs:
            sums.append(o[-1, -1].to(torch.int64).sum())
    s.synchronize()
    for k in range(6):
        assert int(sums[k]) == 300 * 400
        assert np.array_equal(outs[k].cpu().numpy(), orc.integral_histogram(frames[k], 64)), k
    plan.close()


def test_autotuned_plan(ihb, orc):
    rng = np.random.default_rng(23)
    frames = [rng.integers(0, 256, size=(360, 640), dtype=np.uint8) for _ in range(4)]
    bins = [32, 32, 128, 128]
    fr, outs = to_dev(frames, bins)
    plan = ihb.BatchPlan(fr, outs, bins, autotune=True)
    for o in outs:
        o.zero_()
    plan.launch()
    torch.cuda.synchronize()
    for k in range(4):
        tx, ty, _ = plan.frame_tile(k)
        even = {-(-360 // -(-360 // t)) for t in (8, 16, 32, 64, 128, 256)}   # bands made equally tall
        assert tx in (32, 64, 128) and ty in even
        cb = plan.frame_schedule(k)["carry_bands"]
        assert cb in (0, -2) or 1 <= cb <= -(-360 // ty), cb
        assert np.array_equal(outs[k].cpu().numpy(), orc.integral_histogram(frames[k], bins[k]))
    plan.close()


def test_disc_sequence_batched_equals_single_and_oracle(ihb, orc):
    """The full 64-frame 1920x1080 B=64 sequence in the launch configuration
    the benchmark times: every frame of the batched launch equals the oracle,
    and equals per-frame ih_compute."""
    from paper_1711_01919_amd import synth
    frames, B = synth.disc_sequence()
    n = frames.shape[0]
    d = torch.from_numpy(frames).cuda()
    outs = [torch.empty((1080, 1920, B), dtype=torch.uint32, device="cuda") for _ in range(n)]
    plan = ihb.BatchPlan([d[k] for k in range(n)], outs, [B] * n)
    plan.launch()
    single = torch.empty((1080, 1920, B), dtype=torch.uint32, device="cuda")
    for k in range(n):
        ihb.compute(d[k], B, out=single)
        torch.cuda.synchronize()
        assert bool(torch.equal(single.view(torch.int32), outs[k].view(torch.int32))), k
        assert np.array_equal(outs[k].cpu().numpy(), orc.integral_histogram(frames[k], B)), k
    plan.close()


def test_bad_descriptors_rejected(ihb):
    f = torch.zeros((8, 8), dtype=torch.uint8, device="cuda")
    o = torch.zeros((8, 8, 4), dtype=torch.uint32, device="cuda")
    with pytest.raises(ihb.IHError):
        ihb.BatchPlan([f], [o], [0])
    with pytest.raises(ihb.IHError):
        ihb.BatchPlan([f], [o], [4], tile=(48, 16))
    o256 = torch.zeros((8, 8, 256), dtype=torch.uint32, device="cuda")
    with pytest.raises(ihb.IHError):
        ihb.BatchPlan([f], [o256], [256], tile=(64, 16))        # B > 128 needs 32-wide tiles
    o128 = torch.zeros((8, 8, 128), dtype=torch.uint32, device="cuda")
    with pytest.raises(ihb.IHError):
        ihb.BatchPlan([f], [o128], [128], tile=(128, 16))       # 128-wide tiles need B = 64
    o32 = torch.zeros((8, 8, 32), dtype=torch.uint32, device="cuda")
    with pytest.raises(ihb.IHError):
        ihb.BatchPlan([f], [o32], [32], tile=(128, 16))


@pytest.mark.parametrize("group_bytes,use_graph,autotune", [(0, True, False), (40 << 20, True, False), (0, False, True)])
def test_plan_with_bin_tables(ihb, orc, group_bytes, use_graph, autotune):
    """Frames with bin tables (non-decreasing, and in any order) next to frames
    with uniform bins in one plan (graphed, pipelined, autotuned): each equals
    the oracle's result for its binning; the tables are copied at creation
    (the caller's are overwritten right after)."""
    rng = np.random.default_rng(26)
    shapes = [(240, 320, 64), (97, 203, 32), (360, 640, 16), (61, 64, 128), (240, 320, 64), (130, 257, 7),
              (480, 640, 64)]
    frames = [rng.integers(0, 256, size=(h, w), dtype=np.uint8) for h, w, _ in shapes]
    bins = [b for _, _, b in shapes]
    luts = []
    for k, b in enumerate(bins):
        if k % 4 == 0:
            edges = np.sort(rng.integers(0, 257, size=b - 1))
            luts.append(np.searchsorted(edges, np.arange(256), side="right").astype(np.uint8))
        elif k % 4 == 2:
            luts.append(rng.integers(0, b, size=256).astype(np.uint8))        # any order
        else:
            luts.append(None)
    refs = [orc.integral_histogram(f, b) if t is None else orc.integral_histogram_lut(f, b, t)
            for f, b, t in zip(frames, bins, luts)]
    fr, outs = to_dev(frames, bins)
    plan = ihb.BatchPlan(fr, outs, bins, use_graph=use_graph, group_bytes=group_bytes, autotune=autotune,
                         luts=[None if t is None else t.copy() for t in luts])
    for k, t in enumerate(luts):
        if t is not None:
            tx, _, nt = plan.frame_tile(k)
            assert tx <= 64 and not nt
    for rep in range(2):
        for o in outs:
            o.zero_()
        torch.cuda.synchronize()
        plan.launch()
        torch.cuda.synchronize()
        for k in range(len(frames)):
            assert np.array_equal(outs[k].cpu().numpy(), refs[k]), (rep, k)
    plan.close()


@pytest.mark.parametrize("group_bytes,use_graph", [(0, True), (0, False), (1, True)])
def test_plan_with_binmajor_frames(ihb, orc, group_bytes, use_graph):
    """Bin-major outputs (the paper's b x h x w) beside H x W x B ones, uniform
    and table-binned, in one plan: one launch per bin-group width for the
    bin-major pass; graph replays, direct launches and one frame per pipeline
    group all give the oracle's bits."""
    rng = np.random.default_rng(26)
    shapes = [(240, 320, 64, 1), (97, 203, 48, 1), (130, 67, 5, 1), (300, 257, 64, 0), (61, 64, 128, 1),
              (200, 130, 32, 0), (33, 384, 256, 1)]
    frames = [rng.integers(0, 256, size=(h, w), dtype=np.uint8) for h, w, _, _ in shapes]
    bins = [b for _, _, b, _ in shapes]
    layouts = [bool(m) for _, _, _, m in shapes]
    luts = [None] * len(shapes)
    edges = np.sort(rng.integers(0, 257, size=31))
    luts[5] = np.searchsorted(edges, np.arange(256), side="right").astype(np.uint8)
    fr = [torch.from_numpy(f).cuda() for f in frames]
    outs = [torch.full(((b, h, w) if m else (h, w, b)), 0xA5A5A5A5, dtype=torch.uint32, device="cuda")
            for h, w, b, m in shapes]
    refs = []
    for f, b, m, t in zip(frames, bins, layouts, luts):
        if m:
            refs.append(orc.integral_histogram_binmajor(f, b))
        else:
            refs.append(orc.integral_histogram(f, b) if t is None else orc.integral_histogram_lut(f, b, t))
    plan = ihb.BatchPlan(fr, outs, bins, use_graph=use_graph, group_bytes=group_bytes, luts=luts,
                         binmajor=layouts)
    for k, m in enumerate(layouts):
        if m:
            assert plan.frame_tile(k)[0] == 64
    for rep in range(2):
        for o in outs:
            o.zero_()
        torch.cuda.synchronize()
        plan.launch()
        torch.cuda.synchronize()
        for k in range(len(frames)):
            assert np.array_equal(outs[k].cpu().numpy(), refs[k]), (rep, k, shapes[k])
    plan.close()
