"""Serving loop on the GPU: each request's histograms are the same when served
alone and when served in a mix of concurrent streams, equal the oracle, and
budget, retention and shutdown behave as documented.  Tolerance 0."""
import threading

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ihb():
    from paper_1711_01919_amd import binding
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return binding


def make_requests(n=40, seed=31):
    from paper_1711_01919_amd import synth
    rng = np.random.default_rng(seed)
    sizes = [(240, 320), (480, 640), (360, 640), (720, 1280), (101, 203)]
    reqs = []
    for k in range(n):
        H, W = sizes[int(rng.integers(0, len(sizes)))]
        B = [32, 64, 16, 128][int(rng.integers(0, 4))]
        I = rng.integers(0, 256, size=(H, W), dtype=np.uint8)
        rects = synth.random_rects(rng, H, W, int(rng.integers(1, 80)))
        reqs.append((k % 8, I, B, rects))
    return reqs


def oracle_hists(orc, I, B, rects):
    return orc.region_histogram(orc.integral_histogram(I, B), rects)


def test_alone_equals_mix_equals_oracle(ihb, orc):
    reqs = make_requests()
    # alone: one request at a time, one stream, batches of one
    alone = []
    srv = ihb.Server(budget_bytes=2 << 30, max_slots=1, n_hip_streams=1, max_batch=1)
    for sid, I, B, rects in reqs:
        t = srv.submit(sid, I, B, rects)
        h, tm = srv.wait(t)
        assert tm["t_submit_ns"] <= tm["t_admit_ns"] <= tm["t_done_ns"]
        alone.append(h)
    srv.close()
    # mix: everything at once from two submitting threads, four streams, batches of up to eight
    srv = ihb.Server(budget_bytes=4 << 30, max_slots=32, n_hip_streams=4, max_batch=8)
    tickets = [None] * len(reqs)

    def submit(ks):
        for k in ks:
            sid, I, B, rects = reqs[k]
            tickets[k] = srv.submit(sid, I, B, rects)

    th = [threading.Thread(target=submit, args=(range(j, len(reqs), 2),)) for j in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    mix = [srv.wait(t)[0] for t in tickets]
    srv.close()
    for k, (sid, I, B, rects) in enumerate(reqs):
        assert np.array_equal(alone[k], mix[k]), k
        assert np.array_equal(mix[k], oracle_hists(orc, I, B, rects)), k


def test_bin_tables_in_mixed_batches(ihb, orc):
    """Requests with bin tables (random edges) and with uniform bins share
    batches; each equals the oracle's table-binned or uniform result, alone
    and in the mix."""
    from paper_1711_01919_amd import synth
    rng = np.random.default_rng(33)
    reqs = []
    for k in range(24):
        H, W = [(240, 320), (101, 203), (480, 640)][k % 3]
        B = [16, 32, 64, 100][int(rng.integers(0, 4))]
        I = rng.integers(0, 256, size=(H, W), dtype=np.uint8)
        rects = synth.random_rects(rng, H, W, int(rng.integers(1, 50)))
        lut = None
        if k % 4 == 0:
            edges = np.sort(rng.integers(0, 257, size=B - 1))
            lut = np.searchsorted(edges, np.arange(256), side="right").astype(np.uint8)
        elif k % 4 == 2:
            lut = rng.integers(0, B, size=256).astype(np.uint8)              # any order
        reqs.append((k % 4, I, B, rects, lut))
    results = {}
    for cfg in (dict(max_slots=1, n_hip_streams=1, max_batch=1), dict(max_slots=16, n_hip_streams=3, max_batch=6)):
        srv = ihb.Server(budget_bytes=2 << 30, **cfg)
        tickets = [srv.submit(sid, I, B, rects, lut=lut) for sid, I, B, rects, lut in reqs]
        results[cfg["max_batch"]] = [srv.wait(t)[0] for t in tickets]
        srv.close()
    for k, (sid, I, B, rects, lut) in enumerate(reqs):
        ref = orc.integral_histogram(I, B) if lut is None else orc.integral_histogram_lut(I, B, lut)
        want = orc.region_histogram(ref, rects)
        assert np.array_equal(results[1][k], want), k
        assert np.array_equal(results[6][k], want), k


def test_backpressure_under_small_budget(ihb, orc):
    """Budget for about two 720p B=64 requests at once: the rest wait, none fail."""
    rng = np.random.default_rng(32)
    H, W, B = 720, 1280, 64
    frames = [rng.integers(0, 256, size=(H, W), dtype=np.uint8) for _ in range(8)]
    rects = np.array([[0, 0, W - 1, H - 1], [10, 20, 300, 400]], np.int32)
    per_req = H * W * B * 4
    budget = int(2.3 * per_req)
    srv = ihb.Server(budget_bytes=budget, max_slots=16, n_hip_streams=4, max_batch=4)
    srv.hold(True)
    tickets = [srv.submit(k, f, B, rects) for k, f in enumerate(frames)]
    assert srv.stats()["pending"] == len(frames)
    srv.hold(False)
    outs = [srv.wait(t)[0] for t in tickets]
    st = srv.stats()
    srv.close()
    assert st["budget_blocked"] >= 1
    assert per_req < st["device_bytes_peak"] <= budget
    assert st["device_bytes_used"] == 0 and st["admitted"] == 0 and st["pending"] == 0
    for f, h in zip(frames, outs):
        assert np.array_equal(h, oracle_hists(orc, f, B, rects))


def test_retention_and_latest_queries(ihb, orc):
    rng = np.random.default_rng(33)
    H, W, B = 480, 640, 64                               # 78.6 MB per integral histogram
    srv = ihb.Server(budget_bytes=640 << 20, max_slots=8, n_hip_streams=2, max_batch=4, retain=True)
    frames = {s: [rng.integers(0, 256, size=(H, W), dtype=np.uint8) for _ in range(3)] for s in (0, 1)}
    last = {}
    for k in range(3):
        for s in (0, 1):
            t = srv.submit(s, frames[s][k], B, np.array([[0, 0, W - 1, H - 1]], np.int32))
            srv.wait(t)
            last[s] = t
    assert srv.stats()["retained"] == 2
    q = np.array([[5, 6, 100, 200], [0, 0, 0, 0], [W - 1, H - 1, W - 1, H - 1]], np.int32)
    for s in (0, 1):
        h, ft = srv.query_latest(s, q, B)
        assert ft == last[s]
        assert np.array_equal(h, oracle_hists(orc, frames[s][2], B, q))
    # a 1080p B=64 request (about 575 MB with its carries) only fits once the
    # two retained histograms are evicted
    big = rng.integers(0, 256, size=(1080, 1920), dtype=np.uint8)
    t = srv.submit(2, big, 64, np.array([[0, 0, 1919, 1079]], np.int32))
    h, _ = srv.wait(t)
    assert int(h.astype(np.int64).sum()) == 1080 * 1920
    for s in (0, 1):
        with pytest.raises(ihb.IHError):
            srv.query_latest(s, q, B)
    srv.close()


def test_tickets_collected_once(ihb):
    srv = ihb.Server(budget_bytes=256 << 20, max_slots=4, n_hip_streams=1, max_batch=2)
    t = srv.submit(0, np.zeros((64, 64), np.uint8), 8, np.array([[0, 0, 63, 63]], np.int32))
    h, _ = srv.wait(t)
    assert h[0, 0] == 64 * 64
    assert srv.poll_status(t) == 7
    srv.close()


def test_shutdown_with_queued_work(ihb):
    """Destroying the server with requests still queued returns without
    hanging; running batches finish first."""
    rng = np.random.default_rng(34)
    srv = ihb.Server(budget_bytes=512 << 20, max_slots=2, n_hip_streams=1, max_batch=1)
    for k in range(12):
        srv.submit(k, rng.integers(0, 256, size=(720, 1280), dtype=np.uint8), 64,
                   np.array([[0, 0, 9, 9]], np.int32))
    srv.close()
