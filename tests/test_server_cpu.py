"""Serving-loop API checks that need no GPU: argument validation, the whole-
budget rejection, unknown tickets and shutdown.  Every path here returns
before the scheduler touches a device."""
import numpy as np
import pytest

from paper_1711_01919_amd import binding as ihb


@pytest.fixture
def server():
    s = ihb.Server(budget_bytes=64 << 20, max_slots=4, n_hip_streams=2, max_batch=4)
    yield s
    s.close()


def test_bad_config_rejected():
    for kw in ({"budget_bytes": 1000}, {"budget_bytes": 64 << 20, "max_slots": 0},
               {"budget_bytes": 64 << 20, "n_hip_streams": 0}, {"budget_bytes": 64 << 20, "n_hip_streams": 17},
               {"budget_bytes": 64 << 20, "max_batch": 0}):
        with pytest.raises(ihb.IHError) as e:
            ihb.Server(**kw)
        assert e.value.status == 1


def test_submit_validation(server):
    f = np.zeros((16, 16), np.uint8)
    for B in (0, 257):
        with pytest.raises(ihb.IHError) as e:
            server.submit(0, f, B)
        assert e.value.status == 1
    for bad in ([0, 0, 16, 0], [-1, 0, 0, 0], [3, 0, 2, 0], [0, 0, 0, 16]):
        with pytest.raises(ihb.IHError) as e:
            server.submit(0, f, 8, np.array([bad]))
        assert e.value.status == 1


def test_submit_rejects_bad_tables(server):
    f = np.zeros((16, 16), np.uint8)
    ok = np.repeat(np.arange(8, dtype=np.uint8), 32)
    for bad in (np.minimum(ok + 1, 8).astype(np.uint8),                        # entry 8 with B = 8
                np.where(np.arange(256) == 100, 9, ok[::-1]).astype(np.uint8)):  # any order, but 9 >= B
        with pytest.raises(ihb.IHError) as e:
            server.submit(0, f, 8, lut=bad)
        assert e.value.status == 1
    with pytest.raises(ValueError):
        server.submit(0, f, 8, lut=ok[:255])
    # a table in any order, each entry below B, is accepted
    assert server.submit(0, f, 8, lut=ok[::-1].copy()) > 0


def test_request_larger_than_budget(server):
    f = np.zeros((1024, 1024), np.uint8)               # 1024*1024*64*4 B = 256 MiB > 64 MiB
    with pytest.raises(ihb.IHError) as e:
        server.submit(0, f, 64)
    assert e.value.status == 5                          # IH_ERR_BUDGET


def test_unknown_ticket(server):
    assert server.poll_status(12345) == 7               # IH_ERR_UNKNOWN_TICKET


def test_close_is_idempotent(server):
    server.close()
    server.close()
