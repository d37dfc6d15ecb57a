import os
import sys
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parent.parent
if str(ROOT) not in sys.path:
    sys.path.insert(0, str(ROOT))


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def orc():
    import oracle
    return oracle.get()


def compare_with_oracle_rows(orc, ih_dev, I, B, block_bytes=128 << 20):
    """Compare a device integral histogram (H, W, B) with the oracle entry by
    entry, streaming blocks of rows: the oracle continues its recursion block
    after block (integral_rows), and each block is downloaded only when its
    turn comes, so host memory stays bounded whatever the frame size.
    Returns None when every entry agrees, else (y, x, b, got, want) of the
    first difference."""
    import numpy as np
    H, W = I.shape
    rows = max(1, block_bytes // (W * B * 4))
    for y0, want in orc.iter_row_blocks(I, B, rows):
        got = ih_dev[y0:y0 + want.shape[0]].cpu().numpy()
        if not np.array_equal(got, want):
            y, x, b = (int(v) for v in np.argwhere(got != want)[0])
            return (y0 + y, x, b, int(got[y, x, b]), int(want[y, x, b]))
    return None


@pytest.fixture(scope="session")
def rows_compare():
    return compare_with_oracle_rows
