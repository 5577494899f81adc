"""The random test streams are valid encoder-order streams (CPU)."""
import numpy as np
import pytest

from oracle import decode as odec
from oracle import mns
from streams import random_stream


@pytest.mark.parametrize("W,H,bm,bmin,seed", [(96, 160, 32, 4, 1), (64, 48, 16, 4, 3), (64, 64, 4, 4, 5),
                                              (288, 160, 16, 8, 8)])
def test_random_stream_is_valid(W, H, bm, bmin, seed):
    rec = random_stream(W, H, bm, bmin, seed)
    key = mns.stream_key(rec["x"], rec["y"], W, bm, bmin)
    assert np.all(np.diff(key) > 0)                        # encoder order
    B = bm >> rec["level"].astype(np.int64)
    assert np.all(B >= bmin)
    p2 = rec["flags"] == mns.FLAG_PHASE2
    assert np.all(B[p2] >= 8)
    m = rec["lum"].astype(np.int64)
    d = rec["dlum"].astype(np.int64)
    O = np.stack([m + d[:, 0], m + d[:, 1], m + d[:, 2], m - d.sum(1)], 1)[p2]
    assert np.all((O >= 0) & (O <= 255))
    assert np.all(d[~p2] == 0)
    odec.decode(rec, W, H, bm, 1)                          # tiles the image exactly once
