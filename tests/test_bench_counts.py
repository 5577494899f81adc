"""The bench's range-block count (phase-1 evaluations, Sum_l |W_l|) equals
the number of ranges the oracle actually fits, counted by instrumenting its
phase-1 fit (CPU)."""
import numpy as np
import pytest

import bench
from oracle import mns
from paper_1501_02894_amd import synth


@pytest.mark.parametrize("name,make,b_max,b_min,thr", [
    ("c1", lambda: synth.workload("c1"), 8, 4, [600]),
    ("c2", lambda: synth.workload("c2"), 16, 4, [300, 200]),
    ("pw", lambda: synth.piecewise_smooth(192, 256, 13, cells=40), 32, 4, [120, 90, 60]),
    ("c2 low", lambda: synth.workload("c2"), 16, 4, [40, 20]),
])
def test_range_blocks_count_phase1_evaluations(monkeypatch, name, make, b_max, b_min, thr):
    img = make()
    seen = []
    orig = mns.fit_phase1

    def counting(mom, n):
        seen.append(len(mom["sr"]))
        return orig(mom, n)

    monkeypatch.setattr(mns, "fit_phase1", counting)
    rec = mns.encode(img, b_max, b_min, thr)
    tiles = (img.shape[0] // b_max) * (img.shape[1] // b_max)
    got = bench.range_blocks(rec["level"], rec["flags"], tiles, bench.n_levels(b_max, b_min))
    assert got == sum(seen)
    if name == "c2":
        assert np.any(rec["flags"] != 0)       # phase-2 records are counted as leaves
