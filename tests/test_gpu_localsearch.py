"""GPU parity of the local search (Sec. 2, FE_LOCAL_SEARCH) against the
oracle: whole streams byte for byte (records carry the chosen domain
origin)."""
import sys

import numpy as np
import pytest

from oracle import localsearch
from paper_1501_02894_amd import binding as fb
from paper_1501_02894_amd import synth

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


@pytest.fixture(scope="module")
def ctx(torch_dev):
    c = fb.Context(0)
    yield c
    c.close()


CASES = [
    ("c1", lambda: synth.workload("c1"), 8, 4, [600]),
    ("c2", lambda: synth.workload("c2"), 16, 4, [300, 200]),
    ("noise 48x64 16/4", lambda: synth.noise_1f(48, 64, 31), 16, 4, [250, 150]),
    ("pw 64x32 8/4", lambda: synth.piecewise_smooth(64, 32, 32, cells=6), 8, 4, [100]),
    ("noise 4/4", lambda: synth.noise_1f(16, 24, 18), 4, 4, []),
    ("ramp", lambda: synth.ramp(64, 64), 16, 4, [1, 1]),
]


@pytest.mark.parametrize("name,make,b_max,b_min,thr", CASES, ids=[c[0] for c in CASES])
def test_local_search_stream(torch_dev, ctx, name, make, b_max, b_min, thr):
    log(f"local search {name}")
    img = make()
    want = localsearch.encode(img, b_max, b_min, thr)
    got = fb.to_records(ctx.encode(torch_dev.from_numpy(img).cuda(), b_max, b_min, thr, local_search=True))
    assert got.size == want.size
    assert got.tobytes() == np.ascontiguousarray(want).tobytes()


def test_local_search_limits(torch_dev, ctx):
    img = torch_dev.from_numpy(synth.noise_1f(64, 64, 3)).cuda()
    with pytest.raises(fb.FeError) as ei:
        ctx.encode(img, 32, 4, [100, 100, 100], local_search=True)    # b_max <= 16, as the exhaustive search
    assert ei.value.status == fb.FE_ERR_INVALID
