"""GPU parity of the exhaustive-search baseline (int8 MFMA + exact epilogue)
against the oracle's definition: the argmin over every step-1 domain,
isometry and contrast of the scaled collage error, ties to the lowest
domain index, then isometry, then contrast."""
import os
import sys

import numpy as np
import pytest

import oracle_pool
from oracle import decode as odec
from oracle import fullsearch, mns
from paper_1501_02894_amd import binding as fb
from paper_1501_02894_amd import synth

pytestmark = pytest.mark.gpu

# ranges of the C2 exhaustive search checked against the oracle
C2_SAMPLES = int(os.environ.get("FE_FS_SAMPLES", "4096"))


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


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def gpu_best(torch, ctx, img, B, xs, ys):
    xy = dev(torch, (np.asarray(xs) | (np.asarray(ys) << 16)).astype(np.int32))
    out = ctx.full_search_ranges(dev(torch, img), B, xy).cpu().numpy().view(np.uint32)
    S = out[:, 2].astype(np.int64) | (out[:, 3].astype(np.int64) << 32)
    return {"dom": out[:, 0].astype(np.int64), "e": (out[:, 1] & 0xff).astype(np.int64),
            "k": ((out[:, 1] >> 8) & 0xff).astype(np.int64), "m": (out[:, 1] >> 16).astype(np.int64), "S": S}


def assert_best_equal(got, want, label):
    for key in ("S", "dom", "e", "k", "m"):
        bad = np.flatnonzero(got[key] != want[key])
        assert bad.size == 0, f"{label}: {key} differs at {bad[:8]}: got {got[key][bad[:8]]} want {want[key][bad[:8]]}"


@pytest.mark.parametrize("H,W,B,kind", [
    (24, 24, 4, "noise"), (40, 32, 4, "noise"), (32, 48, 8, "noise"), (64, 64, 16, "noise"),
    (48, 64, 8, "pw"), (80, 48, 4, "pw"), (64, 96, 16, "pw"), (32, 32, 8, "flat"), (64, 64, 8, "ramp"),
])
def test_full_search_every_range(torch_dev, ctx, H, W, B, kind):
    log(f"full search {H}x{W} B={B} {kind}")
    if kind == "noise":
        img = synth.noise_1f(H, W, H * 7 + W)
    elif kind == "pw":
        img = synth.piecewise_smooth(H, W, H + W, cells=6)
    elif kind == "flat":
        img = synth.flat(H, W, 90)
    else:
        img = synth.ramp(H, W)
    ys, xs = np.mgrid[0:H:B, 0:W:B]
    xs, ys = xs.ravel(), ys.ravel()
    want = fullsearch.best_matches(img, xs, ys, B)
    got = gpu_best(torch_dev, ctx, img, B, xs, ys)
    assert_best_equal(got, want, f"{H}x{W} B={B}")


def test_full_search_encode_c1(torch_dev, ctx):
    log("full-search encode c1")
    img = synth.workload("c1")
    want = fullsearch.encode(img, 8, 4, [600])
    got = fb.to_records(ctx.encode(dev(torch_dev, img), 8, 4, [600], full_search=True))
    assert got.size == want.size
    assert got.tobytes() == np.ascontiguousarray(want).tobytes()
    # the exhaustive stream tiles the image and decodes
    odec.decode(got, 64, 64, 8, 2)


@pytest.mark.parametrize("H,W,bmax,bmin,thr", [(48, 64, 16, 4, [250, 150]), (64, 32, 8, 4, [100])])
def test_full_search_encode_small(torch_dev, ctx, H, W, bmax, bmin, thr):
    img = synth.noise_1f(H, W, 77 + H)
    want = fullsearch.encode(img, bmax, bmin, thr)
    got = fb.to_records(ctx.encode(dev(torch_dev, img), bmax, bmin, thr, full_search=True))
    assert got.tobytes() == np.ascontiguousarray(want).tobytes()


def evaluated_ranges(rec, b_max: int, levels: int):
    """Per level, the ranges the quadtree evaluated: every record's ancestor
    (or itself) at that level, i.e. the level's accepted ranges and the ones
    it split.  Returns a list of (xs, ys) arrays."""
    out = []
    x, y, lv = (rec[k].astype(np.int64) for k in ("x", "y", "level"))
    for level in range(levels):
        B = b_max >> level
        sel = lv >= level
        key = np.unique(((y[sel] // B) << 20) | (x[sel] // B))
        out.append(((key & 0xfffff) * B, (key >> 20) * B))
    return out


@pytest.mark.slow
def test_full_search_c2_sampled(torch_dev, ctx):
    """C2 (512^2, 16->8->4): up to 4096 ranges drawn uniformly (seed 2) from
    the ranges the exhaustive quadtree evaluated at its three levels (it
    evaluates fewer than that on C2, about 1500, so all of them), each checked
    against the oracle's exhaustive definition (best domain, isometry,
    contrast, luminance and error); a sampled range is a record of the stream
    exactly when the oracle's error is below the level's threshold (or the
    level is the last), with the oracle's fields.  The stream's structure is
    checked at every record."""
    log("full-search encode c2")
    img = synth.workload("c2")
    thr = [300, 200]
    got = fb.to_records(ctx.encode(dev(torch_dev, img), 16, 4, thr, full_search=True))
    odec.decode(got, 512, 512, 16, 1)           # tiles the image exactly once
    ev = evaluated_ranges(got, 16, 3)
    sizes = [xs.size for xs, _ in ev]
    total = sum(sizes)
    rng = np.random.default_rng(2)
    pick = np.sort(rng.choice(total, min(C2_SAMPLES, total), replace=False))
    bounds = np.concatenate([[0], np.cumsum(sizes)])
    with oracle_pool.pool() as ex:
        jobs = []
        for level in range(3):
            B = 16 >> level
            sel = pick[(pick >= bounds[level]) & (pick < bounds[level + 1])] - bounds[level]
            xs, ys = ev[level][0][sel], ev[level][1][sel]
            log(f"  level {level + 1}: checking {sel.size} of {sizes[level]} evaluated ranges")
            jobs.append((level, B, xs, ys, oracle_pool.best_matches(ex, img, xs, ys, B)))
        rec_at = {(int(x), int(y), int(l)): i for i, (x, y, l) in
                  enumerate(zip(got["x"], got["y"], got["level"]))}
        for level, B, xs, ys, futs in jobs:
            parts = [f.result() for f in futs]
            want = {k: np.concatenate([p[k] for p in parts]) for k in parts[0]}
            assert_best_equal(gpu_best(torch_dev, ctx, img, B, xs, ys), want, f"c2 level {level + 1}")
            n = B * B
            accept = np.ones(xs.size, bool) if level == 2 else want["S"] < 64 * n * n * thr[level]
            for j in range(xs.size):
                i = rec_at.get((int(xs[j]), int(ys[j]), level))
                assert (i is not None) == bool(accept[j]), f"level {level + 1} range ({xs[j]}, {ys[j]})"
                if i is not None:
                    assert (int(got["dx"][i]), int(got["dy"][i])) == (int(want["u"][j]), int(want["v"][j]))
                    assert (int(got["iso"][i]), int(got["s_idx"][i]), int(got["lum"][i])) == \
                        (int(want["e"][j]), int(want["k"][j]), int(want["m"][j]))
            log(f"  level {level + 1}: {xs.size} ranges equal the oracle ({int(accept.sum())} stored)")


def test_full_search_not_worse_than_mns(torch_dev, ctx):
    img = synth.workload("c1")
    ys, xs = np.mgrid[0:64:8, 0:64:8]
    xs, ys = xs.ravel(), ys.ravel()
    got = gpu_best(torch_dev, ctx, img, 8, xs, ys)
    mom = mns.range_moments(img.astype(np.int64), mns.downsample(img), xs, ys, 8)
    _, _, _, S_mns = mns.fit_phase1(mom, 64)
    assert np.all(got["S"] <= S_mns)


def test_full_search_limits(torch_dev, ctx):
    big = np.zeros((2048, 2048), np.uint8)
    with pytest.raises(fb.FeError) as ei:
        ctx.encode(dev(torch_dev, big), 16, 4, [1, 1], full_search=True)
    assert ei.value.status == fb.FE_ERR_SHAPE
    with pytest.raises(fb.FeError) as ei:
        ctx.encode(dev(torch_dev, np.zeros((128, 128), np.uint8)), 32, 4, [1, 1, 1], full_search=True)
    assert ei.value.status == fb.FE_ERR_INVALID
