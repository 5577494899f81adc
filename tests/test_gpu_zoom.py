"""GPU parity of zoom decoding (Sec. 1: the maps are resolution
independent) against the oracle: the oracle zooms the records
(oracle.decode.zoom) and decodes them with its integer decoder at the zoomed
size; the GPU's fe_decode_zoom must give the same pixels, on both decoders."""
import sys

import numpy as np
import pytest

from oracle import decode as odec
from oracle import fullsearch, mns
from paper_1501_02894_amd import binding as fb
from paper_1501_02894_amd import synth
from streams import random_stream

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


def _t(torch, rec):
    return torch.from_numpy(np.ascontiguousarray(rec).view(np.uint8).reshape(-1, 16).copy()).cuda()


def _zoom_both(torch, ctx, rec, W, H, bm, z, iters, start=None, expect=fb.FE_DECODE_TILES):
    t = _t(torch, rec)
    s = None if start is None else torch.from_numpy(np.ascontiguousarray(start)).cuda()
    out = {}
    try:
        for mode in (fb.FE_DECODE_AUTO, fb.FE_DECODE_RECORDS):
            ctx.decode_mode(mode)
            out[mode] = ctx.decode_zoom(t, W, H, bm, z, iters, start=s).cpu().numpy()
            assert ctx.decode_last() == (expect if mode == fb.FE_DECODE_AUTO else fb.FE_DECODE_RECORDS)
    finally:
        ctx.decode_mode(fb.FE_DECODE_AUTO)
    return out[fb.FE_DECODE_AUTO], out[fb.FE_DECODE_RECORDS]


@pytest.mark.parametrize("W,H,bm,bmin,seed,z", [
    (64, 48, 16, 4, 3, 2), (112, 80, 8, 4, 4, 2), (112, 80, 8, 4, 4, 4), (64, 64, 4, 4, 5, 8),
    (264, 136, 8, 4, 6, 4), (96, 64, 16, 8, 11, 2),
])
def test_random_streams(torch_dev, ctx, W, H, bm, bmin, seed, z):
    log(f"zoom random {W}x{H} b{bm}/{bmin} x{z}")
    rec = random_stream(W, H, bm, bmin, seed)
    start = np.random.default_rng(seed).integers(0, 256, (z * H, z * W)).astype(np.uint8)
    tiles, records = _zoom_both(torch_dev, ctx, rec, W, H, bm, z, 3, start=start)
    want = odec.decode(odec.zoom(rec, z), z * W, z * H, z * bm, 3, start=start)
    np.testing.assert_array_equal(tiles, want)
    np.testing.assert_array_equal(records, want)


@pytest.mark.parametrize("name,b_max,b_min,thr,z", [("c1", 8, 4, [600], 2), ("c1", 8, 4, [600], 4),
                                                    ("c2", 16, 4, [300, 200], 2)])
def test_encoded_streams(torch_dev, ctx, name, b_max, b_min, thr, z):
    log(f"zoom {name} x{z}")
    img = synth.workload(name)
    H, W = img.shape
    rec = mns.encode(img, b_max, b_min, thr)
    tiles, records = _zoom_both(torch_dev, ctx, rec, W, H, b_max, z, 8)
    want = odec.decode(odec.zoom(rec, z), z * W, z * H, z * b_max, 8)
    np.testing.assert_array_equal(tiles, want)
    np.testing.assert_array_equal(records, want)


def test_zoom_one_is_decode(torch_dev, ctx):
    log("zoom x1 = decode")
    img = synth.workload("c1")
    rec = mns.encode(img, 8, 4, [600])
    t = _t(torch_dev, rec)
    a = ctx.decode_zoom(t, 64, 64, 8, 1, 6).cpu().numpy()
    b = ctx.decode(t, 64, 64, 8, 6).cpu().numpy()
    np.testing.assert_array_equal(a, b)


def test_full_search_stream(torch_dev, ctx):
    log("zoom full-search stream")
    img = synth.noise_1f(32, 32, 4)
    rec = fullsearch.encode(img, 8, 4, [300])
    tiles, records = _zoom_both(torch_dev, ctx, rec, 32, 32, 8, 2, 4, expect=fb.FE_DECODE_RECORDS)
    want = odec.decode(odec.zoom(rec, 2), 64, 64, 16, 4)
    np.testing.assert_array_equal(tiles, want)
    np.testing.assert_array_equal(records, want)


def test_argument_errors(torch_dev, ctx):
    log("zoom argument errors")
    rec = random_stream(64, 48, 16, 4, 3)
    t = _t(torch_dev, rec)
    for z in (3, 0, 4):          # not a power of two; zero; 4 * 16 > 32
        with pytest.raises(fb.FeError):
            ctx.decode_zoom(t, 64, 48, 16, z, 1)
    # a transform that lies outside the native image is rejected
    bad = np.array(rec, copy=True)
    bad[0]["x"] = 64
    with pytest.raises(fb.FeError):
        ctx.decode_zoom(_t(torch_dev, bad), 64, 48, 16, 2, 1)
