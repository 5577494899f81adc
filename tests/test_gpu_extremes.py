"""GPU parity at the edges of the accepted shapes, through the C ABI: image
sides of 65536 (the largest the 16-bit record fields allow) in both
directions, for the fused encoder, the 2 x 2 encoder, both decoders, zoom
decoding and the compressed file; and the empty stream."""
import sys

import numpy as np
import pytest

from oracle import bitstream as bs
from oracle import decode as odec
from oracle import mns
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


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _t(torch, rec):
    return torch.from_numpy(np.ascontiguousarray(rec).view(np.uint8).reshape(-1, 16).copy()).cuda()


def assert_same_stream(got, want):
    assert got.size == want.size, (got.size, want.size)
    gb = got.view(np.uint8).reshape(-1, 16)
    wb = np.ascontiguousarray(want).view(np.uint8).reshape(-1, 16)
    bad = np.flatnonzero(np.any(gb != wb, axis=1))
    assert bad.size == 0, f"{bad.size} records differ; first {bad[0]}: got {got[bad[0]]} want {want[bad[0]]}"


_IMGS = {}


def image(h, w, seed):
    """1/f noise in blocks of 512 along the long side (each block spans
    0..255, so the quadtree reaches every level)."""
    key = (h, w, seed)
    if key not in _IMGS:
        if w >= h:
            _IMGS[key] = np.hstack([synth.noise_1f(h, 512, seed + k) for k in range(w // 512)])
        else:
            _IMGS[key] = np.vstack([synth.noise_1f(512, w, seed + k) for k in range(h // 512)])
    return _IMGS[key]


MAX_CASES = [
    # H, W, b_max, b_min, thresholds
    (32, 65536, 16, 4, [300, 200]),
    (65536, 32, 16, 4, [300, 200]),
    (64, 65536, 32, 4, [900, 600, 300]),
    (32, 65536, 16, 2, [300, 200, 100]),
    (65536, 16, 8, 2, [300, 150]),
]


@pytest.mark.parametrize("H,W,bm,bmin,thr", MAX_CASES)
def test_encode_max_side(torch_dev, ctx, H, W, bm, bmin, thr):
    log(f"encode {W}x{H} b{bm}/{bmin}")
    img = image(H, W, 51)
    want = mns.encode(img, bm, bmin, thr)
    assert len(set(want["level"].tolist())) == len(thr) + 1   # every level is reached
    got = fb.to_records(ctx.encode(dev(torch_dev, img), bm, bmin, thr))
    assert_same_stream(got, want)


@pytest.mark.parametrize("H,W,bm,bmin,thr", [MAX_CASES[0], MAX_CASES[1], MAX_CASES[3]])
def test_decode_max_side(torch_dev, ctx, H, W, bm, bmin, thr):
    log(f"decode {W}x{H} b{bm}/{bmin}")
    img = image(H, W, 51)
    rec = mns.encode(img, bm, bmin, thr)
    t = _t(torch_dev, rec)
    want = odec.decode(rec, W, H, bm, 4)
    try:
        for mode in (fb.FE_DECODE_AUTO, fb.FE_DECODE_RECORDS):
            ctx.decode_mode(mode)
            got = ctx.decode(t, W, H, bm, 4).cpu().numpy()
            np.testing.assert_array_equal(got, want)
    finally:
        ctx.decode_mode(fb.FE_DECODE_AUTO)


def test_zoom_to_max_side(torch_dev, ctx):
    log("zoom 32768x16 -> 65536x32")
    img = image(16, 32768, 52)
    rec = mns.encode(img, 8, 4, [300])
    assert set(rec["level"].tolist()) == {0, 1}
    got = ctx.decode_zoom(_t(torch_dev, rec), 32768, 16, 8, 2, 3).cpu().numpy()
    assert ctx.decode_last() == fb.FE_DECODE_TILES
    np.testing.assert_array_equal(got, odec.decode(odec.zoom(rec, 2), 65536, 32, 16, 3))
    with pytest.raises(fb.FeError):   # 65536 x 2 would exceed the largest side
        ctx.decode_zoom(_t(torch_dev, rec), 32768, 16, 8, 4, 1)


@pytest.mark.parametrize("H,W,bm,bmin,thr", [MAX_CASES[0], MAX_CASES[4]])
def test_pack_max_side(torch_dev, ctx, H, W, bm, bmin, thr):
    log(f"pack {W}x{H} b{bm}/{bmin}")
    img = image(H, W, 51)
    rec = mns.encode(img, bm, bmin, thr)
    want, want_bits = bs.pack(rec, W, H, bm, bmin, isometries=True)
    out, nbits = fb.fe_pack(ctx.handle, _t(torch_dev, rec), W, H, bm, bmin, isometry=True)
    data = out.cpu().numpy().tobytes()[: (nbits + 7) // 8]
    assert nbits == want_bits and data == want
    back, info = fb.fe_unpack(data, nbits)
    assert (info["width"], info["height"]) == (W, H)
    assert back.tobytes() == np.ascontiguousarray(rec).tobytes()


def test_empty_stream_decodes_to_the_start(torch_dev, ctx):
    log("decode of an empty stream")
    import torch
    empty = torch.empty((0, 16), dtype=torch.uint8, device="cuda")
    start = np.random.default_rng(53).integers(0, 256, (48, 64)).astype(np.uint8)
    got = ctx.decode(empty, 64, 48, 16, 5, start=dev(torch_dev, start)).cpu().numpy()
    np.testing.assert_array_equal(got, start)
    grey = ctx.decode(empty, 64, 48, 16, 2).cpu().numpy()
    assert np.all(grey == 128)
    assert ctx.decode_last() == fb.FE_DECODE_RECORDS
