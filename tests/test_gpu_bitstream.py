"""GPU parity of the compressed file (fe_pack, Sec. 3.3 and Technique 2 of
Sec. 3.4) and of the identity-only encoder against the oracle, through the
C ABI: files compared byte for byte, bit counts exactly; the native parser
closes the round trip through the decoder."""
import sys

import numpy as np
import pytest

from oracle import bitstream as bs
from oracle import decode as odec
from oracle import mns
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


def _gpu_file(torch, ctx, rec_t, W, H, bm, bmin, iso):
    out, nbits = fb.fe_pack(ctx.handle, rec_t, W, H, bm, bmin, isometry=iso)
    torch.cuda.synchronize()
    data = out.cpu().numpy().tobytes()
    return data, nbits


def _same_file(gpu, nbits, want, want_bits):
    assert nbits == want_bits
    nbytes = (nbits + 7) // 8
    assert gpu[:nbytes] == want[:nbytes]
    assert gpu[nbytes:(nbits + 63) // 64 * 8] == bytes((nbits + 63) // 64 * 8 - nbytes)   # zero padding


IMAGES = [
    ("c1", lambda: synth.workload("c1"), 8, 4, [600]),
    ("c2", lambda: synth.workload("c2"), 16, 4, [300, 200]),
    ("pw 32", lambda: synth.piecewise_smooth(192, 256, 13, cells=40), 32, 4, [120, 90, 60]),
    ("noise 4", lambda: synth.noise_1f(16, 24, 18), 4, 4, []),
    ("noise 16/8", lambda: synth.noise_1f(128, 128, 15), 16, 8, [300]),
]


@pytest.mark.parametrize("name,make,b_max,b_min,thr", IMAGES, ids=[c[0] for c in IMAGES])
@pytest.mark.parametrize("iso", [True, False], ids=["isometries", "identity"])
def test_pack_encoded(torch_dev, ctx, name, make, b_max, b_min, thr, iso):
    """GPU encode (identity-only when iso is off) -> GPU pack, against the
    oracle's encode and pack of the same image."""
    log(f"pack {name} iso={iso}")
    img = make()
    H, W = img.shape
    want_rec = mns.encode(img, b_max, b_min, thr, isometries=iso)
    got = ctx.encode(torch_dev.from_numpy(img).cuda(), b_max, b_min, thr, identity_only=not iso)
    assert fb.to_records(got).tobytes() == np.ascontiguousarray(want_rec).tobytes()
    want, want_bits = bs.pack(want_rec, W, H, b_max, b_min, isometries=iso)
    data, nbits = _gpu_file(torch_dev, ctx, got, W, H, b_max, b_min, iso)
    _same_file(data, nbits, want, want_bits)


@pytest.mark.parametrize("W,H,bm,bmin,seed", [(96, 160, 32, 4, 1), (160, 96, 32, 8, 2), (64, 48, 16, 4, 3),
                                              (264, 136, 8, 4, 6), (1040, 528, 16, 4, 10)])
def test_pack_random(torch_dev, ctx, W, H, bm, bmin, seed):
    r = random_stream(W, H, bm, bmin, seed, bounded=True)
    want, want_bits = bs.pack(r, W, H, bm, bmin, isometries=True)
    data, nbits = _gpu_file(torch_dev, ctx, _t(torch_dev, r), W, H, bm, bmin, True)
    _same_file(data, nbits, want, want_bits)


@pytest.mark.slow
def test_pack_c3_and_round_trip(torch_dev, ctx):
    """C3: 78 k transforms over 77 chunks; file -> native parser -> GPU
    decode equals the decode of the stream itself."""
    log("pack c3")
    img = synth.workload("c3")
    got = ctx.encode(torch_dev.from_numpy(img).cuda(), 32, 4, [150, 100, 64])
    rec = fb.to_records(got)
    want, want_bits = bs.pack(rec, 4096, 4096, 32, 4, isometries=True)
    data, nbits = _gpu_file(torch_dev, ctx, got, 4096, 4096, 32, 4, True)
    _same_file(data, nbits, want, want_bits)
    back, info = fb.fe_unpack(data, nbits)
    assert back.tobytes() == rec.tobytes()
    d1 = ctx.decode(got, 4096, 4096, 32, 4).cpu().numpy()
    d2 = ctx.decode(_t(torch_dev, back), 4096, 4096, 32, 4).cpu().numpy()
    np.testing.assert_array_equal(d1, d2)


def test_round_trip_through_decoder(torch_dev, ctx):
    img = synth.workload("c2")
    got = ctx.encode(torch_dev.from_numpy(img).cuda(), 16, 4, [300, 200])
    data, nbits = _gpu_file(torch_dev, ctx, got, 512, 512, 16, 4, True)
    back, info = fb.fe_unpack(data, nbits)
    assert info == {"width": 512, "height": 512, "b_max": 16, "b_min": 4, "isometry": True}
    dec = ctx.decode(_t(torch_dev, back), 512, 512, 16, 12).cpu().numpy()
    np.testing.assert_array_equal(dec, odec.decode(mns.encode(img, 16, 4, [300, 200]), 512, 512, 16, 12))


def test_pack_errors(torch_dev, ctx):
    torch = torch_dev
    img = synth.workload("c1")
    got = ctx.encode(torch.from_numpy(img).cuda(), 8, 4, [600])
    # isometries other than the identity need the isometry flag
    with pytest.raises(fb.FeError) as ei:
        fb.fe_pack(ctx.handle, got, 64, 64, 8, 4, isometry=False)
    assert ei.value.status == fb.FE_ERR_INVALID
    # a stream out of encoder order
    rec = fb.to_records(got)
    perm = np.random.default_rng(1).permutation(rec.size)
    with pytest.raises(fb.FeError) as ei:
        fb.fe_pack(ctx.handle, _t(torch, rec[perm]), 64, 64, 8, 4)
    assert ei.value.status == fb.FE_ERR_INVALID
    # phase-2 differences wider than their codes (valid for the decoder)
    wide = random_stream(64, 48, 16, 4, 3, bounded=False)
    assert np.abs(wide["dlum"][wide["flags"] != 0]).max() > 31
    with pytest.raises(fb.FeError) as ei:
        fb.fe_pack(ctx.handle, _t(torch, wide), 64, 48, 16, 4)
    assert ei.value.status == fb.FE_ERR_INVALID
    # too small an output buffer
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(fb.FeError) as ei:
        fb.fe_pack(ctx.handle, got, 64, 64, 8, 4, out=small)
    assert ei.value.status == fb.FE_ERR_CAPACITY
    # an empty stream is a header with no codes... for an image with no tiles
    # there is none: a 64 x 64 image always has transforms
    assert fb.fe_pack_bound(0) == 8
