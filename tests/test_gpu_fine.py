"""GPU parity of quadtrees that reach the paper's 2 x 2 ranges (Sec. 3.3:
four levels, 16 x 16 to 2 x 2), through the C ABI.

The encoder for b_min = 2 (the fused kernel down to 4 x 4, then the 2 x 2
level with domain means formed from pixels at either phase) must give the
oracle's stream byte for byte, alone, in a batch and replayed as a plan; both
decoders, zoom decoding and the compressed file must take such streams (the
tile decoder with its 2 x 2 pieces decoded by a kernel of their own)."""
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


def dev(torch, img):
    return torch.from_numpy(np.ascontiguousarray(img)).cuda()


def _t(torch, rec):
    return torch.from_numpy(np.ascontiguousarray(rec).view(np.uint8).reshape(-1, 16).copy()).cuda()


def assert_same_stream(got, want):
    assert got.size == want.size, (got.size, want.size)
    gb = got.view(np.uint8).reshape(-1, 16)
    wb = np.ascontiguousarray(want).view(np.uint8).reshape(-1, 16)
    bad = np.flatnonzero(np.any(gb != wb, axis=1))
    assert bad.size == 0, f"{bad.size} records differ; first {bad[0]}: got {got[bad[0]]} want {want[bad[0]]}"


CASES = [
    # name, image maker, b_max, thresholds
    ("c1 8->2", lambda: synth.workload("c1"), 8, [600, 300]),
    ("c1 16->2", lambda: synth.workload("c1"), 16, [900, 600, 300]),
    ("c1 4->2", lambda: synth.workload("c1"), 4, [300]),
    ("c2 16->2", lambda: synth.workload("c2"), 16, [300, 200, 100]),
    ("noise 48x80", lambda: synth.noise_1f(80, 48, 31), 16, [400, 250, 120]),
    ("noise 2bmax", lambda: synth.noise_1f(32, 32, 32), 16, [200, 100, 50]),
    ("pw 8->2", lambda: synth.piecewise_smooth(96, 136, 33, cells=30), 8, [150, 60]),
    ("zero thresholds", lambda: synth.noise_1f(64, 64, 34), 16, [0, 0, 0]),
    ("ramp", lambda: synth.ramp(64, 48), 16, [1, 1, 1]),
    ("flat", lambda: np.full((32, 64), 91, np.uint8), 16, [1, 1, 1]),
]


@pytest.mark.parametrize("name,make,b_max,thr", CASES, ids=[c[0] for c in CASES])
def test_encode(torch_dev, ctx, name, make, b_max, thr):
    log(f"fine encode {name}")
    img = make()
    for phase2 in (True, False):
        want = mns.encode(img, b_max, 2, thr, phase2=phase2)
        got = fb.to_records(ctx.encode(dev(torch_dev, img), b_max, 2, thr, phase2=phase2))
        assert_same_stream(got, want)


def test_encode_identity_only(torch_dev, ctx):
    log("fine encode identity only")
    img = synth.workload("c2")
    want = mns.encode(img, 16, 2, [300, 200, 100], isometries=False)
    got = fb.to_records(ctx.encode(dev(torch_dev, img), 16, 2, [300, 200, 100], identity_only=True))
    assert_same_stream(got, want)


def test_encode_strided(torch_dev, ctx):
    log("fine encode strided image")
    img = synth.noise_1f(32, 64, 35)
    buf = np.zeros((32, 80), np.uint8)
    buf[:, :64] = img
    t = dev(torch_dev, buf)[:, :64]
    got = fb.to_records(ctx.encode(t, 8, 2, [300, 150]))
    assert_same_stream(got, mns.encode(img, 8, 2, [300, 150]))


def test_paper_tree_has_every_kind(torch_dev, ctx):
    # the paper's configuration on the 512 x 512 workload: phase-2 records at
    # levels 1-3 (the last over 2 x 2 sub-blocks) and 2 x 2 leaves
    rec = mns.encode(synth.workload("c2"), 16, 2, [300, 200, 100])
    p2 = (rec["flags"] & 1) == 1
    assert set(rec["level"][p2].tolist()) == {0, 1, 2}
    assert np.any(rec["level"] == 3) and np.any(rec["dx"] % 2)


@pytest.mark.parametrize("W,H,bm,seed", [(64, 48, 16, 41), (112, 80, 8, 42), (64, 64, 4, 43), (264, 136, 8, 44)])
def test_decode_random(torch_dev, ctx, W, H, bm, seed):
    log(f"fine decode random {W}x{H} b{bm}/2")
    rec = random_stream(W, H, bm, 2, seed)
    assert np.any(bm >> rec["level"].astype(np.int64) == 2)
    start = np.random.default_rng(seed).integers(0, 256, (H, W)).astype(np.uint8)
    t = _t(torch_dev, rec)
    want = odec.decode(rec, W, H, bm, 3, start=start)
    try:
        for mode, used in ((fb.FE_DECODE_AUTO, fb.FE_DECODE_TILES), (fb.FE_DECODE_RECORDS, fb.FE_DECODE_RECORDS)):
            ctx.decode_mode(mode)
            got = ctx.decode(t, W, H, bm, 3, start=dev(torch_dev, start)).cpu().numpy()
            assert ctx.decode_last() == used
            np.testing.assert_array_equal(got, want)
    finally:
        ctx.decode_mode(fb.FE_DECODE_AUTO)


def test_decode_encoded(torch_dev, ctx):
    log("fine decode c2 16->2")
    img = synth.workload("c2")
    rec = mns.encode(img, 16, 2, [300, 200, 100])
    got = ctx.decode(_t(torch_dev, rec), 512, 512, 16, 8).cpu().numpy()
    assert ctx.decode_last() == fb.FE_DECODE_TILES
    np.testing.assert_array_equal(got, odec.decode(rec, 512, 512, 16, 8))


@pytest.mark.parametrize("bm,z,tiles", [(8, 2, True), (8, 4, True), (16, 2, True), (4, 8, True)])
def test_zoom(torch_dev, ctx, bm, z, tiles):
    # zoomed by 2 or more, every block is at least 4 x 4 and the tile decoder takes the stream
    log(f"fine zoom b{bm} x{z}")
    img = synth.noise_1f(32, 32, 36)
    thr = {4: [200], 8: [300, 150], 16: [400, 300, 150]}[bm]
    rec = mns.encode(img, bm, 2, thr)
    got = ctx.decode_zoom(_t(torch_dev, rec), 32, 32, bm, z, 5).cpu().numpy()
    assert ctx.decode_last() == (fb.FE_DECODE_TILES if tiles else fb.FE_DECODE_RECORDS)
    np.testing.assert_array_equal(got, odec.decode(odec.zoom(rec, z), 32 * z, 32 * z, bm * z, 5))


@pytest.mark.parametrize("iso", [True, False])
def test_pack(torch_dev, ctx, iso):
    log(f"fine pack iso={iso}")
    img = synth.workload("c2")
    rec = mns.encode(img, 16, 2, [300, 200, 100], isometries=iso)
    want, want_bits = bs.pack(rec, 512, 512, 16, 2, isometries=iso)
    out, nbits = fb.fe_pack(ctx.handle, _t(torch_dev, rec), 512, 512, 16, 2, isometry=iso)
    assert nbits == want_bits
    data = out.cpu().numpy().tobytes()[: (nbits + 7) // 8]
    assert data == want
    back, info = fb.fe_unpack(data, nbits)
    assert info["b_min"] == 2 and info["b_max"] == 16
    assert back.tobytes() == np.ascontiguousarray(rec).tobytes()


@pytest.mark.parametrize("b_max,thr", [(16, [300, 200, 100]), (8, [300, 150])])
def test_batch(torch_dev, ctx, b_max, thr):
    # images of several sizes in one launch; each stream equals the oracle's
    log(f"fine batch b{b_max}")
    imgs = [synth.workload("c1"), synth.noise_1f(48, 80, 61), synth.piecewise_smooth(96, 64, 62, cells=12),
            synth.noise_1f(32, 32, 63), synth.workload("c2")]
    views = [dev(torch_dev, im) for im in imgs]
    out, offs, n = ctx.encode_batch(views, b_max, 2, thr)
    offs = offs.cpu().numpy()
    got = fb.to_records(out[:n])
    for k, im in enumerate(imgs):
        assert_same_stream(got[offs[k]:offs[k + 1]], mns.encode(im, b_max, 2, thr))


@pytest.mark.parametrize("timing", [False, True])
def test_plan_replays(torch_dev, ctx, timing):
    # the batch recorded as a HIP graph (zeroing kernel, EXT encode, 2 x 2
    # level, ordering): every replay equals the eager batch and the oracle,
    # with other work and synchronisations between replays
    torch = torch_dev
    log(f"fine plan timing={timing}")
    imgs = [synth.workload("c1"), synth.noise_1f(48, 80, 71), synth.workload("c2")]
    views = [dev(torch, im) for im in imgs]
    thr = [300, 200, 100]
    out, offs, n = ctx.encode_batch(views, 16, 2, thr)
    eager = out[:n].cpu().numpy().tobytes()
    eager_offs = offs.cpu().numpy()
    got = fb.to_records(out[:n])
    for k, im in enumerate(imgs):
        assert_same_stream(got[eager_offs[k]:eager_offs[k + 1]], mns.encode(im, 16, 2, thr))
    out2 = torch.empty_like(out)
    offs2 = torch.zeros_like(offs)
    fb.fe_timing_enable(ctx.handle, timing)
    try:
        with fb.Plan(ctx, views, 16, 2, thr, out2, offs2) as plan:
            for _ in range(3):
                out2.zero_()
                plan.launch()
                torch.cuda.synchronize()
                assert np.array_equal(offs2.cpu().numpy(), eager_offs)
                assert out2[:n].cpu().numpy().tobytes() == eager
                ctx.encode_batch(views[:1], 8, 2, [300, 150])   # other work in between
                torch.cuda.synchronize()
    finally:
        fb.fe_timing_enable(ctx.handle, False)
        fb.fe_timing_read(ctx.handle)


def test_paths_that_do_not_take_2x2(torch_dev, ctx):
    log("fine rejections")
    img = dev(torch_dev, synth.workload("c1"))
    with pytest.raises(fb.FeError):
        ctx.encode(img, 8, 2, [300, 150], full_search=True)
    with pytest.raises(fb.FeError):
        ctx.encode(img, 8, 2, [300, 150], local_search=True)
    with pytest.raises(fb.FeError):
        ctx.encode(img, 32, 2, [1, 1, 1, 1])        # five levels
