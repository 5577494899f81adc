"""GPU parity of the MNS path against the CPU oracle, through the C ABI.

Integer work is compared bit for bit: the domain image, the moments, and the
whole transform stream (every field of every record, in stream order).
Decoding is exact integer arithmetic on both sides, so decoded pixels are
compared exactly as well (which implies the +-1 grey-level and 0.01 dB PSNR
bars).
"""
import sys

import numpy as np
import pytest

from oracle import decode as odec
from oracle import metrics, mns
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


def dev(torch, img):
    return torch.from_numpy(np.ascontiguousarray(img)).cuda()


def gpu_stream(torch, ctx, img, b_max, b_min, thr, phase2=True):
    out = ctx.encode(dev(torch, img), b_max, b_min, thr, phase2=phase2)
    torch.cuda.synchronize()
    return fb.to_records(out)


def assert_same_stream(got, want):
    assert got.size == want.size, (got.size, want.size)
    gb = got.view(np.uint8).reshape(-1, 16)
    wb = np.ascontiguousarray(want).view(np.uint8).reshape(-1, 16)
    bad = np.flatnonzero(np.any(gb != wb, axis=1))
    assert bad.size == 0, f"{bad.size} records differ; first {bad[0]}: got {got[bad[0]]} want {want[bad[0]]}"


# ------------------------------------------------------------------ steps
@pytest.mark.parametrize("shape", [(64, 64), (20, 36), (2, 2), (6, 10), (512, 512), (130, 258)])
def test_downsample(torch_dev, ctx, shape):
    log(f"downsample {shape}")
    rng = np.random.default_rng(shape[0] * 1000 + shape[1])
    img = rng.integers(0, 256, shape).astype(np.uint8)
    stride = (shape[1] + 3) // 4 * 4
    buf = np.zeros((shape[0], stride), np.uint8)
    buf[:, : shape[1]] = img
    t = dev(torch_dev, buf)[:, : shape[1]]
    got = ctx.downsample(t).cpu().numpy()
    np.testing.assert_array_equal(got, mns.downsample(img))


@pytest.mark.parametrize("B", [4, 8, 16, 32])
def test_range_moments(torch_dev, ctx, B):
    log(f"moments B={B}")
    rng = np.random.default_rng(B)
    for (H, W) in [(2 * B, 2 * B), (4 * B, 6 * B), (160, 96)]:
        if H % B or W % B:
            continue
        img = rng.integers(0, 256, (H, W)).astype(np.uint8)
        ys, xs = np.mgrid[0:H:B, 0:W:B]
        xs, ys = xs.ravel(), ys.ravel()
        xy = torch_dev.from_numpy((xs | (ys << 16)).astype(np.int32)).cuda()
        got = ctx.range_moments(dev(torch_dev, img), B, xy).cpu().numpy().view(np.uint32).astype(np.int64)
        want = mns.range_moments(img.astype(np.int64), mns.downsample(img), xs, ys, B)
        np.testing.assert_array_equal(got[:, 0], want["sr"])
        np.testing.assert_array_equal(got[:, 1], want["srr"])
        np.testing.assert_array_equal(got[:, 2], want["sd"])
        np.testing.assert_array_equal(got[:, 3], want["sdd"])
        np.testing.assert_array_equal(got[:, 4:], want["srd"])


def test_range_moments_extremes(torch_dev, ctx):
    """All-255 images give the largest sums (32x32: Sum r d = 1024 * 255^2)."""
    for B in (4, 32):
        img = np.full((2 * B, 2 * B), 255, np.uint8)
        xy = torch_dev.tensor([0, B, B << 16, B | (B << 16)], dtype=torch_dev.int32).cuda()
        got = ctx.range_moments(dev(torch_dev, img), B, xy).cpu().numpy().view(np.uint32)
        n = B * B
        assert np.all(got[:, 0] == 255 * n) and np.all(got[:, 1] == 255 * 255 * n)
        assert np.all(got[:, 4:] == 255 * 255 * n)


# ------------------------------------------------------------------ encode
CASES = [
    # name, image maker, b_max, b_min, thresholds
    ("c1", lambda: synth.workload("c1"), 8, 4, [600]),
    ("c2", lambda: synth.workload("c2"), 16, 4, [300, 200]),
    ("noise96x160_16_4", lambda: synth.noise_1f(96, 160, 11), 16, 4, [250, 150]),
    ("noise200x72_8_4", lambda: synth.noise_1f(200, 72, 12), 8, 4, [400]),
    ("pw192_32_4", lambda: synth.piecewise_smooth(192, 256, 13, cells=40), 32, 4, [120, 90, 60]),
    ("pw64x448_32_8", lambda: synth.piecewise_smooth(64, 448, 14, cells=20), 32, 8, [200, 100]),
    ("noise128_16_8", lambda: synth.noise_1f(128, 128, 15), 16, 8, [300]),
    ("noise64_32_16", lambda: synth.noise_1f(64, 96, 16), 32, 16, [200]),
    ("noise64_16_16", lambda: synth.noise_1f(64, 48, 17), 16, 16, []),
    ("noise16_4_4", lambda: synth.noise_1f(16, 24, 18), 4, 4, []),
    ("min32_16_4", lambda: synth.noise_1f(32, 32, 19), 16, 4, [300, 200]),
    ("thin_32x1024", lambda: synth.noise_1f(32, 1024, 20), 16, 4, [300, 200]),
    ("ramp", lambda: synth.ramp(64, 64), 16, 4, [1, 1]),
    ("ramp_t0", lambda: synth.ramp(64, 64), 16, 4, [0, 0]),
    ("flat", lambda: synth.flat(64, 64, 200), 16, 4, [1, 1]),
    ("all_split", lambda: synth.noise_1f(128, 128, 21), 16, 4, [0, 0]),
    ("all_accept", lambda: synth.noise_1f(128, 128, 22), 16, 4, [10 ** 9, 10 ** 9]),
    ("c2_lowthr", lambda: synth.workload("c2"), 16, 4, [40, 20]),
]


@pytest.mark.parametrize("name,make,b_max,b_min,thr", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("phase2", [True, False], ids=["mns", "nosearch"])
def test_encode_stream(torch_dev, ctx, name, make, b_max, b_min, thr, phase2):
    log(f"encode {name} phase2={phase2}")
    img = make()
    want = mns.encode(img, b_max, b_min, thr, phase2=phase2)
    got = gpu_stream(torch_dev, ctx, img, b_max, b_min, thr, phase2)
    assert_same_stream(got, want)


def test_encode_strided_input(torch_dev, ctx):
    img = synth.noise_1f(96, 128, 31)
    buf = np.zeros((96, 160), np.uint8)
    buf[:, :128] = img
    t = dev(torch_dev, buf)[:, :128]
    got = fb.to_records(ctx.encode(t, 16, 4, [300, 200]))
    assert_same_stream(got, mns.encode(img, 16, 4, [300, 200]))


def test_encode_huge_pitch(torch_dev, ctx):
    """A 32 MiB row pitch: the encoder reads a workgroup's region through a
    buffer resource when the region spans under 2 GiB (tile shapes with 48
    region rows) and through global addresses otherwise (80 rows and more);
    every shape gives the oracle's stream."""
    H, W, pitch = 48, 64, 1 << 25
    img = synth.noise_1f(H, W, 57)
    want = mns.encode(img, 16, 4, [300, 200])
    buf = torch_dev.zeros((H - 1) * pitch + W, dtype=torch_dev.uint8, device="cuda")
    for r in range(H):
        buf[r * pitch:r * pitch + W].copy_(torch_dev.from_numpy(img[r].copy()))
    t = buf.as_strided((H, W), (pitch, 1))
    assert t.stride(0) == pitch
    try:
        for gx, gy in fb.fe_tile_shapes(16, 4):
            log(f"  shape {gx}x{gy} pitch {pitch}")
            fb.fe_set_tile_shape(ctx.handle, 16, 4, gx, gy)
            got = fb.to_records(ctx.encode(t, 16, 4, [300, 200]))
            assert_same_stream(got, want)
    finally:
        fb.fe_set_tile_shape(ctx.handle, 16, 4, 0, 0)
    del t, buf


@pytest.mark.parametrize("b_max,b_min,thr,H,W", [
    (16, 4, [300, 200], 320, 224), (16, 8, [300], 160, 96), (16, 16, [], 96, 48),
    (32, 4, [150, 100, 64], 256, 320), (32, 8, [200, 100], 192, 128), (32, 16, [200], 96, 64),
    (8, 4, [400], 104, 88), (4, 4, [], 36, 20),
])
@pytest.mark.parametrize("layout", ["aligned", "offset4"])
def test_encode_every_tile_shape(torch_dev, ctx, b_max, b_min, thr, H, W, layout):
    """The stream depends neither on the workgroup tile shape nor on the
    input's placement: a dense image, and a view at byte offset 4 with pitch
    W + 12 (not 16-byte aligned)."""
    img = synth.noise_1f(H, W, 41 + b_max + H)
    want = mns.encode(img, b_max, b_min, thr)
    if layout == "aligned":
        t = dev(torch_dev, img)
    else:
        buf = np.zeros((H, W + 12), np.uint8)
        buf[:, 4:W + 4] = img
        t = dev(torch_dev, buf)[:, 4:W + 4]
    shapes = fb.fe_tile_shapes(b_max, b_min)
    assert shapes
    try:
        for gx, gy in shapes:
            log(f"  shape {gx}x{gy} {layout}")
            fb.fe_set_tile_shape(ctx.handle, b_max, b_min, gx, gy)
            got = fb.to_records(ctx.encode(t, b_max, b_min, thr))
            assert_same_stream(got, want)
    finally:
        fb.fe_set_tile_shape(ctx.handle, b_max, b_min, 0, 0)


def test_misaligned_input_rejected(torch_dev, ctx):
    """Images must be 4-byte aligned with a pitch that is a multiple of 4."""
    buf = dev(torch_dev, np.zeros((64, 64 + 13), np.uint8))
    for view in (buf[:, 3:67], buf[:, :64]):          # offset 3; pitch 77
        with pytest.raises(fb.FeError) as ei:
            ctx.encode(view, 16, 4, [300, 200])
        assert ei.value.status == fb.FE_ERR_SHAPE


def test_capacity_error(torch_dev, ctx):
    img = synth.workload("c1")
    want = mns.encode(img, 8, 4, [600])
    small = torch_dev.empty((want.size - 1, 16), dtype=torch_dev.uint8, device="cuda")
    with pytest.raises(fb.FeError) as ei:
        ctx.encode(dev(torch_dev, img), 8, 4, [600], out=small)
    assert ei.value.status == fb.FE_ERR_CAPACITY
    assert str(want.size) in str(ei.value)


def test_deterministic(torch_dev, ctx):
    img = synth.workload("c2")
    a = gpu_stream(torch_dev, ctx, img, 16, 4, [300, 200])
    b = gpu_stream(torch_dev, ctx, img, 16, 4, [300, 200])
    assert a.tobytes() == b.tobytes()


@pytest.mark.slow
def test_encode_c3_full(torch_dev, ctx):
    log("encode c3 (4096x4096, 32->4)")
    img = synth.workload("c3")
    want = mns.encode(img, 32, 4, [150, 100, 64])
    got = gpu_stream(torch_dev, ctx, img, 32, 4, [150, 100, 64])
    assert_same_stream(got, want)


@pytest.mark.parametrize("H,W,b_max,b_min,thr,path", [
    (1024, 2048, 8, 4, [400], "per-chunk sums (128 chunks)"),
    (4096, 4160, 4, 4, [], "scan kernel (4160 chunks)"),
])
def test_ordering_paths(torch_dev, ctx, H, W, b_max, b_min, thr, path):
    """The ordering takes one kernel up to 64 chunks of 256 tiles (every
    other test image), chunk counts summed by each workgroup up to 4096, and
    a separate scan beyond; the stream is the same on each."""
    log(f"encode {H}x{W} b{b_max}/{b_min}: {path}")
    img = synth.noise_1f(H, W, 77 + b_max)
    want = mns.encode(img, b_max, b_min, thr)
    got = gpu_stream(torch_dev, ctx, img, b_max, b_min, thr)
    assert_same_stream(got, want)


def test_context_reuse_across_ordering_paths(torch_dev):
    """One context encodes a sequence whose chunk counts go up and down (the
    one-kernel ordering, summed chunk counts, the scan beyond 4096 chunks, a
    16 -> 2 tree, a batch), so its scratch buffers grow and are reused with
    stale contents; every stream must equal the same call on a fresh
    context."""
    cases = [
        ("single 512", [synth.noise_1f(512, 512, 301)], 16, 4, [300, 200]),
        ("scan 4160 chunks", [synth.noise_1f(4096, 4160, 302)], 4, 4, []),
        ("single 256", [synth.piecewise_smooth(256, 256, 303)], 16, 4, [300, 200]),
        ("16 -> 2", [synth.noise_1f(640, 384, 304)], 16, 2, [300, 200, 100]),
        ("batch", [synth.noise_1f(256 + 64 * k, 512, 305 + k) for k in range(6)], 16, 4, [300, 200]),
        ("sums 128 chunks", [synth.noise_1f(1024, 2048, 311)], 8, 4, [400]),
        ("single 512 again", [synth.noise_1f(512, 512, 301)], 16, 4, [300, 200]),
    ]
    shared = fb.Context(0)
    try:
        for name, imgs, b_max, b_min, thr in cases:
            log(f"context reuse: {name}")
            t_imgs = [dev(torch_dev, im) for im in imgs]
            fresh = fb.Context(0)
            try:
                if len(imgs) == 1:
                    got = fb.to_records(shared.encode(t_imgs[0], b_max, b_min, thr))
                    want = fb.to_records(fresh.encode(t_imgs[0], b_max, b_min, thr))
                else:
                    o1, f1, n1 = shared.encode_batch(t_imgs, b_max, b_min, thr)
                    o2, f2, n2 = fresh.encode_batch(t_imgs, b_max, b_min, thr)
                    torch_dev.cuda.synchronize()
                    assert f1.cpu().numpy().tolist() == f2.cpu().numpy().tolist(), name
                    got, want = fb.to_records(o1[:n1]), fb.to_records(o2[:n2])
                torch_dev.cuda.synchronize()
            finally:
                fresh.close()
            assert got.tobytes() == want.tobytes(), name
    finally:
        shared.close()


# ------------------------------------------------------------------ batch
def test_encode_batch_matches_single(torch_dev, ctx):
    rng = np.random.default_rng(5)
    imgs = []
    for k in range(12):
        side_w = int(rng.integers(2, 12)) * 32
        side_h = int(rng.integers(2, 12)) * 32
        imgs.append(synth.noise_1f(side_h, side_w, 100 + k) if k % 2 else
                    synth.piecewise_smooth(side_h, side_w, 100 + k))
    t_imgs = [dev(torch_dev, im) for im in imgs]
    out, offsets, n = ctx.encode_batch(t_imgs, 16, 4, [300, 200])
    torch_dev.cuda.synchronize()
    offs = offsets.cpu().numpy()
    assert offs[-1] == n
    recs = fb.to_records(out[:n])
    for k, im in enumerate(imgs):
        assert_same_stream(recs[offs[k]:offs[k + 1]], mns.encode(im, 16, 4, [300, 200]))
    # the same batch again reuses the device table and block descriptors;
    # after another call with a different table it is rebuilt
    first = out[:n].cpu().numpy().tobytes()
    for other in (None, [t_imgs[0]], None):
        if other is not None:
            ctx.encode_batch(other, 16, 4, [300, 200])
        out2, offs2, n2 = ctx.encode_batch(t_imgs, 16, 4, [300, 200])
        torch_dev.cuda.synchronize()
        assert n2 == n and out2[:n2].cpu().numpy().tobytes() == first
        np.testing.assert_array_equal(offs2.cpu().numpy(), offs)


def test_plan_replays_match_eager(torch_dev, ctx):
    """A recorded batch (HIP graph) gives the eager batch's output on every
    replay, with other device work and synchronisations in between, and
    follows new contents written into the same image buffers."""
    rng = np.random.default_rng(9)
    shapes = [(int(rng.integers(2, 9)) * 32, int(rng.integers(2, 9)) * 32) for _ in range(6)]
    imgs = [synth.noise_1f(h, w, 300 + k) if k % 2 else synth.piecewise_smooth(h, w, 300 + k)
            for k, (h, w) in enumerate(shapes)]
    thr = [300, 200]
    t_imgs = [dev(torch_dev, im) for im in imgs]
    out_e, offs_e, n_e = ctx.encode_batch(t_imgs, 16, 4, thr)
    want = out_e[:n_e].cpu().numpy().tobytes()
    want_offs = offs_e.cpu().numpy()
    cap = out_e.shape[0]
    out = torch_dev.zeros((cap, 16), dtype=torch_dev.uint8, device="cuda")
    offs = torch_dev.zeros(len(imgs) + 1, dtype=torch_dev.int64, device="cuda")
    with fb.Plan(ctx, t_imgs, 16, 4, thr, out, offs) as plan:
        for rep in range(4):
            log(f"  replay {rep}")
            out.fill_(0)
            offs.fill_(0)
            plan.launch()
            torch_dev.cuda.synchronize()
            got_offs = offs.cpu().numpy()
            np.testing.assert_array_equal(got_offs, want_offs)
            assert out[:n_e].cpu().numpy().tobytes() == want, f"replay {rep} differs"
            ctx.encode_batch(t_imgs, 16, 4, thr)               # eager work between replays
            torch_dev.cuda.synchronize()
        new = [synth.noise_1f(h, w, 400 + k) for k, (h, w) in enumerate(shapes)]
        for k, im in enumerate(new):
            t_imgs[k].copy_(torch_dev.from_numpy(im))
        plan.launch()
        torch_dev.cuda.synchronize()
        offs_h = offs.cpu().numpy()
        recs = fb.to_records(out[: int(offs_h[-1])])
        for k, im in enumerate(new):
            assert_same_stream(recs[offs_h[k]:offs_h[k + 1]], mns.encode(im, 16, 4, thr))
    # a plan created while timing is on times each launch's kernels
    fb.fe_timing_read(ctx.handle)
    fb.fe_timing_enable(ctx.handle, True)
    try:
        with fb.Plan(ctx, t_imgs, 16, 4, thr, out, offs) as plan:
            for _ in range(3):
                plan.launch()
            torch_dev.cuda.synchronize()
            ms, cnt = fb.fe_timing_read(ctx.handle)
            assert cnt[fb.FE_TIMING_ENCODE] == 3 and cnt[fb.FE_TIMING_SCATTER] == 3
            assert ms[fb.FE_TIMING_ENCODE] > 0 and ms[fb.FE_TIMING_SCATTER] > 0
            fb.fe_timing_enable(ctx.handle, False)
            plan.launch()                                      # untimed launch after timing is off
            torch_dev.cuda.synchronize()
            assert out[: int(offs.cpu().numpy()[-1])].cpu().numpy().tobytes() == recs.tobytes()
            assert fb.fe_timing_read(ctx.handle)[1][fb.FE_TIMING_ENCODE] == 0
    finally:
        fb.fe_timing_enable(ctx.handle, False)


def test_timing_select(torch_dev, ctx):
    """fe_timing_select limits the timed launches to the chosen slots."""
    img = dev(torch_dev, synth.workload("c2"))
    fb.fe_timing_read(ctx.handle)
    try:
        for mask, want in ((1 << fb.FE_TIMING_ENCODE, (2, 0)), (1 << fb.FE_TIMING_SCATTER, (0, 2)),
                           (0xffffffff, (2, 2))):
            fb.fe_timing_select(ctx.handle, mask)
            fb.fe_timing_enable(ctx.handle, True)
            for _ in range(2):
                ctx.encode(img, 16, 4, [300, 200])
            torch_dev.cuda.synchronize()
            fb.fe_timing_enable(ctx.handle, False)
            ms, cnt = fb.fe_timing_read(ctx.handle)
            assert (cnt[fb.FE_TIMING_ENCODE], cnt[fb.FE_TIMING_SCATTER]) == want
            assert all(ms[k] > 0 for k in (fb.FE_TIMING_ENCODE, fb.FE_TIMING_SCATTER) if cnt[k])
    finally:
        fb.fe_timing_select(ctx.handle, 0xffffffff)
        fb.fe_timing_enable(ctx.handle, False)


# ------------------------------------------------------------------ decode
@pytest.mark.parametrize("name,b_max,b_min,thr,iters", [
    ("c1", 8, 4, [600], 12),
    ("c2", 16, 4, [300, 200], 12),
])
def test_decode(torch_dev, ctx, name, b_max, b_min, thr, iters):
    log(f"decode {name}")
    img = synth.workload(name)
    H, W = img.shape
    rec = mns.encode(img, b_max, b_min, thr)
    t = torch_dev.from_numpy(np.ascontiguousarray(rec).view(np.uint8).reshape(-1, 16).copy()).cuda()
    for start in (None, np.zeros((H, W), np.uint8), img):
        got = ctx.decode(t, W, H, b_max, iters, start=None if start is None else dev(torch_dev, start))
        got = got.cpu().numpy()
        want = odec.decode(rec, W, H, b_max, iters, start=start)
        np.testing.assert_array_equal(got, want)
        assert abs(metrics.psnr(img, got) - metrics.psnr(img, want)) <= 0.01


def test_decode_zero_iterations_and_bad_input(torch_dev, ctx):
    img = synth.workload("c1")
    rec = mns.encode(img, 8, 4, [600])
    t = torch_dev.from_numpy(np.ascontiguousarray(rec).view(np.uint8).reshape(-1, 16).copy()).cuda()
    got = ctx.decode(t, 64, 64, 8, 0).cpu().numpy()
    assert np.all(got == 128)
    bad = rec.copy()
    bad[3]["x"] = 64          # outside the image
    tb = torch_dev.from_numpy(np.ascontiguousarray(bad).view(np.uint8).reshape(-1, 16).copy()).cuda()
    with pytest.raises(fb.FeError) as ei:
        ctx.decode(tb, 64, 64, 8, 2)
    assert ei.value.status == fb.FE_ERR_INVALID




def test_autotune_picks_a_built_shape(torch_dev, ctx):
    """The autotuner times every built tile shape on the caller's batch and
    selects the fastest for the context; the streams it then produces equal
    the oracle's (the shape never changes the output)."""
    torch = torch_dev
    rng = np.random.default_rng(11)
    imgs = []
    for k in range(6):
        H, W = (int(v) for v in rng.choice([128, 160, 256, 352], 2))
        imgs.append(synth.noise_1f(H, W, 300 + k) if k % 2 else synth.piecewise_smooth(H, W, 300 + k, cells=12))
    views = [dev(torch, im) for im in imgs]
    thr = [300, 200]
    params = fb.make_params(16, 4, thr)
    cap = sum(fb.fe_max_transforms(im.shape[1], im.shape[0], 4) for im in imgs)
    out = torch.empty((cap, 16), dtype=torch.uint8, device="cuda")
    offsets = torch.zeros(len(imgs) + 1, dtype=torch.int64, device="cuda")
    try:
        (gx, gy), ms = fb.fe_autotune(ctx.handle, views, params, out, offsets, reps=2)
        log(f"  autotune: {gx}x{gy}, {ms * 1e3:.1f} us")
        assert (gx, gy) in fb.fe_tile_shapes(16, 4)
        assert ms > 0
        assert fb.fe_get_tile_shape(ctx.handle, 16, 4) == (gx, gy)
        got, offs, n = ctx.encode_batch(views, 16, 4, thr)
        o = offs.cpu().numpy()
        recs = fb.to_records(got[:n])
        for k, im in enumerate(imgs):
            assert_same_stream(recs[o[k]:o[k + 1]], mns.encode(im, 16, 4, thr))
    finally:
        fb.fe_set_tile_shape(ctx.handle, 16, 4, 0, 0)
