"""Continuous-batching server: every result equals the image encoded alone
(and the oracle), whatever else shares the steps -- mixed sizes, a tight
device budget that forces admission to wait, and large images spread over
many steps."""
import sys
import time

import numpy as np
import pytest

from oracle import mns
from paper_1501_02894_amd import binding as fb
from paper_1501_02894_amd import synth

pytestmark = pytest.mark.gpu
THR = [300, 200]


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


def mixed_images(n, seed, lo=64, hi=1024):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        w = int(rng.integers(lo // 16, hi // 16 + 1)) * 16
        h = int(rng.integers(lo // 16, hi // 16 + 1)) * 16
        out.append(synth.noise_1f(h, w, seed * 1000 + k) if k % 2 else
                   synth.piecewise_smooth(h, w, seed * 1000 + k))
    return out


def alone(torch, ctx, img):
    return fb.to_records(ctx.encode(torch.from_numpy(img).cuda(), 16, 4, THR))


def drain(srv, reqs, timeout=120.0):
    results = {}
    t0 = time.time()
    while len(results) < len(reqs):
        for k, r in enumerate(reqs):
            if k in results:
                continue
            done, recs, lat = srv.poll(r)
            if done:
                results[k] = (recs, lat)
        assert time.time() - t0 < timeout, f"server did not finish: {len(results)}/{len(reqs)}"
        time.sleep(0.0005)
    return results


def test_server_mix_equals_alone(torch_dev, ctx):
    imgs = mixed_images(24, 1)
    log(f"server mix of {len(imgs)} images")
    with fb.Server(16, 4, THR, max_slots=64, step_blocks=256) as srv:
        reqs = [srv.submit(im) for im in imgs]
        res = drain(srv, reqs)
        st = srv.stats()
    assert st["completed"] == len(imgs) and st["steps"] >= 1
    for k, im in enumerate(imgs):
        recs, lat = res[k]
        assert lat > 0
        want = alone(torch_dev, ctx, im)
        assert recs.tobytes() == want.tobytes(), f"image {k} differs in the mix"
        if im.size <= 256 * 256:
            assert recs.tobytes() == np.ascontiguousarray(mns.encode(im, 16, 4, THR)).tobytes()


def test_server_tight_budget_and_chunking(torch_dev, ctx):
    imgs = [synth.noise_1f(1024, 1024, 5), synth.piecewise_smooth(64, 64, 6)] + mixed_images(6, 2, 64, 256)
    log("server with a tight budget and 8-block steps")
    # 48 MiB: the 1 MiB-pixel image needs most of it, so the others wait
    with fb.Server(16, 4, THR, hbm_budget=48 << 20, host_budget=64 << 20, max_slots=4, step_blocks=8) as srv:
        reqs = [srv.submit(im) for im in imgs]
        res = drain(srv, reqs)
        st = srv.stats()
    gx, gy = fb.fe_tile_shapes(16, 4)[0]                # the server's (default) tile shape
    blocks = -(-64 // gx) * -(-64 // gy)                # the 1024 x 1024 image's workgroup blocks
    assert blocks > 8 and st["steps"] >= blocks // 8    # spread over several 8-block steps
    for k, im in enumerate(imgs):
        assert res[k][0].tobytes() == alone(torch_dev, ctx, im).tobytes()


def test_server_interleaved_arrivals(torch_dev, ctx):
    imgs = mixed_images(16, 3, 64, 512)
    with fb.Server(16, 4, THR, max_slots=8, step_blocks=64) as srv:
        reqs = []
        for im in imgs:
            reqs.append(srv.submit(im))
            time.sleep(0.0003)
        res = drain(srv, reqs)
    for k, im in enumerate(imgs):
        assert res[k][0].tobytes() == alone(torch_dev, ctx, im).tobytes()


def test_server_errors(torch_dev):
    with fb.Server(16, 4, THR, hbm_budget=16 << 20, host_budget=8 << 20, max_slots=2, step_blocks=16) as srv:
        with pytest.raises(fb.FeError) as ei:
            srv.submit(np.zeros((4096, 4096), np.uint8))     # larger than the host staging
        assert ei.value.status in (fb.FE_ERR_BUSY, fb.FE_ERR_OOM)
        with pytest.raises(fb.FeError) as ei:
            srv.submit(np.zeros((72, 64), np.uint8))         # not a multiple of b_max
        assert ei.value.status == fb.FE_ERR_SHAPE
        r = srv.submit(synth.noise_1f(64, 64, 9))
        done = False
        t0 = time.time()
        while not done:
            done, _, _ = srv.poll(r, fetch=False)
            assert time.time() - t0 < 30
        import ctypes
        n = ctypes.c_size_t(0)
        d = ctypes.c_int(0)
        out = np.empty(1, fb.TRANSFORM_DTYPE)
        st = fb.load().fe_server_poll(srv.handle, r, out.ctypes.data, 1, ctypes.byref(n), ctypes.byref(d), None)
        assert st == fb.FE_ERR_CAPACITY and n.value > 1
        done, recs, _ = srv.poll(r)
        assert done and recs.size == n.value
        with pytest.raises(fb.FeError):
            srv.poll(r)                                       # released


def test_server_wait_reports_each_once(torch_dev, ctx):
    imgs = mixed_images(12, 4, 64, 384)
    with fb.Server(16, 4, THR, max_slots=6, step_blocks=32) as srv:
        assert srv.wait(100) is None                         # nothing submitted
        reqs = [srv.submit(im) for im in imgs]
        seen = []
        t0 = time.time()
        while len(seen) < len(reqs):
            rid = srv.wait(10000)
            if rid is not None:
                seen.append(rid)
            assert time.time() - t0 < 60, f"only {len(seen)} of {len(reqs)} reported"
        assert sorted(seen) == sorted(reqs)
        assert srv.wait(1000) is None                        # each id once
        for k, r in enumerate(reqs):
            done, recs, _ = srv.poll(r)
            assert done and recs.tobytes() == alone(torch_dev, ctx, imgs[k]).tobytes()


def test_server_pinned_submit(torch_dev, ctx):
    """Zero-copy submission from pinned host memory gives the same streams;
    pageable memory is refused."""
    imgs = mixed_images(10, 6, 64, 512)
    pinned = [torch_dev.from_numpy(im).pin_memory() for im in imgs]
    with fb.Server(16, 4, THR, max_slots=8, step_blocks=64) as srv:
        reqs = [srv.submit_pinned(p) for p in pinned]
        res = drain(srv, reqs)
        with pytest.raises(fb.FeError) as ei:
            srv.submit_pinned(torch_dev.from_numpy(imgs[0].copy()))
        assert ei.value.status == fb.FE_ERR_INVALID
    for k, im in enumerate(imgs):
        assert res[k][0].tobytes() == alone(torch_dev, ctx, im).tobytes()


@pytest.mark.parametrize("budget,step_blocks", [(8 << 30, 256), (48 << 20, 8)])
def test_server_2x2_tree(torch_dev, ctx, budget, step_blocks):
    # the paper's 16 -> 2 tree served: each result equals the oracle, in a
    # mix, with small steps that spread an image over several of them
    thr = [300, 200, 100]
    imgs = mixed_images(10, 7, 64, 512)
    log(f"server 16 -> 2, budget {budget >> 20} MiB, {step_blocks}-block steps")
    with fb.Server(16, 2, thr, hbm_budget=budget, host_budget=64 << 20, max_slots=8,
                   step_blocks=step_blocks) as srv:
        reqs = [srv.submit(im) for im in imgs]
        res = drain(srv, reqs)
    for k, im in enumerate(imgs):
        assert res[k][0].tobytes() == np.ascontiguousarray(mns.encode(im, 16, 2, thr)).tobytes(), k


def test_request_stage_times(torch_dev, ctx):
    """The stage times of a finished request are ordered (admitted, first
    step, last step, complete), non-negative and end at its latency; an
    unknown or unfinished id is refused."""
    imgs = mixed_images(6, 31, 128, 768)
    with fb.Server(16, 4, THR, hbm_budget=1 << 30, host_budget=256 << 20, max_slots=8, step_blocks=64) as srv:
        reqs = [srv.submit(im) for im in imgs]
        seen = 0
        t0 = time.time()
        while seen < len(reqs):
            rid = srv.wait(2000)
            assert time.time() - t0 < 60, "server did not finish"
            if rid is None:
                continue
            adm, first, last, done = srv.request_times(rid)
            assert 0.0 <= adm <= first <= last <= done
            ok, recs, lat = srv.poll(rid)
            assert ok and abs(lat - done) < 1e-6
            k = reqs.index(rid)
            assert recs.tobytes() == alone(torch_dev, ctx, imgs[k]).tobytes()
            seen += 1
        with pytest.raises(fb.FeError):
            srv.request_times(reqs[0])          # fetched: unknown now


# parameter sets that share one server: thresholds, Technique 1 on / off,
# identity-only fits
MIXED_SETS = [
    dict(thresholds=[300, 200], phase2=True, identity_only=False),
    dict(thresholds=[40, 900], phase2=True, identity_only=False),
    dict(thresholds=[300, 200], phase2=False, identity_only=False),
    dict(thresholds=[120, 60], phase2=True, identity_only=True),
]


@pytest.mark.parametrize("b_min,extra", [(4, []), (2, [50])])
def test_server_per_request_params(torch_dev, ctx, b_min, extra):
    """Requests with different thresholds and flags share steps; each
    stream equals the image encoded alone with its own parameters (and the
    oracle for the small ones).  Block sizes other than the server's are
    refused."""
    imgs = mixed_images(16, 41, 64, 512)
    sets = [dict(s, thresholds=s["thresholds"] + extra) for s in MIXED_SETS]
    log(f"server 16 -> {b_min}, {len(sets)} parameter sets over {len(imgs)} images")
    with fb.Server(16, b_min, sets[0]["thresholds"], max_slots=16, step_blocks=32) as srv:
        reqs = []
        for k, im in enumerate(imgs):
            s = sets[k % len(sets)]
            reqs.append(srv.submit(im, fb.make_params(16, b_min, s["thresholds"], s["phase2"],
                                                      identity_only=s["identity_only"])))
        res = drain(srv, reqs)
        st = srv.stats()
        with pytest.raises(fb.FeError) as ei:
            srv.submit(imgs[0], fb.make_params(8, b_min, [100] * (len(extra) + 1)))
        assert ei.value.status == fb.FE_ERR_INVALID
        with pytest.raises(fb.FeError) as ei:
            srv.submit(imgs[0], fb.make_params(16, b_min, sets[0]["thresholds"], full_search=True))
        assert ei.value.status == fb.FE_ERR_INVALID
    assert st["steps"] < len(imgs)          # requests shared steps
    for k, im in enumerate(imgs):
        s = sets[k % len(sets)]
        want = fb.to_records(ctx.encode(torch_dev.from_numpy(im).cuda(), 16, b_min, s["thresholds"], s["phase2"],
                                        identity_only=s["identity_only"]))
        assert res[k][0].tobytes() == want.tobytes(), f"image {k} (set {k % len(sets)}) differs in the mix"
        if im.size <= 128 * 128:
            o = mns.encode(im, 16, b_min, s["thresholds"], phase2=s["phase2"], isometries=not s["identity_only"])
            assert res[k][0].tobytes() == np.ascontiguousarray(o).tobytes(), k


def test_server_zero_copy_result(torch_dev, ctx):
    """fe_server_result hands out a finished request's records in the
    server's pinned memory (the same bytes fe_server_poll copies), valid
    until fe_server_release forgets the id; a running request is busy."""
    imgs = mixed_images(8, 51, 64, 512)
    got = {}
    with fb.Server(16, 4, THR, max_slots=8, step_blocks=64) as srv:
        big = srv.submit(synth.noise_1f(1024, 1024, 52))
        try:
            srv.result(big)                      # almost surely still running
        except fb.FeError as e:
            assert e.status == fb.FE_ERR_BUSY
        reqs = [srv.submit(im) for im in imgs]
        t0 = time.time()
        while len(got) < len(reqs) + 1:
            rid = srv.wait(10000)
            assert time.time() - t0 < 60, "server did not finish"
            if rid is None:
                continue
            recs, lat = srv.result(rid)
            assert lat > 0
            got[rid] = recs.copy()
            srv.release(rid)
            with pytest.raises(fb.FeError) as ei:
                srv.result(rid)
            assert ei.value.status == fb.FE_ERR_INVALID
    for k, r in enumerate(reqs):
        assert got[r].tobytes() == alone(torch_dev, ctx, imgs[k]).tobytes(), k
    assert got[big].tobytes() == alone(torch_dev, ctx, synth.noise_1f(1024, 1024, 52)).tobytes()
