"""Benchmark of the MNS encoder on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

A step is one batched MNS encode (fused quadtree kernel + stream ordering)
of the 256-image mixed workload: sides log-uniform in 128..2048 (multiples
of 32), half 1/f noise and half piecewise-smooth, quadtree 16 -> 8 -> 4 with
MSE thresholds (300, 200), inputs resident in HBM.  The value is range
blocks per second: the number of ranges the quadtree evaluates in phase 1
(top tiles + 4 x split ranges), summed over the batch, per second of step
time.  Printed as one JSON line with the roofline of the dominant kernel
(live HIP-event timing on its launch stream) and the CPU oracle timed on a
bounded sample of the same images.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
VALU_DOT4_TMACS = 1024 * 16 * 4 * 2.4e9 / 1e12   # 157.3
B_MAX, B_MIN, THR = 16, 4, (300, 200)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "mns_tiles_c4_traffic.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1501_02894_amd", "csrc", f)
                  for f in ("mns_encode.hip", "fe_device.h", "fe_internal.h")]


def kernel_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def gen_images(n: int):
    from concurrent.futures import ProcessPoolExecutor
    from paper_1501_02894_amd import synth
    entries = synth.c4_sides(n)
    workers = min(8, os.cpu_count() or 1)
    with ProcessPoolExecutor(workers) as ex:
        return list(ex.map(_gen_one, range(n), chunksize=4)), entries


def _gen_one(k):
    from paper_1501_02894_amd import synth
    side, kind, ss = synth.c4_sides()[k]
    return synth._mixed_image(side, kind, ss)


def level_sizes(level, tiles: int, n_levels: int) -> list:
    """|W_l| per level of quadtree streams, from their records' levels: W_1
    holds the top tiles, and the level-l ranges accepted by neither phase
    are split, their four children forming W_l+1 (a phase-2 record stands
    for its level-l range).  The fused kernel also fits the children of
    ranges that phase 2 accepts, which is extra work of this design and not
    counted."""
    p = np.bincount(np.asarray(level).astype(np.int64), minlength=n_levels)   # records per level
    R, sizes = int(tiles), []
    for lv in range(n_levels):
        sizes.append(R)
        split = R - int(p[lv])
        assert split >= 0 and (split == 0 or lv < n_levels - 1)
        R = 4 * split
    return sizes


def range_blocks(level, flags, tiles: int, n_levels: int) -> int:
    """Phase-1 evaluations, Sum_l |W_l| (flags: unused, kept for callers that
    pass whole records)."""
    return sum(level_sizes(level, tiles, n_levels))


def n_levels(b_max: int, b_min: int) -> int:
    return (b_max // b_min).bit_length()


def gpu_level_sizes(out, n: int, tiles: int, b_max: int, b_min: int) -> list:
    """level_sizes of the first n records of a device record array."""
    return level_sizes(out[:n, 8].cpu().numpy(), tiles, n_levels(b_max, b_min))


def gpu_range_blocks(out, n: int, tiles: int, b_max: int, b_min: int) -> int:
    return sum(gpu_level_sizes(out, n, tiles, b_max, b_min))


ORACLE_ENV = {"OMP_NUM_THREADS": "1", "OPENBLAS_NUM_THREADS": "1", "MKL_NUM_THREADS": "1"}


def start_cpu_baseline(images):
    """Start the oracle on every image of the batch in a child process of
    its own, with one BLAS/OpenMP thread set before it imports numpy, so that
    it runs while the GPU legs are measured.  Returns (process, workdir)."""
    import subprocess
    import tempfile
    wd = tempfile.mkdtemp(prefix="fe_oracle_")
    np.save(os.path.join(wd, "shapes.npy"), np.array([im.shape for im in images], np.int64))
    np.save(os.path.join(wd, "pixels.npy"), np.concatenate([im.reshape(-1) for im in images]))
    env = dict(os.environ, **ORACLE_ENV)
    proc = subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-oracle-child", wd], env=env,
                            stdout=subprocess.DEVNULL)
    return proc, wd


def cpu_oracle_child(wd: str):
    """The child's side: the oracle, as it stands, on every image in order,
    single-threaded; writes the streams, per-image offsets and the time."""
    from oracle import mns
    shapes = np.load(os.path.join(wd, "shapes.npy"))
    pix = np.load(os.path.join(wd, "pixels.npy"))
    offs = np.concatenate([[0], np.cumsum(shapes[:, 0] * shapes[:, 1])])
    images = [pix[offs[k]:offs[k + 1]].reshape(shapes[k]) for k in range(len(shapes))]
    t0 = time.perf_counter()
    blocks = 0
    recs = []
    for img in images:
        r = mns.encode(img, B_MAX, B_MIN, list(THR))
        tiles = (img.shape[0] // B_MAX) * (img.shape[1] // B_MAX)
        blocks += range_blocks(r["level"], r["flags"], tiles, n_levels(B_MAX, B_MIN))
        recs.append(r)
    dt = time.perf_counter() - t0
    np.save(os.path.join(wd, "records.npy"), np.ascontiguousarray(np.concatenate(recs)).view(np.uint8))
    np.save(os.path.join(wd, "rec_offsets.npy"), np.concatenate([[0], np.cumsum([r.size for r in recs])]))
    with open(os.path.join(wd, "timing.json"), "w") as f:
        json.dump({"seconds": dt, "range_blocks": blocks, "images": len(images),
                   "pixels": int(offs[-1]), "threads": {k: os.environ.get(k) for k in ORACLE_ENV}}, f)


def finish_cpu_baseline(proc, wd: str):
    """Wait for the child; returns (timing dict, records as uint8 (n, 16),
    per-image record offsets), or raises if the child failed."""
    import shutil
    rc = proc.wait()
    try:
        if rc != 0:
            raise RuntimeError(f"the oracle child process exited with {rc}")
        with open(os.path.join(wd, "timing.json")) as f:
            timing = json.load(f)
        recs = np.load(os.path.join(wd, "records.npy")).reshape(-1, 16)
        roffs = np.load(os.path.join(wd, "rec_offsets.npy"))
        return timing, recs, roffs
    finally:
        shutil.rmtree(wd, ignore_errors=True)


def cpu_fullsearch_sample(img, B=16, n=16, seed=2):
    """The exhaustive-search oracle on a seeded sample of n level-1 ranges
    of one image, its BLAS on the host cores of one GPU's share (at most
    16); ranges/s."""
    from oracle import fullsearch
    from threadpoolctl import threadpool_limits
    H, W = img.shape
    rng = np.random.default_rng(seed)
    pick = rng.choice((H // B) * (W // B), size=n, replace=False)
    xs = (pick % (W // B)) * B
    ys = (pick // (W // B)) * B
    cores = min(16, len(os.sched_getaffinity(0)))
    with threadpool_limits(limits=cores):
        t0 = time.perf_counter()
        fullsearch.best_matches(img, xs, ys, B)
        dt = time.perf_counter() - t0
    ndom = (W - 2 * B + 1) * (H - 2 * B + 1)
    return {"value": n / dt, "unit": "ranges/s", "cores": cores, "kind": "oracle",
            "sample": f"{n} seeded level-1 ranges (B={B}) of C2 against all {ndom} step-1 domains and "
                      f"8 isometries, fp64 BLAS, {dt:.1f} s"}


def pooled(fn, args, workers=8):
    from concurrent.futures import ProcessPoolExecutor
    with ProcessPoolExecutor(min(workers, os.cpu_count() or 1)) as ex:
        return list(ex.map(fn, args))


def _gen_c5(k):
    from paper_1501_02894_amd import synth
    return synth.c5_image(synth.c5_sides()[k])


def _gen_named(name):
    from paper_1501_02894_amd import synth
    return synth.workload(name)


def timed_kernel(fb, ctx, slot, fn, reps):
    """Mean event-timed duration (ms) of kernel `slot` over reps calls of fn."""
    import torch
    fn()
    torch.cuda.synchronize()
    fb.fe_timing_read(ctx.handle)
    fb.fe_timing_enable(ctx.handle, True)
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / reps
    fb.fe_timing_enable(ctx.handle, False)
    ms, cnt = fb.fe_timing_read(ctx.handle)
    return (ms[slot] / cnt[slot] if cnt[slot] else float("nan")), cnt[slot] / reps, wall


def bench_single(fb, ctx, img, b_max, b_min, thr, reps=10, cold_reps=0):
    """One image: encode kernel time (HIP events) and call time; with
    cold_reps, also the kernel time after overwriting 1 GiB of device memory
    before each call (the image and scratch no longer in L2 / Infinity
    Cache)."""
    import torch
    t = torch.from_numpy(img).cuda()
    p = fb.make_params(b_max, b_min, thr)
    out = torch.empty((fb.fe_max_transforms(img.shape[1], img.shape[0], b_min), 16), dtype=torch.uint8,
                      device="cuda")
    n = fb.fe_encode(ctx.handle, t, p, out=out).shape[0]
    kms, _, wall = timed_kernel(fb, ctx, fb.FE_TIMING_ENCODE, lambda: fb.fe_encode(ctx.handle, t, p, out=out), reps)
    tiles = (img.shape[0] // b_max) * (img.shape[1] // b_max)
    blocks = gpu_range_blocks(out, n, tiles, b_max, b_min)
    alg = img.size + 16 * n + 8 * tiles
    res = {"pixels": int(img.size), "records": n, "range_blocks": blocks, "kernel_ms": kms,
           "call_ms": wall, "range_blocks_per_s": blocks / (wall / 1e3),
           "kernel_GBps": alg / (kms / 1e3) / 1e9}
    if cold_reps:
        junk = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        fb.fe_timing_read(ctx.handle)
        fb.fe_timing_enable(ctx.handle, True)
        for _ in range(cold_reps):
            junk.fill_(1)
            fb.fe_encode(ctx.handle, t, p, out=out)
        torch.cuda.synchronize()
        fb.fe_timing_enable(ctx.handle, False)
        ms, cnt = fb.fe_timing_read(ctx.handle)
        cms = ms[fb.FE_TIMING_ENCODE] / max(1, cnt[fb.FE_TIMING_ENCODE])
        res["cold"] = {"kernel_ms": cms, "kernel_GBps": alg / (cms / 1e3) / 1e9}
        del junk
    return res, out[:n]


def bench_decode(fb, ctx, recs, w, h, b_max, iters=12, reps=3):
    """Both decoders on one stream: the tile decoder (the default for
    encoder-order streams) and the per-record decoder, per iteration."""
    import torch
    out = torch.empty((h, w), dtype=torch.uint8, device="cuda")
    fn = lambda: fb.fe_decode(ctx.handle, recs, w, h, b_max, iters, out=out)
    # per iteration: the iterate read once (its 2 x 2 means come from LDS or
    # cache), one byte written per pixel, 16 bytes per transform
    alg = 2 * w * h + 16 * int(recs.shape[0])
    res = {"iterations": iters}
    try:
        for mode, key in ((fb.FE_DECODE_AUTO, "tiles"), (fb.FE_DECODE_RECORDS, "records")):
            fb.fe_decode_set_mode(ctx.handle, mode)
            kms, per_call, wall = timed_kernel(fb, ctx, fb.FE_TIMING_DECODE, fn, reps)
            used = "tiles" if fb.fe_decode_last(ctx.handle) == fb.FE_DECODE_TILES else "records"
            res[key] = {"decoder": used, "iter_ms": kms, "call_ms": wall, "iter_GBps": alg / (kms / 1e3) / 1e9}
    finally:
        fb.fe_decode_set_mode(ctx.handle, fb.FE_DECODE_AUTO)
    res.update(iter_ms=res["tiles"]["iter_ms"], iter_GBps=res["tiles"]["iter_GBps"])
    return res, out


def bench_fullsearch(fb, ctx, img, b_max, b_min, thr, reps=2):
    import torch
    t = torch.from_numpy(img).cuda()
    p = fb.make_params(b_max, b_min, thr, full_search=True)
    out = torch.empty((fb.fe_max_transforms(img.shape[1], img.shape[0], b_min), 16), dtype=torch.uint8,
                      device="cuda")
    recs = fb.to_records(fb.fe_encode(ctx.handle, t, p, out=out))
    kms, launches, wall = timed_kernel(fb, ctx, fb.FE_TIMING_FULLSEARCH,
                                       lambda: fb.fe_encode(ctx.handle, t, p, out=out), reps)
    H, W = img.shape
    R = (H // b_max) * (W // b_max)
    macs = 0
    for level in range(len(thr) + 1):
        B = b_max >> level
        macs += R * 8 * (W - 2 * B + 1) * (H - 2 * B + 1) * B * B
        R = 4 * (R - int(np.sum(recs["level"] == level)))
    search_ms = kms * launches
    return {"records": int(recs.size), "search_ms": search_ms, "call_ms": wall, "int8_macs": macs,
            "int8_TOPS": 2 * macs / (search_ms / 1e3) / 1e12,
            "mfma_frac": 2 * macs / (search_ms / 1e3) / 5.0e15}


def bench_localsearch(fb, ctx, img, b_max, b_min, thr, reps=3):
    """Local search (Sec. 2) against MNS with the identity only, same image
    and thresholds: search-kernel time, call time, transforms and the PSNR
    after 12 decoder iterations from grey."""
    import torch
    H, W = img.shape
    t = torch.from_numpy(img).cuda()
    res = {}
    for name, p, slot in (("local_search", fb.make_params(b_max, b_min, thr, local_search=True),
                           fb.FE_TIMING_FULLSEARCH),
                          ("mns_identity", fb.make_params(b_max, b_min, thr, identity_only=True),
                           fb.FE_TIMING_ENCODE)):
        recs = fb.fe_encode(ctx.handle, t, p)
        kms, launches, wall = timed_kernel(fb, ctx, slot, lambda: fb.fe_encode(ctx.handle, t, p), reps)
        dec = fb.fe_decode(ctx.handle, recs, W, H, b_max, 12).cpu().numpy().astype(np.float64)
        mse = float(np.mean((dec - img.astype(np.float64)) ** 2))
        res[name] = {"transforms": int(recs.shape[0]), "kernel_ms_per_call": kms * launches, "call_ms": wall,
                     "psnr_db_12_iters": 10.0 * np.log10(255.0 ** 2 / mse)}
    return res


def bench_bitstream(fb, ctx, img, b_max, b_min, thr, reps=5):
    """The compressed file of Sec. 3.3 (Technique 2 of Sec. 3.4) for one
    image, with the 8-isometry codes and with the paper's identity-only
    14-bit codes: size (bits per pixel, compression ratio), the PSNR of 12
    decoder iterations from grey, and the time to pack (GPU, call wall
    time) and to parse (native, host)."""
    import torch
    H, W = img.shape
    t = torch.from_numpy(img).cuda()
    res = {}
    for iso in (True, False):
        recs = fb.fe_encode(ctx.handle, t, fb.make_params(b_max, b_min, thr, identity_only=not iso))
        out = torch.empty(fb.fe_pack_bound(int(recs.shape[0])), dtype=torch.uint8, device="cuda")
        fb.fe_pack(ctx.handle, recs, W, H, b_max, b_min, isometry=iso, out=out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            _, nbits = fb.fe_pack(ctx.handle, recs, W, H, b_max, b_min, isometry=iso, out=out)
        pack_ms = (time.perf_counter() - t0) * 1e3 / reps
        data = out[: (nbits + 7) // 8].cpu().numpy().tobytes()
        t0 = time.perf_counter()
        back, _ = fb.fe_unpack(data, nbits)
        unpack_ms = (time.perf_counter() - t0) * 1e3
        same = back.tobytes() == fb.to_records(recs).tobytes()
        dec = fb.fe_decode(ctx.handle, recs, W, H, b_max, 12).cpu().numpy().astype(np.float64)
        mse = float(np.mean((dec - img.astype(np.float64)) ** 2))
        psnr = 10.0 * np.log10(255.0 ** 2 / mse) if mse > 0 else float("inf")
        res["isometries" if iso else "identity_only"] = {
            "transforms": int(recs.shape[0]), "bits": nbits, "bpp": nbits / (W * H),
            "compression_ratio": 8.0 * W * H / (8 * ((nbits + 7) // 8)), "psnr_db_12_iters": psnr,
            "pack_call_ms": pack_ms, "unpack_ms": unpack_ms, "parsed_equal": same}
    return res


def bench_paper_tree(fb, ctx, img, thr4, thr2, reps=5):
    """The paper's quadtree, 16 x 16 down to 2 x 2 (Sec. 3.3), against the
    16 -> 4 tree, both with the paper's identity-only codes: encode kernel
    time (HIP events), call wall time, transforms, file size and the PSNR of
    12 decoder iterations from grey; then zoom decoding (Sec. 1) of the
    16 -> 4 stream at 1x and 2x (decode kernel time per iteration)."""
    import torch
    H, W = img.shape
    t = torch.from_numpy(img).cuda()
    res = {}
    for name, b_min, thr in (("16to4", 4, thr4), ("16to2", 2, thr2)):
        p = fb.make_params(16, b_min, thr, identity_only=True)
        out = torch.empty((fb.fe_max_transforms(W, H, b_min), 16), dtype=torch.uint8, device="cuda")
        recs = fb.fe_encode(ctx.handle, t, p, out=out)
        kms, launches, wall = timed_kernel(fb, ctx, fb.FE_TIMING_ENCODE,
                                           lambda: fb.fe_encode(ctx.handle, t, p, out=out), reps)
        _, nbits = fb.fe_pack(ctx.handle, recs, W, H, 16, b_min, isometry=False)
        dec = fb.fe_decode(ctx.handle, recs, W, H, 16, 12).cpu().numpy().astype(np.float64)
        mse = float(np.mean((dec - img.astype(np.float64)) ** 2))
        res[name] = {"transforms": int(recs.shape[0]), "encode_kernel_ms": kms, "call_ms": wall,
                     "bpp": nbits / (W * H), "psnr_db_12_iters": 10.0 * np.log10(255.0 ** 2 / mse),
                     "decoder": "tiles" if ctx.decode_last() == fb.FE_DECODE_TILES else "records",
                     "pixels_per_s": W * H / (kms / 1e3)}
        # decode iteration time with either decoder
        for mode, key in ((fb.FE_DECODE_AUTO, "decode_iter_ms"), (fb.FE_DECODE_RECORDS, "decode_iter_ms_records")):
            fb.fe_decode_set_mode(ctx.handle, mode)
            dms, _, _ = timed_kernel(fb, ctx, fb.FE_TIMING_DECODE, lambda: fb.fe_decode(ctx.handle, recs, W, H, 16, 12), 3)
            res[name][key] = dms
        fb.fe_decode_set_mode(ctx.handle, fb.FE_DECODE_AUTO)
        if b_min == 4:
            zoom = {}
            for z in (1, 2):
                fn = lambda: fb.fe_decode_zoom(ctx.handle, recs, W, H, 16, z, 12)
                dms, dl, dwall = timed_kernel(fb, ctx, fb.FE_TIMING_DECODE, fn, 3)
                zoom[f"x{z}"] = {"side": W * z, "iter_kernel_ms": dms, "call_ms": dwall,
                                 "decoder": "tiles" if ctx.decode_last() == fb.FE_DECODE_TILES else "records"}
            res["zoom_16to4"] = zoom
    return res


def bench_tradeoff(fb, ctx, images, b_max=16, reps=5):
    """No-search (phase 1 only) against MNS (Technique 1 on) over a sweep of
    thresholds, with the paper's codes (identity only, 14-bit phase 1), for
    the 16 -> 4 tree and the paper's 16 -> 2 tree: per point the file size
    (bpp), the PSNR after 12 decoder iterations from grey, and the encode
    time (encode kernels, HIP events; call wall time)."""
    import torch
    pts = []
    # t2 from 100 to about 900 in steps of 1.15, t1 = 1.5 t2 (the transition
    # from 4 x 4 blocks to whole tiles lies in this range on these images);
    # the 2 x 2 level's threshold t3 = t2 / 1.5
    base = [100 * 1.15 ** k for k in range(16)]
    sweeps = {4: [(int(round(1.5 * v)), int(round(v))) for v in base],
              2: [(int(round(1.5 * v)), int(round(v)), int(round(v / 1.5))) for v in base]}
    for name, img in images.items():
        H, W = img.shape
        t = torch.from_numpy(img).cuda()
        for b_min in (4, 2):
            for phase2 in (False, True):
                for thr in sweeps[b_min]:
                    p = fb.make_params(b_max, b_min, thr, phase2=phase2, identity_only=True)
                    recs = fb.fe_encode(ctx.handle, t, p)
                    kms, _, wall = timed_kernel(fb, ctx, fb.FE_TIMING_ENCODE, lambda: fb.fe_encode(ctx.handle, t, p), reps)
                    _, nbits = fb.fe_pack(ctx.handle, recs, W, H, b_max, b_min, isometry=False)
                    dec = fb.fe_decode(ctx.handle, recs, W, H, b_max, 12).cpu().numpy().astype(np.float64)
                    mse = float(np.mean((dec - img.astype(np.float64)) ** 2))
                    pts.append({"image": name, "tree": f"{b_max}->{b_min}", "method": "mns" if phase2 else "no-search",
                                "thresholds": list(thr),
                                "transforms": int(recs.shape[0]),
                                "phase2_transforms": int((recs[:, 9] != 0).sum().item()), "bits": nbits,
                                "bpp": nbits / (W * H), "psnr_db": 10.0 * np.log10(255.0 ** 2 / mse),
                                "kernel_ms": kms, "call_ms": wall})
    return pts


def serve_run(fb, mode, pool, rate, n_req, warmup, seed, ctx=None):
    """Poisson arrivals at `rate`; returns served images/s and latency
    percentiles (scheduled arrival -> records in host memory).  `pool` holds
    the request images as pinned host tensors; the server takes them without
    a host copy, the plain path copies each to the device itself."""
    import gc
    import threading
    import torch
    # a full collection over the bench's many live objects can stall the
    # submitting thread for tens of milliseconds: move them out of the
    # collector's reach for the run (both modes)
    gc.collect()
    gc.freeze()
    total = n_req + warmup
    rng = np.random.default_rng(seed)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, total))
    which = rng.integers(0, len(pool), total)
    done_at = np.zeros(total)
    if mode == "server":
        # the server is long-lived: created (arenas allocated) before the
        # arrival clock starts
        srv = fb.Server(B_MAX, B_MIN, THR, hbm_budget=16 << 30, host_budget=4 << 30, max_slots=512,
                        step_blocks=2048)
    t0 = time.perf_counter() + 0.05
    if mode == "server":
        lat = np.zeros(total)
        stages = np.zeros((total, 4))
        index = {}
        # the submitting thread and this one share the interpreter lock: hand
        # it over every 0.2 ms rather than every 5 ms, so that arrivals keep
        # their schedule
        switch = sys.getswitchinterval()
        sys.setswitchinterval(2e-4)

        def submitter():
            for i in range(total):
                d = t0 + arrivals[i] - time.perf_counter()
                if d > 0:
                    time.sleep(d)
                while True:
                    try:
                        rid = srv.submit_pinned(pool[which[i]])
                        break
                    except fb.FeError as e:
                        if e.status != fb.FE_ERR_BUSY:
                            raise
                        time.sleep(0.0002)
                lat[i] = time.perf_counter() - (t0 + arrivals[i])   # submit delay
                index[rid] = i

        th = threading.Thread(target=submitter)
        th.start()
        finished = 0
        while finished < total:
            rid = srv.wait(2000)          # blocks in the library, GIL released
            if rid is None:
                continue
            st = srv.request_times(rid)
            recs, l = srv.result(rid)     # the records in the server's pinned memory, no copy
            srv.release(rid)
            while rid not in index:      # the submitter has not recorded it yet
                time.sleep(0)
            i = index[rid]
            finished += 1
            done_at[i] = time.perf_counter() - t0
            stages[i] = st
            lat[i] += l / 1e3
        th.join()
        sys.setswitchinterval(switch)
        stats = srv.stats()
        srv.close()
    else:
        p = fb.make_params(B_MAX, B_MIN, THR)
        lat = np.zeros(total)
        for i in range(total):
            d = t0 + arrivals[i] - time.perf_counter()
            if d > 0:
                time.sleep(d)
            t = pool[which[i]].cuda()
            out = fb.fe_encode(ctx.handle, t, p)
            recs = out.cpu()
            now = time.perf_counter() - t0
            done_at[i] = now
            lat[i] = now - arrivals[i]
        stats = None
    gc.unfreeze()
    m = slice(warmup, total)
    span = done_at[m].max() - arrivals[m].min()
    res = {"mode": mode, "rate": rate, "requests": n_req, "images_per_s": n_req / span,
           "p50_ms": float(np.percentile(lat[m], 50) * 1e3), "p99_ms": float(np.percentile(lat[m], 99) * 1e3),
           "mean_px": float(np.mean([pool[k].numel() for k in which[m]]))}
    if stats:
        res["steps"] = stats["steps"]
        # where the server's latency goes: submit delay (arrival to submit
        # returning), then admitted, first step, last step and complete,
        # each in ms after submission (p50 / p99 over the measured requests)
        sd = lat[m] * 1e3 - stages[m, 3]
        res["stages_ms"] = {name: [float(np.percentile(v, 50)), float(np.percentile(v, 99))]
                            for name, v in (("submit_delay", sd), ("admitted", stages[m, 0]),
                                            ("first_step", stages[m, 1]), ("last_step", stages[m, 2]),
                                            ("complete", stages[m, 3]))}
    return res


def copy_calibration(torch, dev):
    """Three device copies of 256 MiB: the counter readings of a kernel
    whose traffic is known (scales FETCH_SIZE / WRITE_SIZE)."""
    src = torch.empty(256 << 20, dtype=torch.uint8, device=dev).fill_(3)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    return 256 << 20


def decode_only(fb, args):
    import torch
    from paper_1501_02894_amd import synth
    img = synth.workload("c3")
    ctx = fb.Context(0)
    recs = fb.to_records(ctx.encode(torch.from_numpy(img).cuda(), 32, 4, [150, 100, 64]))
    t = torch.from_numpy(np.ascontiguousarray(recs).view(np.uint8).reshape(-1, 16).copy()).cuda()
    res, _ = bench_decode(fb, ctx, t, 4096, 4096, 32, iters=12, reps=args.steps)
    out = {"workload": "c3 decode (4096^2, 32 -> 4, 12 iterations)", "records": int(recs.size), "c3_decode": res}
    if args.copy_calibration:
        out["copy_calibration_bytes"] = copy_calibration(torch, torch.device("cuda:0"))
    ctx.close()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--images", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the comparisons (plain, cold, two batches in flight) and the "
                                                             "single-image, decode and full-search runs")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a device copy of known size (for counter scaling)")
    ap.add_argument("--serve-rates", default="50,100,200,500,1000,2000",
                    help="Poisson arrival rates (requests/s) of the served-encoding sweep")
    ap.add_argument("--serve-extra-rates", default="8000,20000",
                    help="rates beyond the sweep, toward saturation")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-warmup", type=int, default=200)
    ap.add_argument("--serve-pool", type=int, default=512)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--decode-only", action="store_true",
                    help="only decode C3 (4096^2, 32 -> 4) with both decoders (a profiling workload)")
    ap.add_argument("--tradeoff", action="store_true",
                    help="only the no-search vs MNS sweep (bpp, PSNR, time) on two 512^2 images")
    ap.add_argument("--paper-tree", action="store_true",
                    help="only the 16 -> 2 tree against 16 -> 4 on C2 and C3, and zoom decoding")
    ap.add_argument("--fullsearch-only", action="store_true",
                    help="only the exhaustive-search encode of C2 (512^2, 16 -> 4) (a profiling workload)")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default tile shape (no autotuning)")
    ap.add_argument("--cpu-oracle-child", metavar="DIR", help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_oracle_child:
        cpu_oracle_child(args.cpu_oracle_child)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    special = args.decode_only or args.tradeoff or args.paper_tree or args.fullsearch_only
    if not special:
        # the batch, and the oracle's child process (a new program), before
        # anything touches the GPU
        t_gen = time.perf_counter()
        images, _ = gen_images(args.images)
        t_gen = time.perf_counter() - t_gen
        print(f"[bench] generated {len(images)} images in {t_gen:.1f}s", file=sys.stderr, flush=True)
        oracle_child = None if args.no_cpu_baseline else start_cpu_baseline(images)
        serve_pool = None
        if not args.no_serving:
            t_gen = time.perf_counter()
            serve_pool = pooled(_gen_c5, list(range(args.serve_pool)), 16)
            print(f"[bench] generated the {len(serve_pool)}-image request pool in {time.perf_counter() - t_gen:.1f}s",
                  file=sys.stderr, flush=True)

    import torch
    from paper_1501_02894_amd import binding as fb

    assert torch.cuda.is_available(), "needs a GPU"
    dev = torch.device("cuda:0")
    if args.decode_only:
        decode_only(fb, args)
        return
    if args.tradeoff:
        from paper_1501_02894_amd import synth
        ctx = fb.Context(0)
        imgs = {"c2 (1/f noise + polygons)": synth.workload("c2"),
                "rough 1/f noise (beta 1.5)": synth.noise_1f(512, 512, 22, beta=1.5)}
        pts = bench_tradeoff(fb, ctx, imgs)
        ctx.close()
        print(json.dumps({"workload": "no-search vs MNS, 512^2, 16 -> 4 and 16 -> 2, identity-only codes",
                          "points": pts}),
              flush=True)
        return
    if args.paper_tree:
        c2, c3 = pooled(_gen_named, ["c2", "c3"], 2)
        ctx = fb.Context(0)
        res = {"c2": bench_paper_tree(fb, ctx, c2, [300, 200], [300, 200, 100]),
               "c3": bench_paper_tree(fb, ctx, c3, [150, 100], [150, 100, 64])}
        ctx.close()
        print(json.dumps({"workload": "16 -> 2 vs 16 -> 4 trees on C2 (512^2) and C3 (4096^2), zoom decoding",
                          "paper_tree": res}), flush=True)
        return
    if args.fullsearch_only:
        from paper_1501_02894_amd import synth
        ctx = fb.Context(0)
        res = bench_fullsearch(fb, ctx, synth.workload("c2"), 16, 4, [300, 200], reps=args.steps)
        ctx.close()
        print(json.dumps({"workload": "c2 exhaustive search (512^2, 16 -> 4, thresholds 300,200)",
                          "c2_fullsearch": res}), flush=True)
        return

    # one device buffer holding every image back to back (inputs resident in HBM)
    sizes = [im.size for im in images]
    offs = np.concatenate([[0], np.cumsum(sizes)])
    flat = torch.empty(int(offs[-1]), dtype=torch.uint8, device=dev)
    for k, im in enumerate(images):
        flat[int(offs[k]):int(offs[k + 1])].copy_(torch.from_numpy(im.reshape(-1)))
    views = [flat[int(offs[k]):int(offs[k + 1])].view(images[k].shape) for k in range(len(images))]
    total_px = int(offs[-1])
    tiles = [(im.shape[0] // B_MAX) * (im.shape[1] // B_MAX) for im in images]

    ctx = fb.Context(0)
    params = fb.make_params(B_MAX, B_MIN, THR)
    cap = sum(fb.fe_max_transforms(im.shape[1], im.shape[0], B_MIN) for im in images)
    out = torch.empty((cap, 16), dtype=torch.uint8, device=dev)
    offsets = torch.zeros(len(images) + 1, dtype=torch.int64, device=dev)

    # One step: a batch encode call over the resident images, reusing the
    # descriptor array.  HIP events on the launch stream time the fused
    # kernel in the timed steps (only that kernel: each timed launch adds two
    # event records to the step); the ordering is timed in separate steps.
    descs = fb.image_descs(views)

    # tile shape: the autotuner times every built shape on this batch (HIP
    # events around the fused kernel) and selects the fastest for the
    # context; the timed steps and the recorded plan use it
    default_shape = fb.fe_get_tile_shape(ctx.handle, B_MAX, B_MIN)
    if args.no_autotune:
        tuned_shape, tuned_ms = default_shape, None
    else:
        tuned_shape, tuned_ms = fb.fe_autotune(ctx.handle, views, params, out, offsets, reps=5)
    torch.cuda.synchronize()
    print(f"[bench] tile shape {tuned_shape} (autotune {tuned_ms}; default {default_shape})",
          file=sys.stderr, flush=True)

    def step():
        fb.fe_encode_batch(ctx.handle, views, params, out=out, offsets=offsets, wait=False, descs=descs)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    fb.fe_timing_read(ctx.handle)
    fb.fe_timing_select(ctx.handle, 1 << fb.FE_TIMING_ENCODE)
    fb.fe_timing_enable(ctx.handle, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    fb.fe_timing_enable(ctx.handle, False)
    kms, kcnt = fb.fe_timing_read(ctx.handle)
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    # the ordering kernels' time, in steps of their own
    fb.fe_timing_select(ctx.handle, 1 << fb.FE_TIMING_SCATTER)
    fb.fe_timing_enable(ctx.handle, True)
    for _ in range(min(args.steps, 10)):
        step()
    torch.cuda.synchronize()
    fb.fe_timing_enable(ctx.handle, False)
    fb.fe_timing_select(ctx.handle, 0xffffffff)
    sms, scnt = fb.fe_timing_read(ctx.handle)
    # the distribution of single steps: 20 more, each between two events on
    # the stream the library launches on (torch's current stream)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(20)]
    for e0, e1 in evs:
        e0.record()
        step()
        e1.record()
    torch.cuda.synchronize()
    st = np.array([e0.elapsed_time(e1) for e0, e1 in evs])
    step_dist = {"reps": int(st.size), "median_ms": float(np.median(st)), "p99_ms": float(np.percentile(st, 99)),
                 "min_ms": float(st.min()), "max_ms": float(st.max())}

    off_h = offsets.cpu().numpy()
    n_rec = int(off_h[-1])
    per_img = np.diff(off_h)
    sizes = gpu_level_sizes(out, n_rec, sum(tiles), B_MAX, B_MIN)
    blocks = sum(sizes)
    # algorithmic int8 multiply-adds of the moments: per B x B range, Sum r,
    # Sum r^2, Sum d, Sum d^2 and the 8 isometric Sum r T_e(d), B^2 each
    macs = sum(12 * (B_MAX >> lv) ** 2 * r for lv, r in enumerate(sizes))
    value = blocks / (ms_per_step / 1e3)

    # the same step recorded once as a HIP graph and replayed (untimed)
    plan = fb.Plan(ctx, views, B_MAX, B_MIN, THR, out, offsets)
    for _ in range(args.warmup):
        plan.launch()
    torch.cuda.synchronize()
    g0 = time.perf_counter()
    for _ in range(args.steps):
        plan.launch()
    torch.cuda.synchronize()
    graph_ms = (time.perf_counter() - g0) * 1e3 / args.steps
    graph_same = bool(np.array_equal(offsets.cpu().numpy(), off_h))
    plan.close()

    # a new batch every step: two copies of the batch at different device
    # addresses, taken in turn, so that every step uploads its image table
    # and rebuilds the workgroup block descriptors (the step above reuses
    # them while the batch's addresses stay the same)
    flat2 = flat.clone()
    views2 = [flat2[int(offs[k]):int(offs[k + 1])].view(images[k].shape) for k in range(len(images))]
    descs2 = fb.image_descs(views2)
    tables = ((views, descs), (views2, descs2))

    def nstep(i):
        v, d = tables[i & 1]
        fb.fe_encode_batch(ctx.handle, v, params, out=out, offsets=offsets, wait=False, descs=d)

    for i in range(max(2, args.warmup)):
        nstep(i)
    torch.cuda.synchronize()
    n0 = time.perf_counter()
    for i in range(args.steps):
        nstep(i)
    torch.cuda.synchronize()
    new_ms = (time.perf_counter() - n0) * 1e3 / args.steps
    new_table = {"ms_per_step": new_ms, "range_blocks_per_s": blocks / (new_ms / 1e3),
                 "same_offsets": bool(np.array_equal(offsets.cpu().numpy(), off_h))}
    del views2, flat2, tables

    pipelined = None
    if not args.no_extras:
        # two batches in flight: consecutive steps alternate between two
        # contexts on two streams, so one batch's ordering overlaps the next
        # batch's encode (untimed kernels; whole-job throughput)
        ctx2 = fb.Context(0)
        out2 = torch.empty_like(out)
        offsets2 = torch.zeros_like(offsets)
        streams = (torch.cuda.Stream(), torch.cuda.Stream())
        lanes = ((ctx, out, offsets), (ctx2, out2, offsets2))

        def pstep(i):
            c, o, f = lanes[i & 1]
            fb.fe_encode_batch(c.handle, views, params, out=o, offsets=f, wait=False, descs=descs, stream=streams[i & 1])

        for i in range(max(2, args.warmup)):
            pstep(i)
        torch.cuda.synchronize()
        p0 = time.perf_counter()
        for i in range(args.steps):
            pstep(i)
        torch.cuda.synchronize()
        pipe_ms = (time.perf_counter() - p0) * 1e3 / args.steps
        pipe_same = bool(np.array_equal(offsets2.cpu().numpy(), off_h)) and bool(torch.equal(out2[:n_rec], out[:n_rec]))
        ctx2.close()
        pipelined = {"ms_per_step": pipe_ms, "range_blocks_per_s": blocks / (pipe_ms / 1e3),
                     "batches_in_flight": 2, "same_stream": pipe_same}

    enc_ms = kms[fb.FE_TIMING_ENCODE] / max(1, kcnt[fb.FE_TIMING_ENCODE])
    sc_ms = sms[fb.FE_TIMING_SCATTER] / max(1, scnt[fb.FE_TIMING_SCATTER])
    # algorithmic bytes of one launch of the fused kernel: every pixel read
    # once, one 16-byte record written per leaf, one 8-byte occupancy word
    # per top tile
    alg_bytes = total_px + 16 * n_rec + 8 * sum(tiles)
    achieved = alg_bytes / (enc_ms / 1e3) / 1e9
    traffic = None
    try:
        with open(TRAFFIC_FILE) as f:
            tr = json.load(f)
        if tr.get("kernel_hash") == kernel_hash():
            traffic = tr.get("bytes_per_launch")
    except (OSError, ValueError):
        pass

    result = {
        "metric": "MNS range blocks/s + served images/s vs plain, p50/p99 latency, bit-exact",
        "value": value,
        "unit": "range blocks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": "c4: 256 images, sides 128..2048 (x32), 1/f noise + piecewise-smooth, "
                               "MNS 16->8->4, MSE thresholds (300, 200), batched",
                   "images": len(images), "pixels": total_px, "records": n_rec,
                   "range_blocks": blocks},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": f"mns_tiles_kernel<16,3,{tuned_shape[0]},{tuned_shape[1]}>", "kernel_ms": enc_ms,
                     "algorithmic_bytes": alg_bytes,
                     # the same launch against the vector ALU: packed-u8 dot
                     # products, 1024 SIMDs x 16 lanes x 4 MACs x 2.4 GHz
                     "alu": {"int8_macs": macs, "achieved": macs / (enc_ms / 1e3) / 1e12,
                             "peak": VALU_DOT4_TMACS, "unit": "TMAC/s",
                             "frac": macs / (enc_ms / 1e3) / 1e12 / VALU_DOT4_TMACS}},
        "images_per_s": len(images) / (ms_per_step / 1e3),
        "pipelined": pipelined,
        "graph": {"ms_per_step": graph_ms, "range_blocks_per_s": blocks / (graph_ms / 1e3),
                  "same_offsets": graph_same},
        "new_table": new_table,
        "scatter_ms": sc_ms,
        "step_events": step_dist,
        "tile_shape": {"autotuned": list(tuned_shape), "autotune_kernel_ms": tuned_ms,
                       "default": list(default_shape), "eager_ms_per_step": ms_per_step,
                       "graph_ms_per_step": graph_ms},
    }

    if not args.no_extras:
        # plain: the same images encoded one call at a time (each call waits)
        torch.cuda.synchronize()
        outs = [torch.empty((fb.fe_max_transforms(im.shape[1], im.shape[0], B_MIN), 16), dtype=torch.uint8,
                            device=dev) for im in images]
        for k in range(len(images)):
            fb.fe_encode(ctx.handle, views[k], params, out=outs[k])
        torch.cuda.synchronize()
        tp0 = time.perf_counter()
        reps = max(1, min(3, args.steps))
        for _ in range(reps):
            for k in range(len(images)):
                fb.fe_encode(ctx.handle, views[k], params, out=outs[k])
        torch.cuda.synchronize()
        plain_ms = (time.perf_counter() - tp0) * 1e3 / reps
        result["plain"] = {"ms_per_batch": plain_ms, "images_per_s": len(images) / (plain_ms / 1e3),
                           "range_blocks_per_s": blocks / (plain_ms / 1e3)}
        # end to end: the batch from pinned host memory (one copy), the
        # encode, the stream back to pinned host memory
        host_in = torch.empty(int(offs[-1]), dtype=torch.uint8).pin_memory()
        host_in.copy_(torch.from_numpy(np.concatenate([im.reshape(-1) for im in images])))
        host_out = torch.empty((n_rec, 16), dtype=torch.uint8).pin_memory()

        def e2e():
            flat.copy_(host_in, non_blocking=True)
            step()
            host_out.copy_(out[:n_rec], non_blocking=True)

        e2e()
        torch.cuda.synchronize()
        te0 = time.perf_counter()
        reps = 5
        for _ in range(reps):
            e2e()
        torch.cuda.synchronize()
        e2e_ms = (time.perf_counter() - te0) * 1e3 / reps
        result["end_to_end"] = {"ms_per_batch": e2e_ms, "images_per_s": len(images) / (e2e_ms / 1e3),
                                "range_blocks_per_s": blocks / (e2e_ms / 1e3),
                                "bytes_h2d": int(offs[-1]), "bytes_d2h": 16 * n_rec,
                                "same_stream": bool(torch.equal(host_out, out[:n_rec].cpu()))}
        del host_in, host_out
        # cold Infinity Cache: overwrite 1 GiB before each timed launch
        junk = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        fb.fe_timing_enable(ctx.handle, True)
        fb.fe_timing_read(ctx.handle)
        for _ in range(5):
            junk.fill_(1)
            step()
        torch.cuda.synchronize()
        cms, ccnt = fb.fe_timing_read(ctx.handle)
        fb.fe_timing_enable(ctx.handle, False)
        cold_ms = cms[fb.FE_TIMING_ENCODE] / max(1, ccnt[fb.FE_TIMING_ENCODE])
        result["cold"] = {"kernel_ms": cold_ms, "achieved_GBps": alg_bytes / (cold_ms / 1e3) / 1e9}
        del junk

    if not args.no_extras:
        from paper_1501_02894_amd import synth
        c2, c3 = pooled(_gen_named, ["c2", "c3"], 2)
        res_c2, _ = bench_single(fb, ctx, c2, 16, 4, [300, 200])
        res_c3, recs_c3 = bench_single(fb, ctx, c3, 32, 4, [150, 100, 64], reps=5, cold_reps=5)
        res_dec, _ = bench_decode(fb, ctx, recs_c3, 4096, 4096, 32)
        res_fs = bench_fullsearch(fb, ctx, c2, 16, 4, [300, 200])
        result["c2_single"] = res_c2
        result["c3_single"] = res_c3
        result["c3_decode"] = res_dec
        result["c2_fullsearch"] = res_fs
        result["c2_localsearch"] = bench_localsearch(fb, ctx, c2, 16, 4, [300, 200])
        result["bitstream"] = {"c2": bench_bitstream(fb, ctx, c2, 16, 4, [300, 200]),
                               "c3": bench_bitstream(fb, ctx, c3, 32, 4, [150, 100, 64])}
        result["paper_tree"] = {"c2": bench_paper_tree(fb, ctx, c2, [300, 200], [300, 200, 100]),
                                "c3": bench_paper_tree(fb, ctx, c3, [150, 100], [150, 100, 64])}
        print(f"[bench] single/decode/full-search done", file=sys.stderr, flush=True)

    if oracle_child is not None:
        # the oracle child has finished before the serving legs, which are
        # sensitive to host load
        timing, orecs, roffs = finish_cpu_baseline(*oracle_child)
        got = out[:n_rec].cpu().numpy()
        same = [np.array_equal(orecs[roffs[k]:roffs[k + 1]], got[off_h[k]:off_h[k + 1]])
                for k in range(len(images))]
        result["cpu_baseline"] = {"value": timing["range_blocks"] / timing["seconds"], "unit": "range blocks/s",
                                  "cores": 1, "host_cpus": os.cpu_count(), "kind": "oracle",
                                  "sample": f"all {timing['images']} images of the batch ({timing['pixels']} px), "
                                            f"{timing['seconds']:.1f} s, numpy int64, one thread "
                                            f"(OMP/OPENBLAS/MKL threads 1), in a child process"}
        result["bit_exact"] = {"checked_images": int(len(same)), "equal": bool(all(same)),
                               "differing": [k for k, v in enumerate(same) if not v][:16]}
        if not args.no_extras:
            from paper_1501_02894_amd import synth
            result["cpu_baseline"]["fullsearch"] = cpu_fullsearch_sample(synth.workload("c2"))

    if not args.no_serving:
        pool = [torch.from_numpy(im).pin_memory() for im in serve_pool]
        del serve_pool
        def sweep(rates):
            rows = []
            for rate in [float(r) for r in rates.split(",") if r]:
                for mode in ("server", "plain"):
                    rows.append(serve_run(fb, mode, pool, rate, args.serve_requests, args.serve_warmup, 5, ctx=ctx))
                    print(f"[bench] serving {mode} @ {rate}/s: {rows[-1]}", file=sys.stderr, flush=True)
            return rows

        serving = sweep(args.serve_rates)
        extra = sweep(args.serve_extra_rates)
        by = {(r["mode"], r["rate"]): r for r in serving + extra}
        rates = sorted({r["rate"] for r in serving})
        result["serving"] = serving
        result["serving_saturation"] = extra
        result["serving_summary"] = {
            "workload": f"c5: {len(pool)}-image pool, sides 64..4096 (x16), Poisson arrivals, "
                        f"{args.serve_requests} requests after {args.serve_warmup} warm-up per rate",
            "server_p99_le_plain_at_every_swept_rate": all(
                by[("server", r)]["p99_ms"] <= by[("plain", r)]["p99_ms"] for r in rates),
            "max_images_per_s": {m: max(v["images_per_s"] for k, v in by.items() if k[0] == m)
                                 for m in ("server", "plain")},
        }

    if args.copy_calibration:
        result["copy_calibration_bytes"] = copy_calibration(torch, dev)

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
