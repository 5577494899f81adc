"""ctypes binding of libfe.so: argument marshalling only.

Every function mirrors the C entry point of the same name in include/fe.h.
Device buffers are torch tensors on the context's GPU (PyTorch supplies
memory and streams); every step of the method runs in the library's HIP
kernels.  If libfe.so is missing or cannot be loaded, every call raises:
there is no fallback path.

Typical use::

    import torch
    from paper_1501_02894_amd import binding as fb

    img = torch.from_numpy(gray_uint8_array).cuda()          # H x W, sides multiples of b_max
    with fb.Context(0) as ctx:
        t = ctx.encode(img, 16, 4, [300, 200])                # (n, 16) uint8 transform stream
        out = ctx.decode(t, img.shape[1], img.shape[0], 16, 12)       # 12 iterations from grey
        big = ctx.decode_zoom(t, img.shape[1], img.shape[0], 16, 2, 12)  # twice the size
        data, nbits = fb.fe_pack(ctx.handle, t, img.shape[1], img.shape[0], 16, 4)  # the file
    records, info = fb.fe_unpack(data.cpu().numpy().tobytes()[: (nbits + 7) // 8], nbits)

``encode_batch`` encodes a list of images in one launch, ``Plan`` records a
batch as a HIP graph, ``Server`` serves a stream of requests, and
``full_search=True`` / ``local_search=True`` select the search baselines.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfe.so")

FE_OK, FE_ERR_INVALID, FE_ERR_SHAPE, FE_ERR_CAPACITY, FE_ERR_DEVICE, FE_ERR_OOM, FE_ERR_BUSY = range(7)
FE_PHASE2 = 1
FE_FULL_SEARCH = 2
FE_IDENTITY_ONLY = 4
FE_LOCAL_SEARCH = 8
FE_TRANSFORM_PHASE2 = 1

# 16-byte transform layout of include/fe.h (little-endian).
TRANSFORM_DTYPE = np.dtype([
    ("x", "<u2"), ("y", "<u2"), ("dx", "<u2"), ("dy", "<u2"),
    ("level", "u1"), ("flags", "u1"), ("iso", "u1"), ("s_idx", "u1"),
    ("lum", "u1"), ("dlum", "i1", (3,)),
])
assert TRANSFORM_DTYPE.itemsize == 16


class FeError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_STATUS_NAMES = {0: "FE_OK", 1: "FE_ERR_INVALID", 2: "FE_ERR_SHAPE", 3: "FE_ERR_CAPACITY",
                 4: "FE_ERR_DEVICE", 5: "FE_ERR_OOM", 6: "FE_ERR_BUSY"}


class fe_params(ctypes.Structure):
    _fields_ = [("b_max", ctypes.c_uint32), ("b_min", ctypes.c_uint32), ("n_thr", ctypes.c_uint32),
                ("flags", ctypes.c_uint32), ("mse_thr", ctypes.c_uint32 * 4)]


class fe_stream_info(ctypes.Structure):
    _fields_ = [("width", ctypes.c_uint32), ("height", ctypes.c_uint32), ("b_max", ctypes.c_uint32),
                ("b_min", ctypes.c_uint32), ("flags", ctypes.c_uint32)]


class fe_image_desc(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("width", ctypes.c_uint32), ("height", ctypes.c_uint32),
                ("stride", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


_lib = None
_VP = ctypes.c_void_p
_U32 = ctypes.c_uint32
_SZ = ctypes.c_size_t

# name -> (restype, argtypes)
_SIGNATURES = {
    "fe_last_error": (ctypes.c_char_p, []),
    "fe_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "fe_version": (ctypes.c_int, []),
    "fe_validate": (ctypes.c_int, [_U32, _U32, _U32, ctypes.POINTER(fe_params)]),
    "fe_max_transforms": (_SZ, [_U32, _U32, _U32]),
    "fe_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_VP)]),
    "fe_destroy": (None, [_VP]),
    "fe_downsample": (ctypes.c_int, [_VP, _VP, _U32, _U32, _U32, _VP, _VP]),
    "fe_range_moments": (ctypes.c_int, [_VP, _VP, _U32, _U32, _U32, _U32, _VP, _U32, _VP, _VP]),
    "fe_encode": (ctypes.c_int, [_VP, _VP, _U32, _U32, _U32, ctypes.POINTER(fe_params), _VP, _SZ,
                                 ctypes.POINTER(_SZ), _VP]),
    "fe_encode_noalloc": (ctypes.c_int, [_VP, _VP, _U32, _U32, _U32, ctypes.POINTER(fe_params), _VP, _SZ, _VP,
                                         ctypes.POINTER(_SZ), _VP]),
    "fe_encode_batch": (ctypes.c_int, [_VP, ctypes.POINTER(fe_image_desc), _U32, ctypes.POINTER(fe_params),
                                       _VP, _SZ, _VP, ctypes.POINTER(_SZ), _VP]),
    "fe_plan_create": (ctypes.c_int, [_VP, ctypes.POINTER(fe_image_desc), _U32, ctypes.POINTER(fe_params), _VP, _SZ,
                                      _VP, ctypes.POINTER(_VP)]),
    "fe_plan_launch": (ctypes.c_int, [_VP, _VP]),
    "fe_plan_destroy": (None, [_VP]),
    "fe_decode": (ctypes.c_int, [_VP, _VP, _SZ, _U32, _U32, _U32, _U32, _VP, _VP, _VP]),
    "fe_decode_set_mode": (ctypes.c_int, [_VP, ctypes.c_int]),
    "fe_decode_last": (ctypes.c_int, [_VP]),
    "fe_decode_zoom": (ctypes.c_int, [_VP, _VP, _SZ, _U32, _U32, _U32, _U32, _U32, _VP, _VP, _VP]),
    "fe_pack_bound": (_SZ, [_SZ]),
    "fe_pack": (ctypes.c_int, [_VP, _VP, _SZ, _U32, _U32, _U32, _U32, _U32, _VP, _SZ, ctypes.POINTER(ctypes.c_uint64),
                               _VP]),
    "fe_unpack": (ctypes.c_int, [_VP, ctypes.c_uint64, _VP, _SZ, ctypes.POINTER(_SZ), ctypes.POINTER(fe_stream_info)]),
    "fe_full_search_ranges": (ctypes.c_int, [_VP, _VP, _U32, _U32, _U32, _U32, _VP, _U32, _VP, _VP]),
    "fe_server_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(fe_params), _SZ, _SZ, _U32, _U32,
                                        ctypes.POINTER(_VP)]),
    "fe_server_submit": (ctypes.c_int, [_VP, _VP, _U32, _U32, _U32, ctypes.POINTER(fe_params),
                                        ctypes.POINTER(ctypes.c_uint64)]),
    "fe_server_submit_pinned": (ctypes.c_int, [_VP, _VP, _U32, _U32, _U32, ctypes.POINTER(fe_params),
                                               ctypes.POINTER(ctypes.c_uint64)]),
    "fe_server_result": (ctypes.c_int, [_VP, ctypes.c_uint64, ctypes.POINTER(_VP), ctypes.POINTER(_SZ),
                                        ctypes.POINTER(ctypes.c_double)]),
    "fe_server_release": (ctypes.c_int, [_VP, ctypes.c_uint64]),
    "fe_server_poll": (ctypes.c_int, [_VP, ctypes.c_uint64, _VP, _SZ, ctypes.POINTER(_SZ), ctypes.POINTER(ctypes.c_int),
                                      ctypes.POINTER(ctypes.c_double)]),
    "fe_server_stats": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64),
                                       ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(_SZ), ctypes.POINTER(_U32),
                                       ctypes.POINTER(_U32)]),
    "fe_server_wait": (ctypes.c_int, [_VP, _U32, ctypes.POINTER(ctypes.c_uint64)]),
    "fe_server_request_times": (ctypes.c_int, [_VP, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double), _U32]),
    "fe_server_destroy": (None, [_VP]),
    "fe_tile_shapes": (ctypes.c_int, [_U32, _U32, ctypes.POINTER(_U32), ctypes.POINTER(_U32), ctypes.c_int]),
    "fe_set_tile_shape": (ctypes.c_int, [_VP, _U32, _U32, _U32, _U32]),
    "fe_get_tile_shape": (ctypes.c_int, [_VP, _U32, _U32, ctypes.POINTER(_U32), ctypes.POINTER(_U32)]),
    "fe_autotune": (ctypes.c_int, [_VP, ctypes.POINTER(fe_image_desc), _U32, ctypes.POINTER(fe_params), _VP, _SZ,
                                   _VP, _U32, ctypes.POINTER(_U32), ctypes.POINTER(_U32),
                                   ctypes.POINTER(ctypes.c_double), _VP]),
    "fe_timing_enable": (ctypes.c_int, [_VP, ctypes.c_int]),
    "fe_timing_select": (ctypes.c_int, [_VP, _U32]),
    "fe_timing_read": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_uint64),
                                      _U32]),
}

FE_TIMING_ENCODE, FE_TIMING_SCATTER, FE_TIMING_DECODE, FE_TIMING_FULLSEARCH = 0, 1, 2, 3
FE_TIMING_SLOTS = 8


def load(path: str = LIB_PATH):
    """Load libfe.so (once).  Raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run `python -m paper_1501_02894_amd.build`")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(lib, name, None)
        if fn is None:
            continue
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def declared_symbols(header: str) -> list[str]:
    """Names of the functions include/fe.h declares."""
    import re
    text = open(header).read()
    return sorted(set(re.findall(r"\b(fe_[a-z0-9_]+)\s*\(", text)))


def _check(status: int):
    if status != FE_OK:
        msg = load().fe_last_error().decode(errors="replace")
        raise FeError(status, msg)


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


def _stream(stream=None) -> int:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def make_params(b_max: int, b_min: int, thresholds, phase2: bool = True, full_search: bool = False,
                identity_only: bool = False, local_search: bool = False) -> fe_params:
    p = fe_params()
    p.b_max, p.b_min = int(b_max), int(b_min)
    thr = [int(t) for t in thresholds]
    p.n_thr = len(thr)
    p.flags = ((FE_PHASE2 if phase2 else 0) | (FE_FULL_SEARCH if full_search else 0) |
               (FE_IDENTITY_ONLY if identity_only else 0) | (FE_LOCAL_SEARCH if local_search else 0))
    for i, t in enumerate(thr[:4]):
        p.mse_thr[i] = t
    return p


# ------------------------------------------------------------------ C names
def fe_version() -> int:
    return int(load().fe_version())


def fe_validate(width: int, height: int, stride: int, params: fe_params) -> int:
    return int(load().fe_validate(width, height, stride, ctypes.byref(params)))


def fe_max_transforms(width: int, height: int, b_min: int) -> int:
    return int(load().fe_max_transforms(width, height, b_min))


def fe_create(device: int = 0) -> int:
    h = _VP()
    _check(load().fe_create(int(device), ctypes.byref(h)))
    return h.value


def fe_destroy(ctx: int) -> None:
    load().fe_destroy(ctx)


def fe_downsample(ctx: int, img, out=None, stream=None):
    import torch
    H, W = img.shape
    if out is None:
        out = torch.empty((H // 2, W // 2), dtype=torch.uint8, device=img.device)
    _check(load().fe_downsample(ctx, _ptr(img), W, H, img.stride(0), _ptr(out), _stream(stream)))
    return out


def fe_range_moments(ctx: int, img, block: int, xy, out=None, stream=None):
    """xy: int32 tensor of packed x | y << 16; returns (count, 12) int32
    tensor holding the uint32 moments."""
    import torch
    H, W = img.shape
    count = int(xy.numel())
    if out is None:
        out = torch.zeros((count, 12), dtype=torch.int32, device=img.device)
    _check(load().fe_range_moments(ctx, _ptr(img), W, H, img.stride(0), int(block), _ptr(xy), count,
                                   _ptr(out), _stream(stream)))
    return out


def fe_encode(ctx: int, img, params: fe_params, out=None, stream=None):
    """Returns a (n, 16) uint8 device tensor (view of `out`)."""
    import torch
    H, W = img.shape
    cap = fe_max_transforms(W, H, params.b_min)
    if out is None:
        out = torch.empty((cap, 16), dtype=torch.uint8, device=img.device)
    n = _SZ(0)
    _check(load().fe_encode(ctx, _ptr(img), W, H, img.stride(0), ctypes.byref(params), _ptr(out),
                            out.shape[0], ctypes.byref(n), _stream(stream)))
    return out[: n.value]


def fe_encode_noalloc(ctx: int, img, params: fe_params, out, offsets, wait: bool = True, stream=None):
    """The allocation-free encode: `out` ((cap, 16) uint8) and `offsets`
    (2 int64) are caller-owned device tensors.  Returns (out[:n], n) with
    wait=True, (out, None) with wait=False (the length is offsets[1])."""
    H, W = img.shape
    n = _SZ(0)
    _check(load().fe_encode_noalloc(ctx, _ptr(img), W, H, img.stride(0), ctypes.byref(params), _ptr(out),
                                    out.shape[0], _ptr(offsets), ctypes.byref(n) if wait else None,
                                    _stream(stream)))
    return (out[: n.value], n.value) if wait else (out, None)


def fe_encode_batch(ctx: int, imgs, params: fe_params, out=None, offsets=None, wait: bool = True,
                    stream=None, descs=None):
    """Returns (out, offsets, n): image k's stream is out[offsets[k]:offsets[k+1]].
    With wait=False the call does not synchronise and n is None.  `descs`
    (from image_descs) may be passed to reuse a descriptor array."""
    import torch
    if descs is None:
        descs = _descs(imgs)
    dev = imgs[0].device
    if out is None:
        cap = sum(fe_max_transforms(im.shape[1], im.shape[0], params.b_min) for im in imgs)
        out = torch.empty((cap, 16), dtype=torch.uint8, device=dev)
    if offsets is None:
        offsets = torch.zeros(len(imgs) + 1, dtype=torch.int64, device=dev)
    n = _SZ(0)
    _check(load().fe_encode_batch(ctx, descs, len(imgs), ctypes.byref(params), _ptr(out), out.shape[0],
                                  _ptr(offsets), ctypes.byref(n) if wait else None, _stream(stream)))
    return out, offsets, (n.value if wait else None)


def image_descs(imgs):
    """fe_image_desc array of device images (2-D uint8 tensors)."""
    return _descs(imgs)


def fe_plan_create(ctx: int, imgs, params: fe_params, out, offsets) -> int:
    """Record a batch encode of `imgs` into `out` / `offsets` (device tensors
    that must outlive the plan)."""
    descs = _descs(imgs)
    h = _VP()
    _check(load().fe_plan_create(ctx, descs, len(imgs), ctypes.byref(params), _ptr(out), out.shape[0],
                                 _ptr(offsets), ctypes.byref(h)))
    return h.value


def fe_plan_launch(plan: int, stream=None) -> None:
    _check(load().fe_plan_launch(plan, _stream(stream)))


def fe_plan_destroy(plan: int) -> None:
    load().fe_plan_destroy(plan)


class Plan:
    """Recorded batch encode; keeps references to its buffers."""

    def __init__(self, ctx, imgs, b_max, b_min, thresholds, out, offsets, phase2=True):
        self.imgs, self.out, self.offsets = list(imgs), out, offsets
        self.handle = fe_plan_create(ctx.handle, self.imgs, make_params(b_max, b_min, thresholds, phase2), out,
                                     offsets)

    def launch(self, stream=None):
        fe_plan_launch(self.handle, stream)

    def close(self):
        if self.handle:
            fe_plan_destroy(self.handle)
            self.handle = 0

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def fe_decode(ctx: int, transforms, width: int, height: int, b_max: int, iters: int, start=None, out=None,
              stream=None):
    import torch
    if out is None:
        out = torch.empty((height, width), dtype=torch.uint8, device=transforms.device)
    n = int(transforms.shape[0])
    _check(load().fe_decode(ctx, _ptr(transforms), n, width, height, b_max, iters, _ptr(start), _ptr(out),
                            _stream(stream)))
    return out


def fe_decode_zoom(ctx: int, transforms, width: int, height: int, b_max: int, zoom: int, iters: int, start=None,
                   out=None, stream=None):
    """Decode a stream of a width x height image at zoom times the size; the
    result is (zoom height, zoom width)."""
    import torch
    if out is None:
        out = torch.empty((height * zoom, width * zoom), dtype=torch.uint8, device=transforms.device)
    n = int(transforms.shape[0])
    _check(load().fe_decode_zoom(ctx, _ptr(transforms), n, width, height, b_max, zoom, iters, _ptr(start),
                                 _ptr(out), _stream(stream)))
    return out


FE_DECODE_AUTO, FE_DECODE_RECORDS, FE_DECODE_TILES = 0, 1, 2


def fe_decode_set_mode(ctx: int, mode: int) -> None:
    _check(load().fe_decode_set_mode(ctx, mode))


def fe_decode_last(ctx: int) -> int:
    return int(load().fe_decode_last(ctx))


FE_PACK_ISOMETRY = 1


def fe_pack_bound(n: int) -> int:
    return int(load().fe_pack_bound(n))


def fe_pack(ctx: int, transforms, width: int, height: int, b_max: int, b_min: int, isometry: bool = True,
            out=None, stream=None):
    """Compressed file of one image's transform stream (device (n, 16)
    uint8); returns (device uint8 buffer, length in bits)."""
    import torch
    n = int(transforms.shape[0])
    if out is None:
        out = torch.empty(fe_pack_bound(n), dtype=torch.uint8, device=transforms.device)
    nb = ctypes.c_uint64(0)
    _check(load().fe_pack(ctx, _ptr(transforms), n, width, height, b_max, b_min,
                          FE_PACK_ISOMETRY if isometry else 0, _ptr(out), int(out.numel()), ctypes.byref(nb),
                          _stream(stream)))
    return out, int(nb.value)


def fe_unpack(data, n_bits: int):
    """Parse a compressed file (host bytes) -> (records, info dict)."""
    buf = np.frombuffer(bytes(data), dtype=np.uint8)
    info = fe_stream_info()
    n = _SZ(0)
    lib = load()
    st = lib.fe_unpack(buf.ctypes.data, n_bits, None, 0, ctypes.byref(n), ctypes.byref(info))
    if st not in (FE_OK, FE_ERR_CAPACITY):
        _check(st)
    out = np.zeros(n.value, TRANSFORM_DTYPE)
    _check(lib.fe_unpack(buf.ctypes.data, n_bits, out.ctypes.data if n.value else None, n.value, ctypes.byref(n),
                         ctypes.byref(info)))
    return out, {"width": info.width, "height": info.height, "b_max": info.b_max, "b_min": info.b_min,
                 "isometry": bool(info.flags & FE_PACK_ISOMETRY)}


def fe_full_search_ranges(ctx: int, img, block: int, xy, out=None, stream=None):
    """Exhaustive best match of explicit ranges; returns an (n, 4) int32
    tensor: domain index, e | k << 8 | m << 16, S low, S high."""
    import torch
    H, W = img.shape
    count = int(xy.numel())
    if out is None:
        out = torch.zeros((count, 4), dtype=torch.int32, device=img.device)
    _check(load().fe_full_search_ranges(ctx, _ptr(img), W, H, img.stride(0), int(block), _ptr(xy), count,
                                        _ptr(out), _stream(stream)))
    return out


def fe_tile_shapes(b_max: int, b_min: int):
    gx = (_U32 * 16)()
    gy = (_U32 * 16)()
    k = load().fe_tile_shapes(b_max, b_min, gx, gy, 16)
    return [(gx[i], gy[i]) for i in range(min(k, 16))]


def fe_set_tile_shape(ctx: int, b_max: int, b_min: int, gx: int, gy: int) -> None:
    _check(load().fe_set_tile_shape(ctx, b_max, b_min, gx, gy))


def fe_get_tile_shape(ctx: int, b_max: int, b_min: int):
    gx, gy = _U32(0), _U32(0)
    _check(load().fe_get_tile_shape(ctx, b_max, b_min, ctypes.byref(gx), ctypes.byref(gy)))
    return gx.value, gy.value


def _descs(imgs):
    descs = (fe_image_desc * len(imgs))()
    for k, im in enumerate(imgs):
        H, W = im.shape
        descs[k].data = _ptr(im)
        descs[k].width, descs[k].height, descs[k].stride, descs[k].reserved = W, H, im.stride(0), 0
    return descs


def fe_autotune(ctx: int, imgs, params: fe_params, out, offsets, reps: int = 3, stream=None):
    """Time every built tile shape on this batch; the fastest is selected
    for the context.  Returns ((gx, gy), kernel ms)."""
    gx, gy, ms = _U32(0), _U32(0), ctypes.c_double(0)
    _check(load().fe_autotune(ctx, _descs(imgs), len(imgs), ctypes.byref(params), _ptr(out), out.shape[0],
                              _ptr(offsets), reps, ctypes.byref(gx), ctypes.byref(gy), ctypes.byref(ms),
                              _stream(stream)))
    return (gx.value, gy.value), ms.value


def fe_timing_select(ctx: int, slot_mask: int) -> None:
    """Time only the slots whose bits are set (default: all)."""
    _check(load().fe_timing_select(ctx, slot_mask))


def fe_timing_enable(ctx: int, enable: bool = True) -> None:
    _check(load().fe_timing_enable(ctx, 1 if enable else 0))


def fe_timing_read(ctx: int):
    """Returns (ms[8], launches[8]) per timed kernel slot, then clears."""
    ms = (ctypes.c_double * FE_TIMING_SLOTS)()
    cnt = (ctypes.c_uint64 * FE_TIMING_SLOTS)()
    _check(load().fe_timing_read(ctx, ms, cnt, FE_TIMING_SLOTS))
    return list(ms), list(cnt)


def to_records(t) -> np.ndarray:
    """Device (n, 16) uint8 tensor -> host structured array."""
    a = t.detach().cpu().numpy()
    return np.ascontiguousarray(a).view(TRANSFORM_DTYPE).reshape(-1)


def fe_server_create(device: int, params: fe_params, hbm_budget: int, host_budget: int, max_slots: int,
                     step_blocks: int) -> int:
    h = _VP()
    _check(load().fe_server_create(device, ctypes.byref(params), hbm_budget, host_budget, max_slots, step_blocks,
                                   ctypes.byref(h)))
    return h.value


def fe_server_submit(server: int, img: np.ndarray, params: fe_params = None) -> int:
    """Queue a host image; `params` (None: the server's) may change the
    thresholds and the phase-2 / identity-only flags, not the block sizes."""
    img = np.ascontiguousarray(img, dtype=np.uint8)
    H, W = img.shape
    req = ctypes.c_uint64(0)
    _check(load().fe_server_submit(server, img.ctypes.data, W, H, W,
                                   ctypes.byref(params) if params is not None else None, ctypes.byref(req)))
    return req.value


def fe_server_submit_pinned(server: int, img, params: fe_params = None) -> int:
    """Submit a 2-D uint8 torch tensor in pinned host memory (no host copy;
    keep it unchanged until the request is done)."""
    H, W = img.shape
    req = ctypes.c_uint64(0)
    _check(load().fe_server_submit_pinned(server, int(img.data_ptr()), W, H, img.stride(0),
                                          ctypes.byref(params) if params is not None else None, ctypes.byref(req)))
    return req.value


def fe_server_poll(server: int, req: int, fetch: bool = True):
    """Returns (done, records or None, latency_ms)."""
    lib = load()
    n = _SZ(0)
    done = ctypes.c_int(0)
    lat = ctypes.c_double(0)
    _check(lib.fe_server_poll(server, req, None, 0, ctypes.byref(n), ctypes.byref(done), ctypes.byref(lat)))
    if not done.value:
        return False, None, None
    if not fetch:
        return True, None, lat.value
    out = np.empty(max(n.value, 1), TRANSFORM_DTYPE)
    _check(lib.fe_server_poll(server, req, out.ctypes.data, out.size, ctypes.byref(n), ctypes.byref(done),
                              ctypes.byref(lat)))
    return True, out[: n.value], lat.value


def fe_server_result(server: int, req: int):
    """(records, latency_ms) of a done request: a numpy view of its records
    in the server's pinned host memory, valid until fe_server_release."""
    ptr = _VP()
    n = _SZ(0)
    lat = ctypes.c_double(0)
    _check(load().fe_server_result(server, req, ctypes.byref(ptr), ctypes.byref(n), ctypes.byref(lat)))
    if n.value == 0:
        return np.empty(0, TRANSFORM_DTYPE), lat.value
    buf = (ctypes.c_uint8 * (16 * n.value)).from_address(ptr.value)
    return np.frombuffer(buf, dtype=TRANSFORM_DTYPE), lat.value


def fe_server_release(server: int, req: int) -> None:
    _check(load().fe_server_release(server, req))


def fe_server_wait(server: int, timeout_us: int):
    """Id of the next finished request, or None if none finished in time."""
    req = ctypes.c_uint64(0)
    st = load().fe_server_wait(server, int(timeout_us), ctypes.byref(req))
    if st == FE_ERR_BUSY:
        return None
    _check(st)
    return req.value


def fe_server_request_times(server: int, req: int):
    """(admitted, first step, last step, complete), ms after submission, of
    a done request not yet fetched."""
    ms = (ctypes.c_double * 4)()
    _check(load().fe_server_request_times(server, req, ms, 4))
    return tuple(ms)


def fe_server_stats(server: int) -> dict:
    v = [ctypes.c_uint64(0) for _ in range(3)]
    used = _SZ(0)
    fl, q = _U32(0), _U32(0)
    _check(load().fe_server_stats(server, ctypes.byref(v[0]), ctypes.byref(v[1]), ctypes.byref(v[2]),
                                  ctypes.byref(used), ctypes.byref(fl), ctypes.byref(q)))
    return {"steps": v[0].value, "blocks": v[1].value, "completed": v[2].value, "hbm_used": used.value,
            "in_flight": fl.value, "queued": q.value}


def fe_server_destroy(server: int) -> None:
    load().fe_server_destroy(server)


class Server:
    """Continuous-batching encode server: block sizes fixed at creation,
    thresholds and flags per request (default: the creation's)."""

    def __init__(self, b_max, b_min, thresholds, phase2=True, device=0, hbm_budget=8 << 30,
                 host_budget=2 << 30, max_slots=256, step_blocks=4096):
        self.handle = fe_server_create(device, make_params(b_max, b_min, thresholds, phase2), hbm_budget,
                                       host_budget, max_slots, step_blocks)

    def submit(self, img, params=None):
        return fe_server_submit(self.handle, img, params)

    def submit_pinned(self, img, params=None):
        return fe_server_submit_pinned(self.handle, img, params)

    def poll(self, req, fetch=True):
        return fe_server_poll(self.handle, req, fetch)

    def wait(self, timeout_us=1000):
        return fe_server_wait(self.handle, timeout_us)

    def result(self, req):
        return fe_server_result(self.handle, req)

    def release(self, req):
        fe_server_release(self.handle, req)

    def request_times(self, req):
        return fe_server_request_times(self.handle, req)

    def stats(self):
        return fe_server_stats(self.handle)

    def close(self):
        if self.handle:
            fe_server_destroy(self.handle)
            self.handle = 0

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Context:
    """Owns one fe_ctx on a device; thin convenience over the C names."""

    def __init__(self, device: int = 0):
        self.device = device
        self.handle = fe_create(device)

    def close(self):
        if self.handle:
            fe_destroy(self.handle)
            self.handle = 0

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def downsample(self, img, **kw):
        return fe_downsample(self.handle, img, **kw)

    def range_moments(self, img, block, xy, **kw):
        return fe_range_moments(self.handle, img, block, xy, **kw)

    def encode(self, img, b_max, b_min, thresholds, phase2=True, full_search=False, identity_only=False,
               local_search=False, **kw):
        return fe_encode(self.handle, img, make_params(b_max, b_min, thresholds, phase2, full_search, identity_only,
                                                       local_search), **kw)

    def encode_batch(self, imgs, b_max, b_min, thresholds, phase2=True, **kw):
        return fe_encode_batch(self.handle, imgs, make_params(b_max, b_min, thresholds, phase2), **kw)

    def full_search_ranges(self, img, block, xy, **kw):
        return fe_full_search_ranges(self.handle, img, block, xy, **kw)

    def decode(self, transforms, width, height, b_max, iters, start=None, **kw):
        return fe_decode(self.handle, transforms, width, height, b_max, iters, start=start, **kw)

    def decode_zoom(self, transforms, width, height, b_max, zoom, iters, start=None, **kw):
        return fe_decode_zoom(self.handle, transforms, width, height, b_max, zoom, iters, start=start, **kw)

    def decode_mode(self, mode):
        fe_decode_set_mode(self.handle, mode)

    def decode_last(self):
        return fe_decode_last(self.handle)
