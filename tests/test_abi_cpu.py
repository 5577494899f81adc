"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function the header declares, validates requests exactly like the
oracle's statement of the constraints, and fails cleanly without a device."""
import ctypes
import itertools
import os

import pytest

from oracle import mns
from paper_1501_02894_amd import binding as fb

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "fe.h")


@pytest.fixture(scope="module")
def lib():
    return fb.load()


def test_exports_every_declared_symbol(lib):
    names = fb.declared_symbols(HEADER)
    assert "fe_encode" in names and "fe_decode" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert missing == []


def test_status_strings(lib):
    for code, name in fb._STATUS_NAMES.items():
        assert lib.fe_status_string(code).decode() == name
    assert lib.fe_version() >= 10000


def test_transform_layout():
    assert fb.TRANSFORM_DTYPE == mns.RECORD_DTYPE.newbyteorder("<") or \
        fb.TRANSFORM_DTYPE.descr == mns.RECORD_DTYPE.descr
    assert ctypes.sizeof(fb.fe_params) == 32


def _oracle_ok(w, h, b_max, b_min, n_thr):
    try:
        mns.validate(w, h, b_max, b_min, [1] * n_thr)
        return True
    except ValueError:
        return False


def test_validation_agrees_with_oracle(lib):
    sizes = [(64, 64), (48, 64), (16, 16), (8, 8), (60, 64), (32, 40), (96, 32), (4, 4), (128, 8)]
    blocks = [(4, 4), (8, 4), (16, 4), (16, 8), (32, 4), (32, 16), (64, 8), (8, 2), (6, 3), (8, 16), (16, 2),
              (32, 2), (4, 2), (2, 2), (8, 1)]
    for (w, h), (bmax, bmin) in itertools.product(sizes, blocks):
        for n_thr in range(0, 5):
            p = fb.fe_params()
            p.b_max, p.b_min, p.n_thr, p.flags = bmax, bmin, n_thr, fb.FE_PHASE2
            st = fb.fe_validate(w, h, w, p)
            assert (st == fb.FE_OK) == _oracle_ok(w, h, bmax, bmin, n_thr), (w, h, bmax, bmin, n_thr, st)
            if st != fb.FE_OK:
                assert lib.fe_last_error().decode()


def test_validation_codes():
    p = fb.make_params(16, 4, [300, 200])
    assert fb.fe_validate(64, 64, 64, p) == fb.FE_OK
    assert fb.fe_validate(64, 64, 62, p) == fb.FE_ERR_SHAPE      # stride < width
    assert fb.fe_validate(64, 64, 66, p) == fb.FE_ERR_SHAPE      # stride not a multiple of 4
    assert fb.fe_validate(64, 64, 68, p) == fb.FE_OK
    assert fb.fe_validate(72, 64, 72, p) == fb.FE_ERR_SHAPE      # not a multiple of b_max
    assert fb.fe_validate(16, 64, 16, p) == fb.FE_ERR_SHAPE      # smaller than 2 b_max
    assert fb.fe_validate(65536 + 16, 64, 65536 + 16, p) == fb.FE_ERR_SHAPE
    bad = fb.make_params(16, 4, [300])
    assert fb.fe_validate(64, 64, 64, bad) == fb.FE_ERR_INVALID
    bad = fb.make_params(16, 4, [300, 200])
    bad.flags = 16                                                # unknown flag
    assert fb.fe_validate(64, 64, 64, bad) == fb.FE_ERR_INVALID
    for flags in (fb.FE_FULL_SEARCH | fb.FE_LOCAL_SEARCH, fb.FE_FULL_SEARCH | fb.FE_IDENTITY_ONLY,
                  fb.FE_LOCAL_SEARCH | fb.FE_IDENTITY_ONLY):
        bad.flags = flags                                         # combinations that exclude each other
        assert fb.fe_validate(64, 64, 64, bad) == fb.FE_ERR_INVALID
    assert fb.load().fe_validate(64, 64, 64, None) == fb.FE_ERR_INVALID


def test_max_transforms():
    assert fb.fe_max_transforms(512, 512, 4) == mns.max_transforms(512, 512, 4) == 16384
    assert fb.fe_max_transforms(64, 32, 8) == 32
    assert fb.fe_max_transforms(64, 32, 0) == 0


def test_no_device_is_a_clean_error(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    st = lib.fe_create(0, ctypes.byref(h))
    assert st == fb.FE_ERR_DEVICE and not h.value
    assert lib.fe_last_error().decode()


def test_null_arguments(lib):
    assert lib.fe_create(0, None) == fb.FE_ERR_INVALID
    p = fb.make_params(16, 4, [300, 200])
    n = ctypes.c_size_t(0)
    assert lib.fe_encode(None, None, 64, 64, 64, ctypes.byref(p), None, 0, ctypes.byref(n), None) == fb.FE_ERR_INVALID
    assert lib.fe_decode(None, None, 0, 64, 64, 16, 1, None, None, None) == fb.FE_ERR_INVALID
    assert lib.fe_decode_zoom(None, None, 0, 64, 64, 16, 2, 1, None, None, None) == fb.FE_ERR_INVALID
    lib.fe_destroy(None)
    assert lib.fe_timing_select(None, 1) == fb.FE_ERR_INVALID
    assert lib.fe_decode_set_mode(None, 0) == fb.FE_ERR_INVALID
    assert lib.fe_decode_last(None) == fb.FE_DECODE_RECORDS
