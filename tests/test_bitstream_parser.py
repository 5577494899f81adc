"""The library's native parser of the compressed file (fe_unpack, host
code, no GPU) against the oracle's packer (Sec. 3.3, Sec. 3.4)."""
import numpy as np
import pytest

from oracle import bitstream as bs
from oracle import mns
from paper_1501_02894_amd import binding as fb
from paper_1501_02894_amd import synth
from streams import random_stream
from test_oracle_bitstream import tiny_mixed, tiny_phase1, to_bytes


@pytest.mark.parametrize("name,make,b_max,b_min,thr,iso", [
    ("c1", lambda: synth.workload("c1"), 8, 4, [600], True),
    ("c2", lambda: synth.workload("c2"), 16, 4, [300, 200], True),
    ("c2 identity", lambda: synth.workload("c2"), 16, 4, [300, 200], False),
    ("c2 16->2", lambda: synth.workload("c2"), 16, 2, [300, 200, 100], False),
    ("c1 8->2", lambda: synth.workload("c1"), 8, 2, [600, 300], True),
    ("pw 32", lambda: synth.piecewise_smooth(192, 256, 13, cells=40), 32, 4, [120, 90, 60], True),
    ("noise 4", lambda: synth.noise_1f(16, 24, 18), 4, 4, [], True),
])
def test_parser_reads_oracle_files(name, make, b_max, b_min, thr, iso):
    img = make()
    H, W = img.shape
    r = mns.encode(img, b_max, b_min, thr, isometries=iso)
    data, nbits = bs.pack(r, W, H, b_max, b_min, isometries=iso)
    got, info = fb.fe_unpack(data, nbits)
    assert info == {"width": W, "height": H, "b_max": b_max, "b_min": b_min, "isometry": iso}
    assert got.tobytes() == np.ascontiguousarray(r).tobytes()


@pytest.mark.parametrize("W,H,bm,bmin,seed", [(96, 160, 32, 4, 1), (160, 96, 32, 8, 2), (64, 48, 16, 4, 3),
                                              (264, 136, 8, 4, 6), (64, 48, 16, 2, 7), (40, 24, 4, 2, 8)])
def test_parser_random_streams(W, H, bm, bmin, seed):
    r = random_stream(W, H, bm, bmin, seed, bounded=True)
    data, nbits = bs.pack(r, W, H, bm, bmin, isometries=True)
    assert fb.fe_unpack(data, nbits)[0].tobytes() == r.tobytes()


@pytest.mark.parametrize("maker", [tiny_phase1, tiny_mixed])
def test_parser_spelled_out_files(maker):
    recs, bits = maker()
    got, _ = fb.fe_unpack(to_bytes(bits), len(bits))
    assert got.tobytes() == recs.tobytes()


def test_parser_errors():
    recs, bits = tiny_mixed()
    data = to_bytes(bits)
    with pytest.raises(fb.FeError) as ei:
        fb.fe_unpack(data, len(bits) - 3)                 # truncated inside the last code
    assert ei.value.status == fb.FE_ERR_INVALID
    bad = bytearray(data)
    bad[7] |= 0x80                                        # a reserved header bit
    with pytest.raises(fb.FeError) as ei:
        fb.fe_unpack(bytes(bad), len(bits))
    assert ei.value.status == fb.FE_ERR_INVALID
    # too small an output buffer: the count needed is reported
    import ctypes
    buf = np.frombuffer(data, np.uint8)
    out = np.zeros(2, fb.TRANSFORM_DTYPE)
    n = ctypes.c_size_t(0)
    st = fb.load().fe_unpack(buf.ctypes.data, len(bits), out.ctypes.data, 2, ctypes.byref(n), None)
    assert st == fb.FE_ERR_CAPACITY and n.value == recs.size
