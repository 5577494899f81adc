"""The usage example of the binding's module docstring, run as written on
the 64 x 64 workload, and checked against the oracle."""
import numpy as np
import pytest

from oracle import bitstream as bs
from oracle import decode as odec
from oracle import mns
from paper_1501_02894_amd import binding as fb
from paper_1501_02894_amd import synth

pytestmark = pytest.mark.gpu


def test_docstring_example():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    gray_uint8_array = synth.workload("c1")
    img = torch.from_numpy(gray_uint8_array).cuda()
    with fb.Context(0) as ctx:
        t = ctx.encode(img, 8, 4, [600])
        out = ctx.decode(t, img.shape[1], img.shape[0], 8, 12)
        big = ctx.decode_zoom(t, img.shape[1], img.shape[0], 8, 2, 12)
        data, nbits = fb.fe_pack(ctx.handle, t, img.shape[1], img.shape[0], 8, 4)
    records, info = fb.fe_unpack(data.cpu().numpy().tobytes()[: (nbits + 7) // 8], nbits)
    want = mns.encode(gray_uint8_array, 8, 4, [600])
    assert fb.to_records(t).tobytes() == np.ascontiguousarray(want).tobytes()
    np.testing.assert_array_equal(out.cpu().numpy(), odec.decode(want, 64, 64, 8, 12))
    np.testing.assert_array_equal(big.cpu().numpy(), odec.decode(odec.zoom(want, 2), 128, 128, 16, 12))
    assert nbits == bs.pack(want, 64, 64, 8, 4)[1]
    assert records.tobytes() == np.ascontiguousarray(want).tobytes()
    assert (info["width"], info["height"], info["b_max"], info["b_min"]) == (64, 64, 8, 4)
