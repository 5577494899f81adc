"""Zoom decoding (Sec. 1: the decoder is resolution independent), CPU pins.

The attractor of the unrounded maps applied at twice the size, averaged
over 2 x 2 blocks, is the attractor at the native size: averaging a zoomed
range block 2 x 2 turns each zoomed domain value (a 2 x 2 mean of the zoomed
image) into the native one (a 2 x 2 mean of the averaged image), for every
isometry, and the native map has one fixed point.  Both attractors come from
the direct sparse solve, not from iterating."""
import numpy as np

from oracle import decode as odec
from oracle import mns
from paper_1501_02894_amd import synth
from streams import random_stream


def _avg2(x):
    return (x[0::2, 0::2] + x[0::2, 1::2] + x[1::2, 0::2] + x[1::2, 1::2]) / 4.0


def test_zoom_one_is_identity():
    rec = mns.encode(synth.workload("c1"), 8, 4, [600])
    assert odec.zoom(rec, 1).tobytes() == rec.tobytes()


def test_zoomed_attractor_averages_to_the_native_one():
    rec = mns.encode(synth.noise_1f(32, 32, 4), 8, 4, [300])
    assert np.any(rec["iso"] != 0)
    x1 = odec.fixed_point(rec, 32, 32, 8)
    x2 = odec.fixed_point(odec.zoom(rec, 2), 64, 64, 16)
    np.testing.assert_allclose(_avg2(x2), x1, atol=1e-7)


def test_zoomed_attractor_with_phase2_records():
    rec = random_stream(32, 32, 16, 4, 21, bounded=True)
    assert np.any(rec["flags"] != 0)
    x1 = odec.fixed_point(rec, 32, 32, 16)
    x2 = odec.fixed_point(odec.zoom(rec, 2), 64, 64, 32)
    np.testing.assert_allclose(_avg2(x2), x1, atol=1e-7)


def test_zoom_maps_odd_domains_to_even_ones():
    # 2 x 2 ranges have their domains at odd origins; zoomed by 2 they become
    # 4 x 4 ranges with even origins, so this ties the odd-phase means of the
    # 2 x 2 level to the plain 2 x 2 mean filter
    rec = mns.encode(synth.noise_1f(32, 32, 5), 8, 2, [300, 200])
    assert np.any(rec["level"] == 2) and np.any(rec["dx"] % 2)
    x1 = odec.fixed_point(rec, 32, 32, 8)
    x2 = odec.fixed_point(odec.zoom(rec, 2), 64, 64, 16)
    np.testing.assert_allclose(_avg2(x2), x1, atol=1e-7)
