"""Seeded random transform streams for decoder tests.

A stream here is any valid set of records in the encoder's order: top tiles
in raster order, each split by a random quadtree whose leaves follow in
Morton order (y bit above x), every leaf a phase-1 record (random isometry,
contrast k/8 and mean, co-centred domain) or, for B >= 8 (B >= 4 when the
tree reaches 2 x 2), a phase-2 record
(random contrast bits and luminances O_c inside 0..255, Sec. 3.3).  The
decoded result of such a stream is fixed by the decoder's definition alone,
whatever the encoder would have chosen, so these streams reach record mixes
(level-0 phase-2 records, deep splits next to whole tiles) that encoded test
images rarely produce.
"""
import numpy as np

from oracle import mns


def random_stream(width: int, height: int, b_max: int, b_min: int, seed: int,
                  p_split: float = 0.5, p_phase2: float = 0.3, bounded: bool = False) -> np.ndarray:
    """With ``bounded`` the phase-2 differences O_c - O_i (all four, O_3 from
    eq. (1)) stay within the bound Technique 1 accepts, +-15 at level 1 and
    +-31 below, so that the stream fits the stored widths of Sec. 3.3."""
    rng = np.random.default_rng(seed)
    out = []

    def leaf(x, y, B, level):
        r = np.zeros((), mns.RECORD_DTYPE)
        r["x"], r["y"], r["level"] = x, y, level
        # phase 2 stands for a range that phase 1 did not accept, so an
        # encoder never emits it at the last level (a decoder still can take it)
        # phase-2 sub-blocks are at least 4 x 4, or 2 x 2 in a tree that reaches 2 x 2
        if B >= (4 if b_min == 2 else 8) and level <= 2 and (B > b_min or not bounded) and rng.random() < p_phase2:
            m = int(rng.integers(40, 216))
            if bounded:
                delta = mns.PHASE2_DELTA[level + 1]
                d = rng.integers(-delta, delta + 1, size=3)
                s01 = int(d[0] + d[1])   # d_2 and O_3 - m = -(d_0 + d_1 + d_2) both within +-delta
                d[2] = int(np.clip(d[2], max(-s01 - delta, -delta), min(-s01 + delta, delta)))
            else:
                d = rng.integers(-40, 41, size=3)
                s01 = int(d[0] + d[1])   # O_2 = m + d_2 and O_3 = m - (d_0 + d_1 + d_2) both in 0..255
                d[2] = int(np.clip(d[2], max(-s01 - 40, -m), min(-s01 + 40, 255 - m)))
            r["flags"] = mns.FLAG_PHASE2
            r["s_idx"] = int(rng.integers(0, 16))
            r["lum"] = m
            r["dlum"] = d
            r["dx"] = int(mns.domain_origin(x, B, width))
            r["dy"] = int(mns.domain_origin(y, B, height))
        else:
            r["iso"] = int(rng.integers(0, 8))
            r["s_idx"] = int(rng.integers(0, 8))
            r["lum"] = int(rng.integers(0, 256))
            r["dx"] = int(mns.domain_origin(x, B, width))
            r["dy"] = int(mns.domain_origin(y, B, height))
        out.append(r)

    def node(x, y, B, level):
        if B > b_min and rng.random() < p_split:
            h = B // 2
            for (ox, oy) in ((0, 0), (h, 0), (0, h), (h, h)):
                node(x + ox, y + oy, h, level + 1)
        else:
            leaf(x, y, B, level)

    for ty in range(height // b_max):
        for tx in range(width // b_max):
            node(tx * b_max, ty * b_max, b_max, 0)
    return np.array(out, mns.RECORD_DTYPE)
