"""Oracle: the compressed file of Sec. 3.3 and Sec. 3.4 (Technique 2).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 3.3 stores, per range block in stream order, one bit telling phase 1
from phase 2 and two bits of level number (no domain position: the domain
is the co-centred one).  A phase-1 block then stores its luminance in one
byte and its contrast in three bits, 14 bits in all.  A phase-2 block stores
O_i in one byte, O_1..O_3 as M-bit differences from O_i whose first bit is
the sign (M = 5 at level 1, 6 at levels 2 and 3; O_4 follows from eq. (1)),
and one contrast bit S_j per sub-block.  Technique 2 (Sec. 3.4) drops the
level number of the three blocks that follow the first block of a group of
four siblings at the last level: they are known to lie at that level.

Readings (the paper gives the fields and their widths, not a file layout):

* bits are written least significant first, at increasing positions of the
  stream, stream bit p being bit p % 8 of byte p // 8; every field is
  written least significant bit first; the stream is zero-padded to a byte;
* a 64-bit header comes first: W - 1 (16 bits), H - 1 (16), log2 B_max (3),
  log2 B_min (3), the isometry flag (1), 25 zero bits;
* the phase bit is 1 for phase 2; the level number is the 0-based level;
* the encoder's phase 1 also fits the 8 isometries: with the isometry flag
  set each phase-1 block stores e in 3 more bits (17 bits); without it the
  stream must hold the identity only (encode with isometries off) and the
  phase-1 code is the paper's 14 bits;
* a stored difference O_k - O_i is sign (1 = negative) then magnitude in
  M - 1 bits, covering the +-(2^(M-1) - 1) that Technique 1 allows;
* Technique 2 applies when the quadtree has at least two levels: a block at
  the last level whose position is not the top-left child of its parent
  stores no level number (the decoder knows it continues a sibling group).

Decoding walks the quadtree: top tiles in raster order and, inside a tile,
blocks in depth-first (Morton) order, each block taking the next free cell.
"""
from __future__ import annotations

import numpy as np

from .mns import FLAG_PHASE2, PHASE2_BITS, RECORD_DTYPE, domain_origin, num_levels

HEADER_BITS = 64
LEVEL_BITS = 2
PHASE_BITS = 1


def level_elided(rec: np.ndarray, b_max: int, b_min: int) -> np.ndarray:
    """Technique 2: True for records that store no level number."""
    L = num_levels(b_max, b_min)
    rec = np.asarray(rec)
    if L < 2:
        return np.zeros(rec.size, bool)
    last = rec["level"].astype(np.int64) == L - 1
    child = ((rec["y"].astype(np.int64) // b_min) % 2) * 2 + (rec["x"].astype(np.int64) // b_min) % 2
    return last & (child != 0)


def code_lengths(rec: np.ndarray, b_max: int, b_min: int, isometries: bool) -> np.ndarray:
    """Bits of each record's code (Sec. 3.3, Sec. 3.4)."""
    rec = np.asarray(rec)
    p2 = (rec["flags"] & FLAG_PHASE2) != 0
    lvl1 = rec["level"].astype(np.int64) + 1                 # 1-based level
    M = np.array([PHASE2_BITS.get(int(v), 0) for v in lvl1], np.int64).reshape(-1)
    body1 = 8 + 3 + (3 if isometries else 0)
    body2 = 8 + 3 * M + 4
    n = PHASE_BITS + np.where(level_elided(rec, b_max, b_min), 0, LEVEL_BITS)
    return n + np.where(p2, body2, body1)


class _Writer:
    def __init__(self):
        self.bits: list[int] = []

    def put(self, value: int, width: int):
        if width and not 0 <= value < (1 << width):
            raise ValueError(f"{value} does not fit {width} bits")
        for b in range(width):
            self.bits.append((value >> b) & 1)

    def bytes(self) -> bytes:
        out = bytearray((len(self.bits) + 7) // 8)
        for p, bit in enumerate(self.bits):
            out[p // 8] |= bit << (p % 8)
        return bytes(out)


class _Reader:
    def __init__(self, data: bytes, nbits: int):
        self.data = data
        self.nbits = nbits
        self.pos = 0

    def get(self, width: int) -> int:
        if self.pos + width > self.nbits:
            raise ValueError("bitstream ends inside a code")
        v = 0
        for b in range(width):
            p = self.pos + b
            v |= ((self.data[p // 8] >> (p % 8)) & 1) << b
        self.pos += width
        return v


def _sign_magnitude(v: int, M: int) -> int:
    mag = abs(int(v))
    if mag > (1 << (M - 1)) - 1:
        raise ValueError(f"difference {v} does not fit {M} bits")
    return (1 if v < 0 else 0) | (mag << 1)


def pack(rec: np.ndarray, width: int, height: int, b_max: int, b_min: int,
         isometries: bool = True) -> tuple[bytes, int]:
    """The compressed stream of ``rec`` (stream order) and its length in bits."""
    rec = np.asarray(rec)
    L = num_levels(b_max, b_min)
    w = _Writer()
    w.put(width - 1, 16)
    w.put(height - 1, 16)
    w.put(int(b_max).bit_length() - 1, 3)
    w.put(int(b_min).bit_length() - 1, 3)
    w.put(1 if isometries else 0, 1)
    w.put(0, HEADER_BITS - 39)
    elided = level_elided(rec, b_max, b_min)
    for r, skip in zip(rec, elided):
        lvl = int(r["level"])
        if not 0 <= lvl < L:
            raise ValueError("level out of range")
        p2 = bool(int(r["flags"]) & FLAG_PHASE2)
        w.put(1 if p2 else 0, PHASE_BITS)
        if not skip:
            w.put(lvl, LEVEL_BITS)
        w.put(int(r["lum"]), 8)
        if not p2:
            w.put(int(r["s_idx"]), 3)
            if isometries:
                w.put(int(r["iso"]), 3)
            elif int(r["iso"]) != 0:
                raise ValueError("an isometry other than the identity needs the isometry flag")
        else:
            if lvl >= L - 1:
                raise ValueError("phase 2 stands for a range above the last level")
            M = PHASE2_BITS[lvl + 1]
            for c in range(3):
                w.put(_sign_magnitude(int(r["dlum"][c]), M), M)
            w.put(int(r["s_idx"]), 4)
    nbits = len(w.bits)
    return w.bytes(), nbits


def _morton_xy(code: int, bits: int):
    x = y = 0
    for b in range(bits):
        x |= ((code >> (2 * b)) & 1) << b
        y |= ((code >> (2 * b + 1)) & 1) << b
    return x, y


def unpack(data: bytes, nbits: int | None = None):
    """Parse a stream written by ``pack``: (records, W, H, b_max, b_min,
    isometries).  The records carry their co-centred domain origins."""
    if nbits is None:
        nbits = 8 * len(data)
    rd = _Reader(data, nbits)
    W = rd.get(16) + 1
    H = rd.get(16) + 1
    b_max = 1 << rd.get(3)
    b_min = 1 << rd.get(3)
    isometries = bool(rd.get(1))
    if rd.get(HEADER_BITS - 39) != 0:
        raise ValueError("reserved header bits set")
    L = num_levels(b_max, b_min)
    tiles_x, tiles_y = W // b_max, H // b_max
    cells = 4 ** (L - 1)
    out = []
    tile, cell = 0, 0
    prev_last_child = None        # child index of the previous record if it was at the last level
    while tile < tiles_x * tiles_y:
        r = np.zeros((), RECORD_DTYPE)
        p2 = rd.get(PHASE_BITS) == 1
        if L >= 2 and prev_last_child is not None and prev_last_child < 3:
            lvl = L - 1
        else:
            lvl = rd.get(LEVEL_BITS)
        if lvl >= L:
            raise ValueError("level number out of range")
        B = b_max >> lvl
        span = (B // b_min) ** 2
        if cell % span:
            raise ValueError("block not aligned at the next free cell")
        lx, ly = _morton_xy(cell, L - 1)
        x = (tile % tiles_x) * b_max + lx * b_min
        y = (tile // tiles_x) * b_max + ly * b_min
        r["x"], r["y"], r["level"] = x, y, lvl
        r["dx"] = int(domain_origin(x, B, W))
        r["dy"] = int(domain_origin(y, B, H))
        r["lum"] = rd.get(8)
        if not p2:
            r["s_idx"] = rd.get(3)
            r["iso"] = rd.get(3) if isometries else 0
        else:
            if lvl >= L - 1:
                raise ValueError("phase 2 at the last level")
            r["flags"] = FLAG_PHASE2
            M = PHASE2_BITS[lvl + 1]
            d = []
            for _ in range(3):
                v = rd.get(M)
                mag = v >> 1
                d.append(-mag if v & 1 else mag)
            r["dlum"] = d
            r["s_idx"] = rd.get(4)
        out.append(r)
        prev_last_child = ((y // b_min) % 2) * 2 + (x // b_min) % 2 if (L >= 2 and lvl == L - 1) else None
        cell += span
        if cell == cells:
            tile, cell = tile + 1, 0
    return np.array(out, RECORD_DTYPE), W, H, b_max, b_min, isometries


def bits_per_pixel(nbits: int, width: int, height: int) -> float:
    return nbits / float(width * height)


def compression_ratio(nbits: int, width: int, height: int) -> float:
    """8-bit image size over the stream size (whole bytes)."""
    return (8.0 * width * height) / (8 * ((nbits + 7) // 8))
