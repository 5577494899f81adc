"""Oracle: the modified no-search (MNS) quadtree encoder, step by step.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Integer arithmetic in
numpy int64 throughout; no blocking, fusion or reordering beyond chunking the
list of ranges to bound memory.

The method (Sec. 3 and Sec. 3.1-3.3 of the paper):

* Ranges are B x B blocks; the top level partitions the image into
  B_max x B_max tiles (Sec. 3).  Levels l = 1..L with B_l = B_max >> (l-1).
* Each range has exactly one domain: the 2B x 2B block with the same centre,
  reduced to B x B by the mean of each 2 x 2 pixel group (Sec. 3, Fig. 1b).
* Only the contrast s and the luminance are fitted; if the error is below the
  level's threshold, or the level is the last one, the range is stored,
  otherwise it is split into four (Sec. 3).
* MNS adds a second phase for ranges that fail (Sec. 3.1, Technique 1): with
  O_i the range mean and O_k the four sub-block means, if every O_k is close
  to O_i, each sub-block is fitted with a contrast from a two-element set
  that depends on the level (Sec. 3.2), and the range is stored if all four
  sub-block errors are acceptable; O_4 is not stored but recovered from
  eq. (1), O_4 = 4 O_i - (O_1 + O_2 + O_3) (Sec. 3.3).

Readings of points the paper leaves open (each is listed with its reason in
the design notes):

* luminance is the quantised range mean m: the prediction is
  r^ = s (d - mean(d)) + m   (mean form; Sec. 3.3 stores one byte of it);
* phase-1 contrast uses 3 bits (Sec. 3.3) as s = k/8, k = 0..7;
* the 8 square isometries are tried in phase 1 (table ``ISOMETRY_TABLE``);
  phase 2 uses the identity only (one bit per sub-block, Sec. 3.2);
* the 2 x 2 mean rounds half up: (a + b + c + d + 2) >> 2;
* the co-centred domain origin is clamped into the image:
  dx = clamp(x - B/2, 0, W - 2B), likewise dy;
* the error is the collage error sum (r^ - r)^2 of the unrounded prediction,
  thresholds t_l are integer MSE values per level and the test is strict
  (MSE < t_l);
* "small enough" in Technique 1 means the difference fits the stored signed
  width of Sec. 3.3: |O_k - O_i| <= 2^(M-1) - 1, i.e. 15 at level 1 and 31 at
  levels 2 and 3; the derived O_4 must also be a valid 8-bit value;
* each sub-block in phase 2 uses its own co-centred domain (the one it would
  get at the next level) and must reach MSE < t_l of the parent's level;
* ties: lowest isometry, then lowest k; the mean rounds half up; phase 2
  prefers the first contrast of the set on equal error;
* the emitted stream is in depth-first (Z-order) sequence per top tile, tiles
  in raster order: children are numbered 0 = top-left, 1 = top-right,
  2 = bottom-left, 3 = bottom-right.

Scaled integer errors.  With n = B^2, Q = n*Sum d^2 - (Sum d)^2,
R = n*Sum r^2 - (Sum r)^2 and P_e = n*Sum r T_e(d) - Sum r * Sum d, the
phase-1 collage error E for contrast k/8 and luminance m satisfies
    64 n E = k^2 Q - 16 k P_e + 64 R + 64 (n m - Sum r)^2,
and for a phase-2 sub-block (contrast c/20, luminance O, nb = b^2 pixels)
    400 nb E = c^2 Q - 40 c P + 400 R + 400 (nb O - Sum r)^2.
"""
from __future__ import annotations

import numpy as np

# ---------------------------------------------------------------------------
# Record format: 16 bytes, little-endian, every byte defined.
# ---------------------------------------------------------------------------
RECORD_DTYPE = np.dtype([
    ("x", "<u2"), ("y", "<u2"),      # range top-left, pixels
    ("dx", "<u2"), ("dy", "<u2"),    # domain origin, pixels
    ("level", "u1"),                 # 0-based level: B = B_max >> level
    ("flags", "u1"),                 # bit 0: phase-2 record
    ("iso", "u1"),                   # phase 1: isometry 0..7; phase 2: 0
    ("s_idx", "u1"),                 # phase 1: k (s = k/8); phase 2: bit c -> 2nd contrast for child c
    ("lum", "u1"),                   # phase 1: m; phase 2: O_i
    ("dlum", "i1", (3,)),            # phase 2: O_c - O_i for c = 0, 1, 2; zero in phase 1
])
assert RECORD_DTYPE.itemsize == 16

FLAG_PHASE2 = 1

# Sec. 3.3: three bits of contrast in phase 1 -> s = k / 8, k = 0..7.
CONTRAST_DENOM = 8
CONTRAST_STEPS = 8

# Sec. 3.2: contrast sets for phase 2 per level, {.2,.5}, {.4,.65}, {.5,.9},
# held exactly as twentieths.
PHASE2_DENOM = 20
PHASE2_SETS = {1: (4, 10), 2: (8, 13), 3: (10, 18)}

# Sec. 3.3: M bits for each stored mean difference, one of them the sign;
# 5 bits at level 1 and 6 bits at levels 2 and 3.
PHASE2_BITS = {1: 5, 2: 6, 3: 6}
PHASE2_DELTA = {lvl: (1 << (bits - 1)) - 1 for lvl, bits in PHASE2_BITS.items()}

# Square isometries T_e: T_e(d)[i][j] = d[row(i, j)][col(i, j)], B x B block.
ISOMETRY_TABLE = {
    0: "identity",
    1: "mirror left-right",
    2: "mirror top-bottom",
    3: "rotate 180",
    4: "transpose",
    5: "rotate 90 clockwise",
    6: "rotate 90 counter-clockwise",
    7: "anti-transpose",
}

MAX_SIDE = 65536


def isometry_source(e: int, B: int):
    """Row and column index arrays (B x B) of the source pixel of T_e."""
    i, j = np.meshgrid(np.arange(B), np.arange(B), indexing="ij")
    last = B - 1
    table = {
        0: (i, j),
        1: (i, last - j),
        2: (last - i, j),
        3: (last - i, last - j),
        4: (j, i),
        5: (last - j, i),
        6: (j, last - i),
        7: (last - j, last - i),
    }
    return table[e]


def apply_isometry(block: np.ndarray, e: int) -> np.ndarray:
    """T_e applied to the last two axes of ``block``."""
    B = block.shape[-1]
    rows, cols = isometry_source(e, B)
    return block[..., rows, cols]


def _is_pow2(v: int) -> bool:
    return v > 0 and (v & (v - 1)) == 0


def num_levels(b_max: int, b_min: int) -> int:
    return int(np.log2(b_max // b_min)) + 1


def validate(width: int, height: int, b_max: int, b_min: int, thresholds) -> int:
    """Check the parameters; return the number of levels L.

    B_max and B_min are powers of two with 2 <= B_min <= B_max and
    4 <= B_max <= 32, and the quadtree has four levels at most (Sec. 3.3:
    two bits of level number; the paper's own tree runs 16 x 16 down to
    2 x 2); W and H are multiples of B_max and at least 2 B_max so that every
    co-centred 2B x 2B domain fits in the image; one threshold per level
    except the last, which is always stored (Sec. 3).
    """
    if not (_is_pow2(b_max) and _is_pow2(b_min)):
        raise ValueError("block sizes must be powers of two")
    if not (2 <= b_min <= b_max and 4 <= b_max <= 32):
        raise ValueError("need 2 <= b_min <= b_max, 4 <= b_max <= 32")
    if num_levels(b_max, b_min) > 4:
        raise ValueError("at most four quadtree levels (two level bits)")
    if width % b_max or height % b_max:
        raise ValueError("image sides must be multiples of b_max")
    if width < 2 * b_max or height < 2 * b_max:
        raise ValueError("image sides must be at least 2*b_max")
    if width > MAX_SIDE or height > MAX_SIDE:
        raise ValueError("image side too large")
    L = num_levels(b_max, b_min)
    if len(thresholds) != L - 1:
        raise ValueError("need one threshold per level except the last")
    for t in thresholds:
        if int(t) < 0 or int(t) >= 1 << 32:
            raise ValueError("thresholds are unsigned 32-bit MSE values")
    return L


def max_transforms(width: int, height: int, b_min: int) -> int:
    """Upper bound on the stream length: every range at the smallest size."""
    return (width // b_min) * (height // b_min)


# ---------------------------------------------------------------------------
# Sec. 3: the domain is the co-centred 2B x 2B block, 2 x 2 mean filtered.
# ---------------------------------------------------------------------------
def downsample(img: np.ndarray) -> np.ndarray:
    """H0[j][i] = round-half-up mean of I[2j..2j+1][2i..2i+1] (int64)."""
    I = np.asarray(img).astype(np.int64)
    a = I[0::2, 0::2]
    b = I[0::2, 1::2]
    c = I[1::2, 0::2]
    d = I[1::2, 1::2]
    return (a + b + c + d + 2) // 4


def phase_means(img: np.ndarray) -> np.ndarray:
    """The 2 x 2 round-half-up mean images at the four pixel phases:
    out[q, p, j, i] = mean of I[2j+q..2j+q+1][2i+p..2i+p+1] (zero where the
    group would leave the image); out[0, 0] is H0.  A 2 x 2 range at x has
    its domain at the odd origin x - 1, whose means lie on phase 1."""
    I = np.asarray(img).astype(np.int64)
    H, W = I.shape
    out = np.zeros((2, 2, H // 2, W // 2), np.int64)
    for q in range(2):
        for p in range(2):
            h, w = (H - q) // 2, (W - p) // 2
            out[q, p, :h, :w] = downsample(I[q:q + 2 * h, p:p + 2 * w])
    return out


def domain_origin(p, B: int, extent: int):
    """Origin of the 2B-wide domain co-centred with a B-wide range at p,
    clamped into [0, extent - 2B]."""
    return np.clip(np.asarray(p, np.int64) - B // 2, 0, extent - 2 * B)


def range_moments(I: np.ndarray, h0: np.ndarray, xs, ys, B: int) -> dict:
    """Integer moments of each range and its co-centred domain.

    Returns int64 arrays: sr = Sum r, srr = Sum r^2, sd = Sum d, sdd = Sum d^2
    and srd[:, e] = Sum r * T_e(d), where r is the B x B range at (x, y) and d
    the B x B window of H0 at the domain origin halved (of the phase-mean
    image of the origin's parity when an origin is odd, B = 2).
    """
    I = np.asarray(I, np.int64)
    H, W = I.shape
    xs = np.asarray(xs, np.int64)
    ys = np.asarray(ys, np.int64)
    R = xs.size
    n = B * B
    ox = domain_origin(xs, B, W)
    oy = domain_origin(ys, B, H)
    wx, wy = ox // 2, oy // 2
    if np.any(ox % 2) or np.any(oy % 2):
        ph = phase_means(I)
        h0 = None
    out = {k: np.zeros(R, np.int64) for k in ("sr", "srr", "sd", "sdd")}
    out["srd"] = np.zeros((R, 8), np.int64)
    ii = np.arange(B)
    src = [isometry_source(e, B) for e in range(8)]
    step = max(1, (1 << 21) // n)
    for s in range(0, R, step):
        sl = slice(s, min(R, s + step))
        r = I[ys[sl, None, None] + ii[None, :, None], xs[sl, None, None] + ii[None, None, :]]
        if h0 is not None:
            d = h0[wy[sl, None, None] + ii[None, :, None], wx[sl, None, None] + ii[None, None, :]]
        else:
            d = ph[(oy[sl] % 2)[:, None, None], (ox[sl] % 2)[:, None, None],
                   wy[sl, None, None] + ii[None, :, None], wx[sl, None, None] + ii[None, None, :]]
        out["sr"][sl] = r.sum(axis=(1, 2))
        out["srr"][sl] = (r * r).sum(axis=(1, 2))
        out["sd"][sl] = d.sum(axis=(1, 2))
        out["sdd"][sl] = (d * d).sum(axis=(1, 2))
        for e in range(8):
            rows, cols = src[e]
            out["srd"][sl, e] = (r * d[:, rows, cols]).sum(axis=(1, 2))
    return out


def quantised_mean(sr, n: int):
    """round-half-up(Sum r / n) in integers."""
    return (2 * np.asarray(sr, np.int64) + n) // (2 * n)


def fit_phase1(mom: dict, n: int):
    """Best (isometry e, contrast k/8) and luminance m of each range, and the
    scaled collage error S = 64 n E (Sec. 3: the no-search coder fits only
    the contrast to the one domain, then measures the error of that fit).

    Every (e, k) is scored; the first minimum in (e, k) order wins.
    """
    sr, srr, sd, sdd, srd = (mom[k] for k in ("sr", "srr", "sd", "sdd", "srd"))
    Q = n * sdd - sd * sd
    Rr = n * srr - sr * sr
    P = n * srd - (sr * sd)[:, None]                       # (R, 8)
    k = np.arange(CONTRAST_STEPS, dtype=np.int64)
    f = (k * k)[None, None, :] * Q[:, None, None] - 16 * k[None, None, :] * P[:, :, None]
    flat = f.reshape(len(sr), 8 * CONTRAST_STEPS)
    best = np.argmin(flat, axis=1)
    e = best // CONTRAST_STEPS
    kk = best % CONTRAST_STEPS
    fmin = flat[np.arange(len(sr)), best]
    m = quantised_mean(sr, n)
    S = fmin + 64 * Rr + 64 * (n * m - sr) ** 2
    return e, kk, m, S


def children_xy(xs, ys, B: int):
    """Top-left corners of the four B/2 sub-blocks, Z order (TL, TR, BL, BR)."""
    b = B // 2
    ox = np.array([0, b, 0, b], np.int64)
    oy = np.array([0, 0, b, b], np.int64)
    cx = (np.asarray(xs, np.int64)[:, None] + ox[None, :])
    cy = (np.asarray(ys, np.int64)[:, None] + oy[None, :])
    return cx, cy


def fit_phase2(I: np.ndarray, h0: np.ndarray, xs, ys, B: int, level: int, m, t: int):
    """Technique 1 (Sec. 3.1-3.3) for ranges that failed phase 1 at ``level``.

    Returns (accept, O, bits, S): O[:, c] the sub-block luminances with O[:, 3]
    from eq. (1), bits the per-child choice of the second contrast, S[:, c]
    the scaled sub-block errors 400 nb E_c.
    """
    b = B // 2
    nb = b * b
    c1, c2 = PHASE2_SETS[level]
    delta = PHASE2_DELTA[level]
    m = np.asarray(m, np.int64)
    R = m.size
    cx, cy = children_xy(xs, ys, B)
    mom = [range_moments(I, h0, cx[:, c], cy[:, c], b) for c in range(4)]
    O = np.zeros((R, 4), np.int64)
    for c in range(3):
        O[:, c] = quantised_mean(mom[c]["sr"], nb)
    O[:, 3] = 4 * m - O[:, 0] - O[:, 1] - O[:, 2]                      # eq. (1)
    accept = np.all(np.abs(O - m[:, None]) <= delta, axis=1)
    accept &= (O[:, 3] >= 0) & (O[:, 3] <= 255)
    bits = np.zeros(R, np.int64)
    S = np.zeros((R, 4), np.int64)
    for c in range(4):
        mc = mom[c]
        Q = nb * mc["sdd"] - mc["sd"] * mc["sd"]
        Rr = nb * mc["srr"] - mc["sr"] * mc["sr"]
        P = nb * mc["srd"][:, 0] - mc["sr"] * mc["sd"]
        f1 = c1 * c1 * Q - 40 * c1 * P
        f2 = c2 * c2 * Q - 40 * c2 * P
        use2 = f2 < f1
        f = np.where(use2, f2, f1)
        S[:, c] = f + 400 * Rr + 400 * (nb * O[:, c] - mc["sr"]) ** 2
        bits |= use2.astype(np.int64) << c
        accept &= S[:, c] < 400 * nb * nb * int(t)
    return accept, O, bits, S


def stream_key(x, y, width: int, b_max: int, b_min: int):
    """Depth-first position key: top-tile raster index * 4^(L-1) + Morton
    code of the b_min cell inside the tile (y bit above x bit per level)."""
    x = np.asarray(x, np.int64)
    y = np.asarray(y, np.int64)
    L = num_levels(b_max, b_min)
    tile = (y // b_max) * (width // b_max) + (x // b_max)
    lx = (x % b_max) // b_min
    ly = (y % b_max) // b_min
    code = np.zeros_like(x)
    for bit in range(L - 1):
        code |= ((lx >> bit) & 1) << (2 * bit)
        code |= ((ly >> bit) & 1) << (2 * bit + 1)
    return tile * (4 ** (L - 1)) + code


def _records(n: int) -> np.ndarray:
    return np.zeros(n, RECORD_DTYPE)


def encode(img: np.ndarray, b_max: int, b_min: int, thresholds, phase2: bool = True,
           trace: list | None = None, isometries: bool = True) -> np.ndarray:
    """MNS encoder: the record stream of ``img`` (uint8, H x W) in stream order.

    ``thresholds`` holds the integer MSE threshold of levels 1..L-1.  With
    ``phase2`` False this is the plain no-search coder of Sec. 3.  With
    ``isometries`` False phase 1 fits the identity only (the paper's 14-bit
    phase-1 code of Sec. 3.3 stores no isometry).  If ``trace`` is a list,
    one dict per level is appended with that level's worklist, moments, fit
    and decisions.
    """
    img = np.asarray(img)
    if img.dtype != np.uint8 or img.ndim != 2:
        raise ValueError("image must be a 2-D uint8 array")
    H, W = img.shape
    L = validate(W, H, b_max, b_min, thresholds)
    I = img.astype(np.int64)
    h0 = downsample(img)
    ys, xs = np.mgrid[0:H:b_max, 0:W:b_max]
    xs = xs.ravel().astype(np.int64)
    ys = ys.ravel().astype(np.int64)
    parts = []
    for level in range(1, L + 1):
        if xs.size == 0:
            break
        B = b_max >> (level - 1)
        n = B * B
        mom = range_moments(I, h0, xs, ys, B)
        if not isometries:
            # every isometry scores as the identity, so the first (e = 0) wins
            mom = dict(mom, srd=np.repeat(mom["srd"][:, :1], 8, axis=1))
        e, k, m, S = fit_phase1(mom, n)
        last = level == L
        if last:
            accept = np.ones(xs.size, bool)
        else:
            accept = S < 64 * n * n * int(thresholds[level - 1])
        rec = _records(int(accept.sum()))
        rec["x"], rec["y"] = xs[accept], ys[accept]
        rec["dx"] = domain_origin(xs[accept], B, W)
        rec["dy"] = domain_origin(ys[accept], B, H)
        rec["level"] = level - 1
        rec["iso"], rec["s_idx"], rec["lum"] = e[accept], k[accept], m[accept]
        parts.append(rec)
        info = {"level": level, "B": B, "x": xs, "y": ys, "moments": mom,
                "e": e, "k": k, "m": m, "S": S, "accept1": accept}
        if last:
            if trace is not None:
                trace.append(info)
            break
        fail = ~accept
        fx, fy, fm = xs[fail], ys[fail], m[fail]
        if phase2:
            ok2, O, bits, S2 = fit_phase2(I, h0, fx, fy, B, level, fm, thresholds[level - 1])
            rec2 = _records(int(ok2.sum()))
            rec2["x"], rec2["y"] = fx[ok2], fy[ok2]
            rec2["dx"] = domain_origin(fx[ok2], B, W)
            rec2["dy"] = domain_origin(fy[ok2], B, H)
            rec2["level"] = level - 1
            rec2["flags"] = FLAG_PHASE2
            rec2["s_idx"] = bits[ok2]
            rec2["lum"] = fm[ok2]
            rec2["dlum"] = (O[ok2, :3] - fm[ok2, None]).astype(np.int8)
            parts.append(rec2)
            split = ~ok2
            info.update({"accept2": ok2, "O": O, "bits": bits, "S2": S2})
        else:
            split = np.ones(fx.size, bool)
        if trace is not None:
            trace.append(info)
        cx, cy = children_xy(fx[split], fy[split], B)
        xs, ys = cx.ravel(), cy.ravel()
    rec = np.concatenate(parts) if parts else _records(0)
    key = stream_key(rec["x"], rec["y"], W, b_max, b_min)
    return rec[np.argsort(key, kind="stable")]


def stream_bytes(rec: np.ndarray) -> bytes:
    return np.ascontiguousarray(rec).tobytes()
