"""Oracle: decoding by iterating the stored contractive maps (Sec. 1, IFS).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The decoder starts from an arbitrary image and applies every stored transform
to the current iterate (Jacobi: all pixels of iterate t+1 are computed from
iterate t).  A phase-1 record maps its domain, 2 x 2 mean filtered and taken
under isometry e, to the range with r^ = (k/8)(d - mean d) + m; a phase-2
record maps each of its four sub-blocks from the sub-block's own co-centred
domain with contrast from the level's set and luminance O_c, O_3 (the
paper's O_4) recovered by eq. (1) (Sec. 3.1-3.3).

Three variants:
  decode(..., mode="int")        exact integers: domain pixels are
                                 round-half-up 2 x 2 means, the prediction
                                 rounds half up (floor division) and clamps
                                 to 0..255;
  decode(..., mode="float")      the same map in float64 with floor(v + 0.5);
  decode(..., mode="unrounded")  no rounding of domain means or of the
                                 prediction and no clamp -- the affine IFS map
                                 whose fixed point ``fixed_point`` solves
                                 directly.
"""
from __future__ import annotations

import numpy as np

from .mns import (FLAG_PHASE2, PHASE2_DENOM, PHASE2_SETS, CONTRAST_DENOM,
                  isometry_source)


def pieces(rec: np.ndarray, width: int, height: int, b_max: int) -> dict:
    """Expand records into affine pieces, one per mapped block.

    Each piece: block (x, y, B), domain origin (dx, dy), isometry e, contrast
    num/den and luminance lum.  A phase-2 record yields four pieces.
    """
    out = {k: [] for k in ("x", "y", "B", "dx", "dy", "e", "num", "den", "lum")}
    rec = np.asarray(rec)
    p1 = (rec["flags"] & FLAG_PHASE2) == 0
    r1 = rec[p1]
    out["x"].append(r1["x"].astype(np.int64))
    out["y"].append(r1["y"].astype(np.int64))
    out["B"].append(b_max >> r1["level"].astype(np.int64))
    out["dx"].append(r1["dx"].astype(np.int64))
    out["dy"].append(r1["dy"].astype(np.int64))
    out["e"].append(r1["iso"].astype(np.int64))
    out["num"].append(r1["s_idx"].astype(np.int64))
    out["den"].append(np.full(r1.size, CONTRAST_DENOM, np.int64))
    out["lum"].append(r1["lum"].astype(np.int64))
    r2 = rec[~p1]
    if r2.size:
        lvl = r2["level"].astype(np.int64) + 1          # 1-based level of the parent
        B = b_max >> (lvl - 1)
        b = B // 2
        m = r2["lum"].astype(np.int64)
        d = r2["dlum"].astype(np.int64)
        O = np.stack([m + d[:, 0], m + d[:, 1], m + d[:, 2],
                      4 * m - (m + d[:, 0]) - (m + d[:, 1]) - (m + d[:, 2])], 1)
        sets = np.array([PHASE2_SETS[int(v)] for v in lvl], np.int64).reshape(-1, 2)
        for c in range(4):
            cx = r2["x"].astype(np.int64) + (c % 2) * b
            cy = r2["y"].astype(np.int64) + (c // 2) * b
            bit = (r2["s_idx"].astype(np.int64) >> c) & 1
            out["x"].append(cx)
            out["y"].append(cy)
            out["B"].append(b)
            # each sub-block's own co-centred domain, clamped into the image
            out["dx"].append(np.clip(cx - b // 2, 0, width - 2 * b))
            out["dy"].append(np.clip(cy - b // 2, 0, height - 2 * b))
            out["e"].append(np.zeros(r2.size, np.int64))
            out["num"].append(sets[np.arange(r2.size), bit])
            out["den"].append(np.full(r2.size, PHASE2_DENOM, np.int64))
            out["lum"].append(O[:, c])
    return {k: np.concatenate(v) if v else np.zeros(0, np.int64) for k, v in out.items()}


def _domain_blocks(x: np.ndarray, dx, dy, B: int, rounded: bool):
    """2 x 2 means of the iterate over each 2B x 2B domain -> (R, B, B)."""
    ii = np.arange(B)
    rows = dy[:, None, None] + 2 * ii[None, :, None]
    cols = dx[:, None, None] + 2 * ii[None, None, :]
    s = x[rows, cols] + x[rows, cols + 1] + x[rows + 1, cols] + x[rows + 1, cols + 1]
    if rounded:
        return (s + 2) // 4
    return s / 4.0


def _apply(x: np.ndarray, pc: dict, mode: str) -> np.ndarray:
    H, W = x.shape
    rounded = mode != "unrounded"
    new = np.zeros((H, W), np.int64 if mode == "int" else np.float64)
    cover = np.zeros((H, W), np.int64)
    keys = set(zip(pc["B"].tolist(), pc["e"].tolist()))
    for B, e in sorted(keys):
        sel = (pc["B"] == B) & (pc["e"] == e)
        n = B * B
        d = _domain_blocks(x, pc["dx"][sel], pc["dy"][sel], B, rounded)
        rows, cols = isometry_source(e, B)
        td = d[:, rows, cols]
        sd = d.sum(axis=(1, 2))
        num = pc["num"][sel][:, None, None]
        den = pc["den"][sel][:, None, None]
        lum = pc["lum"][sel][:, None, None]
        if mode == "int":
            v = num * (n * td - sd[:, None, None]) + den * n * lum
            v = (v + den * n // 2) // (den * n)
            v = np.clip(v, 0, 255)
        else:
            v = (num / den) * (td - (sd / n)[:, None, None]) + lum
            if mode == "float":
                v = np.clip(np.floor(v + 0.5), 0, 255)
        ii = np.arange(B)
        ry = pc["y"][sel][:, None, None] + ii[None, :, None]
        rx = pc["x"][sel][:, None, None] + ii[None, None, :]
        ry, rx = np.broadcast_arrays(ry, rx)
        new[ry, rx] = v
        np.add.at(cover, (ry.ravel(), rx.ravel()), 1)
    if not np.all(cover == 1):
        raise ValueError("transforms do not tile the image exactly once")
    return new


def decode(rec: np.ndarray, width: int, height: int, b_max: int, iters: int,
           start: np.ndarray | None = None, mode: str = "int") -> np.ndarray:
    """Iterate the transforms ``iters`` times from ``start`` (grey 128 if
    None).  Returns uint8 for "int"/"float", float64 for "unrounded"."""
    if mode not in ("int", "float", "unrounded"):
        raise ValueError(mode)
    pc = pieces(rec, width, height, b_max)
    if start is None:
        x = np.full((height, width), 128, np.int64)
    else:
        x = np.asarray(start).astype(np.int64 if mode == "int" else np.float64)
    if mode != "int":
        x = x.astype(np.float64)
    for _ in range(iters):
        x = _apply(x, pc, mode)
    if mode == "unrounded":
        return x
    return x.astype(np.uint8)


def zoom(rec: np.ndarray, factor: int) -> np.ndarray:
    """Resolution-independent decoding (Sec. 1): the same maps at `factor`
    times the size.  Ranges and domain origins scale by the factor, while
    levels, contrasts and luminances stay; decode the result as a
    (factor W) x (factor H) image with factor * b_max.  The co-centred
    domain of a phase-2 sub-block scales the same way:
    clamp(f x - f b / 2, 0, f W - 2 f b) = f clamp(x - b / 2, 0, W - 2 b)."""
    out = np.array(rec, copy=True)
    for k in ("x", "y", "dx", "dy"):
        out[k] = out[k].astype(np.int64) * int(factor)
    return out


def fixed_point(rec: np.ndarray, width: int, height: int, b_max: int) -> np.ndarray:
    """Attractor of the unrounded map x = A x + b, by a direct sparse solve of
    (I - A) x = b (small images only)."""
    from scipy.sparse import coo_matrix, identity
    from scipy.sparse.linalg import spsolve

    pc = pieces(rec, width, height, b_max)
    N = width * height
    rows, cols, vals = [], [], []
    b = np.zeros(N)
    for idx in range(pc["x"].size):
        B = int(pc["B"][idx])
        n = B * B
        e = int(pc["e"][idx])
        s = pc["num"][idx] / pc["den"][idx]
        dx, dy = int(pc["dx"][idx]), int(pc["dy"][idx])
        srow, scol = isometry_source(e, B)
        # every pixel of the 2B x 2B domain enters mean(d) with weight 1/(4n)
        dom = [(dy + a) * width + (dx + c) for a in range(2 * B) for c in range(2 * B)]
        for i in range(B):
            for j in range(B):
                p = (int(pc["y"][idx]) + i) * width + int(pc["x"][idx]) + j
                b[p] = pc["lum"][idx]
                si, sj = int(srow[i, j]), int(scol[i, j])
                for (a, c) in ((0, 0), (0, 1), (1, 0), (1, 1)):
                    rows.append(p)
                    cols.append((dy + 2 * si + a) * width + dx + 2 * sj + c)
                    vals.append(s / 4.0)
                for q in dom:
                    rows.append(p)
                    cols.append(q)
                    vals.append(-s / (4.0 * n))
    A = coo_matrix((vals, (rows, cols)), shape=(N, N)).tocsr()
    x = spsolve((identity(N, format="csr") - A).tocsc(), b)
    return x.reshape(height, width)
