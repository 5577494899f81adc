"""Oracle: local search (Sec. 2, "local fractal coding"), between no-search
and the exhaustive search.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 2 restricts the domain pool of a range to the domain blocks that
surround it, with no isometries: for an 8 x 8 range, the 16 x 16 blocks that
contain it, 81 of them at step 1.  Here, for a B x B range at (x, y), the
candidates are the 2B x 2B blocks at step-1 origins (u, v) with
x - B <= u <= x and y - B <= v <= y (each contains the range), kept inside
the image; (B + 1)^2 of them away from the borders.  Each is reduced by the
2 x 2 round-half-up mean and fitted with the identity only, contrast k/8 and
luminance m as in phase 1 (same scaled error S = 64 n E).  The best candidate
has the least S; ties go to the lowest domain index v (W - 2B + 1) + u, then
the lowest k.  The quadtree uses the same thresholds and forced last level
as the exhaustive search, phase 1 only.

The co-centred domain of no-search, origin clamp(x - B/2, 0, W - 2B), is
always one of the candidates, so local search never does worse than
no-search with the identity only; and it never does better than the
exhaustive search restricted to the identity.
"""
from __future__ import annotations

import numpy as np

from .fullsearch import all_domains, closed_form_k
from .mns import RECORD_DTYPE, quantised_mean, stream_key, validate


def candidates(x: int, y: int, B: int, width: int, height: int):
    """Step-1 origins (u, v) of the domains surrounding the range at (x, y),
    in domain-index order (v major)."""
    us = np.arange(max(0, x - B), min(x, width - 2 * B) + 1)
    vs = np.arange(max(0, y - B), min(y, height - 2 * B) + 1)
    return [(int(u), int(v)) for v in vs for u in us]


def best_matches(img: np.ndarray, xs, ys, B: int):
    """Best surrounding domain of every range (x, y) of size B: int64 arrays
    (u, v, k, m, S)."""
    I = np.asarray(img).astype(np.int64)
    H, W = I.shape
    n = B * B
    nu = W - 2 * B + 1
    D = all_domains(img, B)
    out = {k: np.zeros(len(xs), np.int64) for k in ("u", "v", "k", "m", "S")}
    ii = np.arange(B)
    for r, (x, y) in enumerate(zip(np.asarray(xs, np.int64), np.asarray(ys, np.int64))):
        rng = I[y + ii[:, None], x + ii[None, :]].reshape(-1)
        sr, srr = int(rng.sum()), int((rng * rng).sum())
        cand = candidates(int(x), int(y), B, W, H)
        dom = np.array([v * nu + u for u, v in cand], np.int64)
        d = D[dom]                                   # (C, n)
        sd = d.sum(axis=1)
        Q = n * (d * d).sum(axis=1) - sd * sd
        P = n * (d @ rng) - sr * sd
        k = closed_form_k(P, Q)
        f = k * k * Q - 16 * k * P
        best = int(np.argmin(f))                     # lowest domain index on ties
        m = int(quantised_mean(sr, n))
        out["u"][r], out["v"][r] = cand[best]
        out["k"][r], out["m"][r] = int(k[best]), m
        out["S"][r] = int(f[best]) + 64 * (n * srr - sr * sr) + 64 * (n * m - sr) ** 2
    return out


def encode(img: np.ndarray, b_max: int, b_min: int, thresholds) -> np.ndarray:
    """Local-search quadtree coder: record stream in stream order (records
    carry the chosen domain origin in dx, dy; isometry 0)."""
    img = np.asarray(img)
    H, W = img.shape
    L = validate(W, H, b_max, b_min, thresholds)
    ys, xs = np.mgrid[0:H:b_max, 0:W:b_max]
    xs = xs.ravel().astype(np.int64)
    ys = ys.ravel().astype(np.int64)
    parts = []
    for level in range(1, L + 1):
        if xs.size == 0:
            break
        B = b_max >> (level - 1)
        n = B * B
        bm = best_matches(img, xs, ys, B)
        if level == L:
            accept = np.ones(xs.size, bool)
        else:
            accept = bm["S"] < 64 * n * n * int(thresholds[level - 1])
        rec = np.zeros(int(accept.sum()), RECORD_DTYPE)
        rec["x"], rec["y"] = xs[accept], ys[accept]
        rec["dx"], rec["dy"] = bm["u"][accept], bm["v"][accept]
        rec["level"] = level - 1
        rec["s_idx"], rec["lum"] = bm["k"][accept], bm["m"][accept]
        parts.append(rec)
        fx, fy = xs[~accept], ys[~accept]
        b = B // 2
        xs = (fx[:, None] + np.array([0, b, 0, b])).ravel()
        ys = (fy[:, None] + np.array([0, 0, b, b])).ravel()
    rec = np.concatenate(parts)
    return rec[np.argsort(stream_key(rec["x"], rec["y"], W, b_max, b_min), kind="stable")]
