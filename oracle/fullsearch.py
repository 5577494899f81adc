"""Oracle: exhaustive range-domain search, the baseline that no-search replaces.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 1: every 2B x 2B block of the image at step 1 is a candidate domain,
(W - 2B + 1)(H - 2B + 1) of them for a B x B range; the best domain, isometry
and contrast are the ones of minimum collage error.  The domain is reduced to
B x B by the same 2 x 2 round-half-up mean as in no-search, and the error is
the same scaled integer S = 64 n E (see ``mns``).  The quadtree uses the same
thresholds and forced last level, with phase 1 only.

For each (domain, isometry) the best k/8 is the closed form
k = clamp(ceil((16 P - Q) / (2 Q)), 0, 7) (k = 0 when Q = 0): the minimiser
over integers of the convex k^2 Q - 16 k P, lower k on ties.  Ties between
candidates go to the lowest domain index v * (W - 2B + 1) + u, then the lowest
isometry.  Sum r T_e(d) over all domains is a float64 matrix product, exact
because every partial sum is an integer below 2^53.
"""
from __future__ import annotations

import numpy as np

from .mns import (RECORD_DTYPE, domain_origin, isometry_source, num_levels,
                  quantised_mean, stream_key, validate)


def all_domains(img: np.ndarray, B: int) -> np.ndarray:
    """(ND, B*B) int64: the 2 x 2 mean-reduced domain at every step-1 origin
    (u, v), row index v * (W - 2B + 1) + u."""
    I = np.asarray(img).astype(np.int64)
    H, W = I.shape
    # 2 x 2 round-half-up mean at every pixel origin
    M = (I[:-1, :-1] + I[:-1, 1:] + I[1:, :-1] + I[1:, 1:] + 2) // 4
    win = np.lib.stride_tricks.sliding_window_view(M, (2 * B - 1, 2 * B - 1))
    win = win[: H - 2 * B + 1, : W - 2 * B + 1, ::2, ::2]
    return np.ascontiguousarray(win).reshape(-1, B * B)


def closed_form_k(P, Q):
    P = np.asarray(P, np.int64)
    Q = np.asarray(Q, np.int64)
    safeQ = np.where(Q > 0, Q, 1)
    num = 16 * P - Q
    k = -((-num) // (2 * safeQ))            # ceil division
    k = np.clip(k, 0, 7)
    return np.where(Q > 0, k, 0)


def best_matches(img: np.ndarray, xs, ys, B: int, chunk: int | None = None):
    """Exhaustive search for every range (x, y) of size B.

    Returns int64 arrays (dom, u, v, e, k, m, S): the best candidate's domain
    index and origin, isometry, contrast step, luminance and scaled error.
    """
    I = np.asarray(img).astype(np.int64)
    H, W = I.shape
    n = B * B
    xs = np.asarray(xs, np.int64)
    ys = np.asarray(ys, np.int64)
    D = all_domains(img, B)
    nu = W - 2 * B + 1
    sd = D.sum(axis=1)
    sdd = (D * D).sum(axis=1)
    Q = n * sdd - sd * sd
    Df = D.astype(np.float64)
    # T_e(d)[p] = d[src_e(p)] with src_e a permutation of the n positions, so
    # Sum_p r[p] T_e(d)[p] = Sum_q r_e[q] d[q] where r_e[src_e(p)] = r[p]: the
    # range is moved to the domain positions the isometry reads, and one
    # matrix product gives every (domain, isometry) pair at once
    flat_src = []
    for e in range(8):
        rows, cols = isometry_source(e, B)
        flat_src.append((rows * B + cols).ravel())
    R = xs.size
    ND = D.shape[0]
    if chunk is None:
        chunk = max(1, (1 << 24) // (8 * ND))
    out = {k: np.zeros(R, np.int64) for k in ("dom", "u", "v", "e", "k", "m", "S")}
    ii = np.arange(B)
    for s in range(0, R, chunk):
        sl = slice(s, min(R, s + chunk))
        r = I[ys[sl, None, None] + ii[None, :, None], xs[sl, None, None] + ii[None, None, :]]
        r = r.reshape(-1, n)
        sr = r.sum(axis=1)
        srr = (r * r).sum(axis=1)
        c = r.shape[0]
        re = np.empty((8, c, n), np.float64)
        for e in range(8):
            re[e][:, flat_src[e]] = r
        # (ND, 8 c): Sum r T_e(d) for every domain, isometry and range
        srd_all = np.rint(Df @ re.reshape(8 * c, n).T).astype(np.int64).reshape(ND, 8, c)
        f = np.empty((c, ND, 8), np.int64)
        kk = np.empty((c, ND, 8), np.int64)
        for e in range(8):
            P = n * srd_all[:, e, :].T - sr[:, None] * sd[None, :]
            k = closed_form_k(P, Q[None, :])
            kk[:, :, e] = k
            f[:, :, e] = k * k * Q[None, :] - 16 * k * P
        flat = f.reshape(c, -1)
        best = np.argmin(flat, axis=1)        # lowest domain index, then isometry
        dom = best // 8
        e = best % 8
        m = quantised_mean(sr, n)
        Rr = n * srr - sr * sr
        out["dom"][sl] = dom
        out["u"][sl] = dom % nu
        out["v"][sl] = dom // nu
        out["e"][sl] = e
        out["k"][sl] = kk[np.arange(c), dom, e]
        out["m"][sl] = m
        out["S"][sl] = flat[np.arange(c), best] + 64 * Rr + 64 * (n * m - sr) ** 2
    return out


def encode(img: np.ndarray, b_max: int, b_min: int, thresholds) -> np.ndarray:
    """Exhaustive-search quadtree coder: record stream in stream order."""
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
        rec["iso"], rec["s_idx"], rec["lum"] = bm["e"][accept], bm["k"][accept], bm["m"][accept]
        parts.append(rec)
        fx, fy = xs[~accept], ys[~accept]
        b = B // 2
        xs = (fx[:, None] + np.array([0, b, 0, b])).ravel()
        ys = (fy[:, None] + np.array([0, 0, b, b])).ravel()
    rec = np.concatenate(parts)
    return rec[np.argsort(stream_key(rec["x"], rec["y"], W, b_max, b_min), kind="stable")]


def num_candidates(width: int, height: int, B: int) -> int:
    """(W - 2B + 1)(H - 2B + 1) step-1 domain positions (Sec. 1)."""
    return (width - 2 * B + 1) * (height - 2 * B + 1)


__all__ = ["all_domains", "closed_form_k", "best_matches", "encode", "num_candidates",
           "domain_origin", "num_levels"]
