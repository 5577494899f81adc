"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: constants
the paper prints (tests/golden/paper_constants.json), library routines for
the square isometries, brute force over the quantised grids, pixelwise
errors in exact rational arithmetic, closed-form fixed points and invariants.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import decode, fullsearch, metrics, mns
from paper_1501_02894_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")


@pytest.fixture(scope="module")
def golden():
    with open(GOLDEN) as f:
        return json.load(f)


def geometric_isometry(d, e):
    """The eight square isometries by their geometric names (numpy routines)."""
    return [
        d,
        np.fliplr(d),
        np.flipud(d),
        np.rot90(d, 2),
        d.T,
        np.rot90(d, -1),      # clockwise
        np.rot90(d, 1),       # counter-clockwise
        np.rot90(d, 2).T,     # anti-transpose
    ][e]


# ---------------------------------------------------------------- constants
def test_paper_constants(golden):
    sets = golden["phase2_contrast_sets"]["values"]
    for lvl, (a, b) in sets.items():
        c1, c2 = mns.PHASE2_SETS[int(lvl)]
        assert Fraction(c1, mns.PHASE2_DENOM) == Fraction(str(a))
        assert Fraction(c2, mns.PHASE2_DENOM) == Fraction(str(b))
    bits = golden["phase1_bits"]
    assert 2 ** bits["contrast"] == mns.CONTRAST_STEPS
    assert mns.CONTRAST_STEPS <= mns.CONTRAST_DENOM   # all s < 1 (contractive)
    for lvl, M in golden["phase2_mean_bits"]["values"].items():
        # M bits with one sign bit: magnitudes 0 .. 2^(M-1) - 1
        assert mns.PHASE2_DELTA[int(lvl)] == 2 ** (M - 1) - 1
    b = golden["phase1_bits_per_block"]
    assert b["luminance"] + b["contrast"] + b["level_id"] + b["phase"] == b["total"]
    q = golden["quadtree_levels"]
    assert int(np.log2(q["b_max"] // q["b_min"])) + 1 == q["levels"]


def test_eq1_examples(golden):
    # O_4 = 4 O_i - (O_1 + O_2 + O_3), and the decoder's expansion recovers it
    for Oi, O1, O2, O3, O4 in golden["eq1"]["examples"]:
        assert 4 * Oi - (O1 + O2 + O3) == O4
        rec = np.zeros(1, mns.RECORD_DTYPE)
        rec["level"], rec["flags"], rec["lum"] = 0, mns.FLAG_PHASE2, Oi
        rec["dlum"] = [O1 - Oi, O2 - Oi, O3 - Oi]
        pc = decode.pieces(rec, 64, 64, 16)
        assert sorted(pc["lum"].tolist()) == sorted([O1, O2, O3, O4])


def test_counting_formulas(golden):
    for N, n, ranges, domains in golden["counts"]["examples"]:
        img = np.zeros((N, N), np.uint8)
        ys, xs = np.mgrid[0:N:n, 0:N:n]
        assert xs.size == ranges == (N // n) ** 2
        assert fullsearch.num_candidates(N, N, n) == domains
        if N <= 64:
            assert fullsearch.all_domains(img, n).shape == (domains, n * n)
    ls = golden["local_search_candidates"]
    # domains of the given size that contain the range, at step 1
    assert (ls["domain"] - ls["range"] + 1) ** 2 == ls["candidates"]


def test_psnr_closed_form(golden):
    rng = np.random.default_rng(7)
    a = rng.integers(0, 256, (32, 32)).astype(np.uint8)
    for mse_val, db in golden["psnr"]["examples"]:
        assert 10 * np.log10(255.0 ** 2 / mse_val) == pytest.approx(db, abs=1e-12)
    b = a.astype(np.int64).copy()
    b[::2, ::2] += np.where(b[::2, ::2] < 255, 1, -1)   # 256 pixels off by exactly 1
    assert metrics.mse(a, b) == pytest.approx(256 / 1024)
    assert metrics.psnr(a, b) == pytest.approx(10 * np.log10(255 ** 2 * 4), abs=1e-12)
    assert metrics.psnr(a, a) == float("inf")


# ---------------------------------------------------------------- isometries
@pytest.mark.parametrize("B", [4, 8, 16, 32])
def test_isometry_table_is_the_square_group(B):
    rng = np.random.default_rng(B)
    d = rng.integers(0, 256, (B, B))
    seen = set()
    for e in range(8):
        t = mns.apply_isometry(d, e)
        np.testing.assert_array_equal(t, geometric_isometry(d, e))
        seen.add(t.tobytes())
    assert len(seen) == 8


# ---------------------------------------------------------------- domain
def test_downsample_round_half_up():
    rng = np.random.default_rng(1)
    img = rng.integers(0, 256, (12, 20)).astype(np.uint8)
    img[0:2, 0:2] = [[0, 1], [0, 1]]          # mean 0.5 -> 1
    img[0:2, 2:4] = [[255, 254], [255, 255]]  # mean 254.75 -> 255
    img[2:4, 0:2] = [[1, 1], [1, 0]]          # mean 0.75 -> 1
    h0 = mns.downsample(img)
    for j in range(6):
        for i in range(10):
            s = sum(int(img[2 * j + a, 2 * i + b]) for a in (0, 1) for b in (0, 1))
            want = int(Fraction(s, 4) + Fraction(1, 2))   # floor(mean + 1/2)
            assert h0[j, i] == want


def test_domain_is_cocentred_and_inside():
    for W in (16, 64, 96):
        for B in (4, 8):
            if W < 2 * B:
                continue
            for x in range(0, W, B):
                dx = int(mns.domain_origin(x, B, W))
                assert 0 <= dx <= W - 2 * B
                assert dx % 2 == 0
                if B // 2 <= x <= W - 3 * B // 2:
                    # same centre: x + B/2 == dx + B
                    assert x + B / 2 == dx + B
                assert dx <= x and x + B <= dx + 2 * B   # range inside its domain


# ---------------------------------------------------------------- moments
def test_moments_bruteforce():
    rng = np.random.default_rng(2)
    img = rng.integers(0, 256, (32, 48)).astype(np.uint8)
    I = img.astype(np.int64)
    h0 = mns.downsample(img)
    for B in (2, 4, 8, 16):        # B = 2: odd domain origins
        ys, xs = np.mgrid[0:32:B, 0:48:B]
        mom = mns.range_moments(I, h0, xs.ravel(), ys.ravel(), B)
        for idx, (x, y) in enumerate(zip(xs.ravel(), ys.ravel())):
            dx = min(max(x - B // 2, 0), 48 - 2 * B)
            dy = min(max(y - B // 2, 0), 32 - 2 * B)
            r = I[y:y + B, x:x + B]
            big = I[dy:dy + 2 * B, dx:dx + 2 * B]
            d = np.array([[int(Fraction(int(big[2 * a:2 * a + 2, 2 * b:2 * b + 2].sum()), 4)
                                + Fraction(1, 2)) for b in range(B)] for a in range(B)])
            assert mom["sr"][idx] == r.sum() and mom["srr"][idx] == (r * r).sum()
            assert mom["sd"][idx] == d.sum() and mom["sdd"][idx] == (d * d).sum()
            for e in range(8):
                assert mom["srd"][idx, e] == (r * geometric_isometry(d, e)).sum()


# ---------------------------------------------------------------- fit
def _brute_fit(r, d):
    """Minimum pixelwise collage error over e in 0..7, k in 0..7, m in 0..255.

    Exact: 64 n^2 E = sum_p u_p^2 with u_p = k (n d_p - sum d) + 8 n (m - r_p).
    Ties: lowest e, then lowest k, then the mean rounding half up (larger m).
    """
    n = r.size
    best = None
    sd = int(d.sum())
    ms = np.arange(256)
    for e in range(8):
        t = geometric_isometry(d, e).astype(np.int64).ravel()
        rr = r.astype(np.int64).ravel()
        for k in range(8):
            u = k * (n * t - sd)[None, :] + 8 * n * (ms[:, None] - rr[None, :])
            err = (u * u).sum(axis=1)            # 64 n^2 E for every m
            m = int(np.flatnonzero(err == err.min())[-1])
            key = (int(err[m]), e, k)
            if best is None or key < best[0]:
                best = (key, m)
    (err, e, k), m = best
    assert err % n == 0
    return e, k, m, err // n                     # S = 64 n E


@pytest.mark.parametrize("B", [2, 4, 8])
def test_fit_equals_bruteforce_grid(B):
    rng = np.random.default_rng(10 + B)
    cases = []
    for _ in range(12):
        cases.append((rng.integers(0, 256, (B, B)), rng.integers(0, 256, (B, B))))
    # degenerate and tie cases: flat domain, flat range, symmetric domain, ramp
    cases.append((rng.integers(0, 256, (B, B)), np.full((B, B), 77)))
    cases.append((np.full((B, B), 13), rng.integers(0, 256, (B, B))))
    sym = rng.integers(0, 256, (B, B))
    sym = sym + sym.T + np.fliplr(sym + sym.T)
    cases.append((rng.integers(0, 256, (B, B)), sym // 4))
    ii, jj = np.mgrid[0:B, 0:B]
    cases.append((2 * ii + 2 * jj + 3, 4 * ii + 4 * jj + 2))
    cases.append((np.full((B, B), 200) - 2 * ii, np.full((B, B), 100) + 4 * ii))
    for r, d in cases:
        r = np.asarray(r, np.int64)
        d = np.asarray(d, np.int64)
        mom = {"sr": np.array([r.sum()]), "srr": np.array([(r * r).sum()]),
               "sd": np.array([d.sum()]), "sdd": np.array([(d * d).sum()]),
               "srd": np.array([[(r * geometric_isometry(d, e)).sum() for e in range(8)]])}
        e, k, m, S = mns.fit_phase1(mom, B * B)
        assert (int(e[0]), int(k[0]), int(m[0]), int(S[0])) == _brute_fit(r, d)


def test_closed_form_k_is_grid_argmin():
    rng = np.random.default_rng(3)
    Q = np.concatenate([rng.integers(0, 10 ** 9, 4000), [0, 0, 1, 16, 16, 160]])
    # Q = 0 (flat domain) forces P = 0 by Cauchy-Schwarz
    P = np.concatenate([rng.integers(-10 ** 9, 10 ** 9, 4000), [0, 0, 0, 1, 15, 75]])
    # exact ties: 16 P = (2k+1) Q
    kt = rng.integers(0, 7, 500)
    Qt = 16 * rng.integers(1, 10 ** 6, 500)
    Q = np.concatenate([Q, Qt])
    P = np.concatenate([P, (2 * kt + 1) * Qt // 16])
    k = np.arange(8)
    f = (k * k)[None, :] * Q[:, None] - 16 * k[None, :] * P[:, None]
    np.testing.assert_array_equal(fullsearch.closed_form_k(P, Q), np.argmin(f, axis=1))


@pytest.mark.parametrize("e", range(8))
def test_exact_affine_image_of_each_isometry(e):
    """A range equal to (1/2)(T_e(d) - mean d) + m has zero error at (e, k=4)."""
    B = 8
    rng = np.random.default_rng(100 + e)
    v = rng.integers(0, 60, (B, B))
    v[0, 0] += (-v.sum()) % (B * B)            # integer mean
    d = 4 * v
    m = 120
    r = 2 * (geometric_isometry(v, e) - v.sum() // (B * B)) + m
    assert r.min() >= 0 and r.max() <= 255
    mom = {"sr": np.array([r.sum()]), "srr": np.array([(r * r).sum()]),
           "sd": np.array([d.sum()]), "sdd": np.array([(d * d).sum()]),
           "srd": np.array([[(r * geometric_isometry(d, f)).sum() for f in range(8)]])}
    ee, k, mm, S = mns.fit_phase1(mom, B * B)
    assert (int(ee[0]), int(k[0]), int(mm[0]), int(S[0])) == (e, 4, m, 0)


def test_ramp_has_zero_error_everywhere():
    img = synth.ramp(64, 64)
    I = img.astype(np.int64)
    h0 = mns.downsample(img)
    for B in (32, 16, 8, 4, 2):
        ys, xs = np.mgrid[0:64:B, 0:64:B]
        mom = mns.range_moments(I, h0, xs.ravel(), ys.ravel(), B)
        e, k, m, S = mns.fit_phase1(mom, B * B)
        assert np.all(S == 0) and np.all(e == 0) and np.all(k == 4)
    rec = mns.encode(img, 16, 4, [0, 0])
    # threshold 0 rejects everything except at the forced last level ...
    assert np.all(rec["level"] == 2)
    rec = mns.encode(img, 16, 4, [1, 1])
    # ... and any positive threshold accepts every top-level tile
    assert rec.size == 16 and np.all(rec["level"] == 0) and np.all(rec["s_idx"] == 4)
    # the ramp is an exact fixed point of the rounded decoder
    out = decode.decode(rec, 64, 64, 16, 3, start=img)
    np.testing.assert_array_equal(out, img)


def test_flat_image():
    img = synth.flat(64, 64, 77)
    rec = mns.encode(img, 16, 4, [1, 1])
    assert rec.size == 16
    assert np.all(rec["lum"] == 77) and np.all(rec["s_idx"] == 0) and np.all(rec["iso"] == 0)
    out = decode.decode(rec, 64, 64, 16, 1)
    assert np.all(out == 77)


# ---------------------------------------------------------------- quadtree
def _pixel_mse_phase1(I, rec, B):
    x, y, dx, dy = (int(rec[f]) for f in ("x", "y", "dx", "dy"))
    r = I[y:y + B, x:x + B]
    big = I[dy:dy + 2 * B, dx:dx + 2 * B]
    d = np.array([[int(Fraction(int(big[2 * a:2 * a + 2, 2 * b:2 * b + 2].sum()), 4) + Fraction(1, 2))
                   for b in range(B)] for a in range(B)])
    t = geometric_isometry(d, int(rec["iso"]))
    s = Fraction(int(rec["s_idx"]), 8)
    dbar = Fraction(int(d.sum()), B * B)
    err = sum((s * (int(t[i, j]) - dbar) + int(rec["lum"]) - int(r[i, j])) ** 2
              for i in range(B) for j in range(B))
    return err / (B * B)


def _preorder(rec, W, H, b_max):
    leaves = {(int(r["x"]), int(r["y"]), b_max >> int(r["level"])): i for i, r in enumerate(rec)}
    order = []

    def visit(x, y, B):
        if (x, y, B) in leaves:
            order.append(leaves[(x, y, B)])
            return
        assert B > 2, "missing leaf"
        b = B // 2
        for ox, oy in ((0, 0), (b, 0), (0, b), (b, b)):
            visit(x + ox, y + oy, b)

    for y in range(0, H, b_max):
        for x in range(0, W, b_max):
            visit(x, y, b_max)
    return order


@pytest.mark.parametrize("name,b_max,b_min,thr", [
    ("c1", 8, 4, [600]),
    ("c2", 16, 4, [300, 200]),
    ("c1", 8, 2, [600, 300]),
    ("c2", 16, 2, [300, 200, 100]),     # the paper's four levels, 16 x 16 to 2 x 2
])
def test_stream_structure_and_decisions(name, b_max, b_min, thr):
    img = synth.workload(name)
    H, W = img.shape
    I = img.astype(np.int64)
    trace = []
    rec = mns.encode(img, b_max, b_min, thr, trace=trace)
    # leaves tile the image exactly once (decode.pieces + cover check)
    decode.decode(rec, W, H, b_max, 1)
    # stream order is the depth-first pre-order of the quadtree, tiles in raster order
    assert _preorder(rec, W, H, b_max) == list(range(rec.size))
    L = len(thr) + 1
    rng = np.random.default_rng(0)
    p1 = rec[(rec["flags"] & 1) == 0]
    for r in p1[rng.choice(p1.size, min(60, p1.size), replace=False)]:
        lvl = int(r["level"]) + 1
        B = b_max >> (lvl - 1)
        assert int(r["s_idx"]) < 8 and int(r["iso"]) < 8
        if lvl < L:     # accepted before the forced last level: pixelwise MSE < t
            assert _pixel_mse_phase1(I, r, B) < thr[lvl - 1]
        # luminance is the range mean rounded half up
        rmean = Fraction(int(I[r["y"]:r["y"] + B, r["x"]:r["x"] + B].sum()), B * B)
        assert int(r["lum"]) == int(rmean + Fraction(1, 2))
    p2 = rec[(rec["flags"] & 1) == 1]
    assert p2.size > 0
    for r in p2:
        lvl = int(r["level"]) + 1
        B = b_max >> (lvl - 1)
        b = B // 2
        x, y, m = int(r["x"]), int(r["y"]), int(r["lum"])
        c1, c2 = mns.PHASE2_SETS[lvl]
        O = [m + int(v) for v in r["dlum"]]
        O.append(4 * m - sum(O))
        assert 0 <= O[3] <= 255
        for c in range(4):
            cx, cy = x + (c % 2) * b, y + (c // 2) * b
            child = I[cy:cy + b, cx:cx + b]
            if c < 3:
                assert O[c] == int(Fraction(int(child.sum()), b * b) + Fraction(1, 2))
            assert abs(O[c] - m) <= mns.PHASE2_DELTA[lvl]
            cdx = min(max(cx - b // 2, 0), W - 2 * b)
            cdy = min(max(cy - b // 2, 0), H - 2 * b)
            big = I[cdy:cdy + 2 * b, cdx:cdx + 2 * b]
            d = (big[0::2, 0::2] + big[0::2, 1::2] + big[1::2, 0::2] + big[1::2, 1::2] + 2) // 4
            s = Fraction([c1, c2][(int(r["s_idx"]) >> c) & 1], 20)
            dbar = Fraction(int(d.sum()), b * b)
            err = sum((s * (int(d[i, j]) - dbar) + O[c] - int(child[i, j])) ** 2
                      for i in range(b) for j in range(b))
            assert err / (b * b) < thr[lvl - 1]
    # every split range failed phase 1 (pixelwise check of the fit it took;
    # its phase-2 rejection is checked by definition in
    # test_phase2_decisions_by_definition)
    for info in trace[:-1]:
        B = info["B"]
        split = ~info["accept1"]
        split_idx = np.flatnonzero(split)
        if "accept2" in info:
            split_idx = split_idx[~info["accept2"]]
        for idx in split_idx[:20]:
            x, y = int(info["x"][idx]), int(info["y"][idx])
            probe = np.zeros(1, mns.RECORD_DTYPE)[0]
            probe["x"], probe["y"] = x, y
            probe["dx"] = mns.domain_origin(x, B, W)
            probe["dy"] = mns.domain_origin(y, B, H)
            probe["iso"], probe["s_idx"], probe["lum"] = info["e"][idx], info["k"][idx], info["m"][idx]
            assert _pixel_mse_phase1(I, probe, B) >= thr[info["level"] - 1]


def _phase2_by_definition(I, xs, ys, B, level, m, t, golden):
    """Technique 1 (Sec. 3.1-3.3) decided from the pixels and the paper's
    printed constants, for parents at (xs, ys) of side B whose phase-1 mean
    is m.  Returns (accept, admissible, O, err): O[:, c] the child means with
    O[:, 3] from eq. (1), err[:, c] = 400 nb^2 E_c of the better contrast of
    the level's set, E_c the child's pixelwise collage error.

    Child c (Z order) is fitted to its own co-centred domain, each 2 x 2
    group averaged and rounded half up.  With s = c'/20 and mean O,
    20 nb (r^_p - r_p) = c' (nb d_p - Sum d) + 20 nb (O - r_p), an integer,
    so 400 nb^2 E_c is the exact sum of its squares and
    MSE < t  <=>  400 nb^2 E_c < 400 nb^3 t.  The means round half up as
    floor(mean + 1/2), exact here because nb is a power of two."""
    H, W = I.shape
    b = B // 2
    nb = b * b
    cs = [Fraction(str(v)) * 20 for v in golden["phase2_contrast_sets"]["values"][str(level)]]
    assert all(c.denominator == 1 for c in cs)
    cs = [int(c) for c in cs]
    M = golden["phase2_mean_bits"]["values"][str(level)]
    bound = 2 ** (M - 1) - 1          # M bits, one of them the sign
    xs, ys, m = (np.asarray(v, np.int64) for v in (xs, ys, m))
    ii, jj = np.arange(b), np.arange(2 * b)
    O = np.zeros((xs.size, 4), np.int64)
    err = np.zeros((xs.size, 4), np.int64)
    for c, (ox, oy) in enumerate(((0, 0), (b, 0), (0, b), (b, b))):
        cx, cy = xs + ox, ys + oy
        r = I[cy[:, None, None] + ii[None, :, None], cx[:, None, None] + ii[None, None, :]]
        dx = np.clip(cx - b // 2, 0, W - 2 * b)
        dy = np.clip(cy - b // 2, 0, H - 2 * b)
        big = I[dy[:, None, None] + jj[None, :, None], dx[:, None, None] + jj[None, None, :]]
        d = (big[:, 0::2, 0::2] + big[:, 0::2, 1::2] + big[:, 1::2, 0::2] + big[:, 1::2, 1::2] + 2) // 4
        if c < 3:
            O[:, c] = np.floor(r.sum(axis=(1, 2)) / nb + 0.5).astype(np.int64)
        else:
            O[:, 3] = 4 * m - O[:, 0] - O[:, 1] - O[:, 2]          # eq. (1)
        sd = d.sum(axis=(1, 2))
        e = [((cc * (nb * d - sd[:, None, None]) + 20 * nb * (O[:, c][:, None, None] - r)) ** 2).sum(axis=(1, 2))
             for cc in cs]
        err[:, c] = np.minimum(e[0], e[1])
    adm = np.all(np.abs(O - m[:, None]) <= bound, axis=1) & (O[:, 3] >= 0) & (O[:, 3] <= 255)
    ok = adm & np.all(err < 400 * nb ** 3 * int(t), axis=1)
    return ok, adm, O, err


def _child_mse_fraction(I, x, y, B, c, O, s):
    """Pixelwise MSE of child c of the parent at (x, y) with contrast s and
    mean O, in rationals (the definition the scaled integers stand for)."""
    H, W = I.shape
    b = B // 2
    cx, cy = x + (c % 2) * b, y + (c // 2) * b
    child = I[cy:cy + b, cx:cx + b]
    dx, dy = min(max(cx - b // 2, 0), W - 2 * b), min(max(cy - b // 2, 0), H - 2 * b)
    big = I[dy:dy + 2 * b, dx:dx + 2 * b]
    d = [[Fraction(int(big[2 * i:2 * i + 2, 2 * j:2 * j + 2].sum()), 4) for j in range(b)] for i in range(b)]
    d = [[int(v + Fraction(1, 2)) for v in row] for row in d]
    dbar = Fraction(sum(map(sum, d)), b * b)
    return sum((s * (d[i][j] - dbar) + O - int(child[i, j])) ** 2 for i in range(b) for j in range(b)) / (b * b)


PHASE2_STREAMS = [
    ("c1", 8, 4, [600]),
    ("c2", 16, 4, [300, 200]),
    ("c2", 16, 4, [40, 20]),
    ("c2", 16, 2, [300, 200, 100]),     # the paper's four levels, 16 x 16 to 2 x 2
]


@pytest.mark.parametrize("name,b_max,b_min,thr", PHASE2_STREAMS)
def test_phase2_decisions_by_definition(golden, name, b_max, b_min, thr):
    """Every range that fails phase 1 above the last level is stored by
    Technique 1 exactly when the definition says so: all four child means
    (O_4 by eq. (1), inside 0..255) within the stored M-bit signed width of
    the parent mean, and every child's MSE under the better contrast of the
    level's set below t_l (Sec. 3.1-3.3).  Rejections are checked as well as
    acceptances, and the boundary cases the streams reach (a difference at
    the bound, a worst child MSE within one grey level squared of t_l) are
    required to occur, so a stricter rule cannot pass."""
    img = synth.workload(name)
    I = img.astype(np.int64)
    trace = []
    rec = mns.encode(img, b_max, b_min, thr, trace=trace)
    reach = {"delta at bound": False, "worst MSE in [t-1, t)": False, "rejected on MSE alone": False}
    for info in trace[:-1]:
        lvl, B = info["level"], info["B"]
        t = thr[lvl - 1]
        fail = ~info["accept1"]
        xs, ys, m = info["x"][fail], info["y"][fail], info["m"][fail]
        ok, adm, O, err = _phase2_by_definition(I, xs, ys, B, lvl, m, t, golden)
        np.testing.assert_array_equal(info["accept2"], ok, err_msg=f"level {lvl}")
        nb = (B // 2) ** 2
        np.testing.assert_array_equal(info["O"], O)
        # the oracle's scaled errors are the chosen contrast's: the better one
        np.testing.assert_array_equal(info["S2"] * nb, err)
        bound = 2 ** (golden["phase2_mean_bits"]["values"][str(lvl)] - 1) - 1
        worst = err.max(axis=1)
        near = adm & (worst >= 400 * nb ** 3 * (t - 1)) & (worst < 400 * nb ** 3 * t)
        reach["delta at bound"] |= bool(np.any(ok & np.any(np.abs(O - m[:, None]) == bound, axis=1)))
        reach["worst MSE in [t-1, t)"] |= bool(near.any())
        reach["rejected on MSE alone"] |= bool(np.any(adm & ~ok))
        # the scaled integers against rational arithmetic, on the ranges
        # nearest the threshold on either side
        sets = [Fraction(str(v)) for v in golden["phase2_contrast_sets"]["values"][str(lvl)]]
        for idx in np.argsort(np.abs(worst - 400 * nb ** 3 * t))[:3]:
            c = int(np.argmax(err[idx]))
            mse = min(_child_mse_fraction(I, int(xs[idx]), int(ys[idx]), B, c, int(O[idx, c]), s) for s in sets)
            assert mse == Fraction(int(err[idx, c]), 400 * nb ** 3)
    if (name, b_min, thr[0]) in (("c2", 4, 300), ("c2", 2, 300)):
        assert all(reach.values()), reach
    assert np.count_nonzero(rec["flags"] & 1) == sum(int(i["accept2"].sum()) for i in trace[:-1])


def _flat_blocks(vals, q):
    """An image of flat q x q blocks with the given grey values (rows of blocks)."""
    return np.kron(np.asarray(vals, np.int64), np.ones((q, q), np.int64)).astype(np.uint8)


def test_phase2_mean_difference_at_the_stored_width(golden):
    """A parent whose flat children sit at +-2^(M-1)-1 grey levels from its
    mean is stored by Technique 1; one level further it is split (Sec. 3.1:
    the means must be close; Sec. 3.3: M-bit signed differences, O_4 from
    eq. (1)).  8 -> 4 on a 16 x 16 image of flat 4 x 4 blocks: every parent
    8 x 8 is a checkerboard of its children, m + D, m - D, m - D, m + D, so
    phase 1 (one contrast for the whole parent) fails a small threshold."""
    bound = 2 ** (golden["phase2_mean_bits"]["values"]["1"] - 1) - 1
    m = 120
    for D, stored in ((bound, True), (bound + 1, False)):
        v = [[m + D, m - D], [m - D, m + D]]
        img = _flat_blocks(np.tile(v, (2, 2)), 4)
        I = img.astype(np.int64)
        trace = []
        rec = mns.encode(img, 8, 4, [20], trace=trace)
        info = trace[0]
        assert not info["accept1"].any()          # phase 1 fails every parent
        ok, adm, O, err = _phase2_by_definition(I, info["x"], info["y"], 8, 1, info["m"], 20, golden)
        assert np.all(np.abs(O - m) == D) and np.all(info["m"] == m)
        assert ok.all() == stored and adm.all() == stored
        np.testing.assert_array_equal(info["accept2"], ok)
        p2 = rec[(rec["flags"] & 1) == 1]
        assert p2.size == (4 if stored else 0)
        if stored:
            assert np.all(np.abs(p2["dlum"].astype(np.int64)) == D)


def test_phase2_threshold_is_strict_at_the_worst_child(golden):
    """Technique 1 stores a parent when every child's MSE is below t_l and
    splits it when the worst child's MSE reaches t_l (Sec. 3.1), with the
    threshold placed from the definition at the worst child's error: just
    above it the parent is stored, at its floor it is split."""
    img = synth.workload("c2")
    I = img.astype(np.int64)
    trace = []
    mns.encode(img, 16, 4, [300, 200], trace=trace)
    info = trace[1]                                  # level 2, 8 x 8 parents, 4 x 4 children
    fail = ~info["accept1"]
    xs, ys, m = info["x"][fail], info["y"][fail], info["m"][fail]
    ok, adm, O, err = _phase2_by_definition(I, xs, ys, 8, 2, m, 200, golden)
    nb = 16
    worst = err.max(axis=1)
    # admissible parents whose worst child MSE is not an integer
    cand = np.flatnonzero(adm & (worst % (400 * nb ** 3) != 0) & (worst < 400 * nb ** 3 * 250))
    assert cand.size > 0
    for idx in cand[:5]:
        mse = Fraction(int(worst[idx]), 400 * nb ** 3)
        x, y = int(xs[idx]), int(ys[idx])
        for t, stored in ((int(mse) + 1, True), (int(mse), False)):
            a, _, _, _ = mns.fit_phase2(I, mns.downsample(img), [x], [y], 8, 2, [int(m[idx])], t)
            assert bool(a[0]) == stored, (x, y, t, mse)


def test_no_search_variant_has_no_phase2_records():
    img = synth.workload("c1")
    rec = mns.encode(img, 8, 4, [600], phase2=False)
    assert np.all(rec["flags"] == 0)
    mns_rec = mns.encode(img, 8, 4, [600])
    # Technique 1 only ever replaces four next-level leaves by one record
    assert mns_rec.size <= rec.size


def test_validation():
    img = np.zeros((64, 64), np.uint8)
    with pytest.raises(ValueError):
        mns.encode(img, 8, 4, [])           # one threshold per non-final level
    with pytest.raises(ValueError):
        mns.encode(img, 64, 4, [1, 1, 1, 1])
    with pytest.raises(ValueError):
        mns.encode(img, 32, 2, [1, 1, 1, 1])   # five levels: more than two level bits hold
    with pytest.raises(ValueError):
        mns.encode(img, 8, 1, [1, 1, 1])
    with pytest.raises(ValueError):
        mns.encode(img, 2, 2, [])
    assert mns.encode(img, 16, 2, [1, 1, 1]).size > 0
    with pytest.raises(ValueError):
        mns.encode(np.zeros((60, 64), np.uint8), 8, 4, [1])
    with pytest.raises(ValueError):
        mns.encode(np.zeros((16, 64), np.uint8), 16, 4, [1, 1])
    assert mns.max_transforms(64, 64, 4) == 256


# ---------------------------------------------------------------- decoder
@pytest.fixture(scope="module")
def c1_stream():
    img = synth.workload("c1")
    return img, mns.encode(img, 8, 4, [600])


def test_decoder_int_equals_float(c1_stream):
    img, rec = c1_stream
    for start in (None, np.zeros((64, 64), np.uint8), img):
        a = decode.decode(rec, 64, 64, 8, 6, start=start, mode="int")
        b = decode.decode(rec, 64, 64, 8, 6, start=start, mode="float")
        np.testing.assert_array_equal(a, b)


def test_decoder_converges_to_linear_fixed_point(c1_stream):
    img, rec = c1_stream
    rng = np.random.default_rng(5)
    starts = [np.zeros((64, 64)), np.full((64, 64), 128.0), np.full((64, 64), 255.0),
              rng.integers(0, 256, (64, 64)).astype(np.float64)]
    outs = [decode.decode(rec, 64, 64, 8, 80, start=s, mode="unrounded") for s in starts]
    for o in outs[1:]:
        assert np.max(np.abs(o - outs[0])) < 1e-9
    xstar = decode.fixed_point(rec, 64, 64, 8)
    assert np.max(np.abs(outs[0] - xstar)) < 1e-6


def test_rounded_decoder_agrees_across_starts(c1_stream):
    img, rec = c1_stream
    rng = np.random.default_rng(6)
    starts = [None, np.zeros((64, 64), np.uint8), np.full((64, 64), 255, np.uint8),
              rng.integers(0, 256, (64, 64)).astype(np.uint8)]
    outs = [decode.decode(rec, 64, 64, 8, 40, start=s).astype(np.int64) for s in starts]
    for o in outs[1:]:
        assert np.max(np.abs(o - outs[0])) <= 1
    assert metrics.psnr(img, outs[0]) > 15.0


# ---------------------------------------------------------------- full search
def test_fullsearch_bruteforce_tiny():
    rng = np.random.default_rng(8)
    img = rng.integers(0, 256, (16, 16)).astype(np.uint8)
    I = img.astype(np.int64)
    B = 4
    n = B * B
    ys, xs = np.mgrid[0:16:B, 0:16:B]
    bm = fullsearch.best_matches(img, xs.ravel(), ys.ravel(), B)
    for idx, (x, y) in enumerate(zip(xs.ravel(), ys.ravel())):
        r = I[y:y + B, x:x + B]
        sr = int(r.sum())
        m = (2 * sr + n) // (2 * n)
        best = None
        for v in range(16 - 2 * B + 1):
            for u in range(16 - 2 * B + 1):
                big = I[v:v + 2 * B, u:u + 2 * B]
                d = (big[0::2, 0::2] + big[0::2, 1::2] + big[1::2, 0::2] + big[1::2, 1::2] + 2) // 4
                sd = int(d.sum())
                for e in range(8):
                    t = geometric_isometry(d, e)
                    for k in range(8):
                        u_p = k * (n * t - sd) + 8 * n * (m - r)
                        S = int((u_p * u_p).sum()) // n
                        key = (S, v * (16 - 2 * B + 1) + u, e, k)
                        if best is None or key < best:
                            best = key
        S, dom, e, k = best
        assert (int(bm["S"][idx]), int(bm["dom"][idx]), int(bm["e"][idx]), int(bm["k"][idx])) == (S, dom, e, k)


def test_fullsearch_never_worse_than_mns():
    img = synth.workload("c1")
    I = img.astype(np.int64)
    h0 = mns.downsample(img)
    for B in (8, 4):
        ys, xs = np.mgrid[0:64:B, 0:64:B]
        xs, ys = xs.ravel()[:40], ys.ravel()[:40]
        mom = mns.range_moments(I, h0, xs, ys, B)
        _, _, _, S_mns = mns.fit_phase1(mom, B * B)
        bm = fullsearch.best_matches(img, xs, ys, B)
        assert np.all(bm["S"] <= S_mns)
        # and the MNS domain's error is what full search finds at that origin
        assert np.any(bm["S"] < S_mns)


def test_fullsearch_stream_tiles_image():
    img = synth.workload("c1")[:32, :32].copy()
    rec = fullsearch.encode(img, 8, 4, [300])
    decode.decode(rec, 32, 32, 8, 2)
    assert _preorder(rec, 32, 32, 8) == list(range(rec.size))


def _decode_step_by_definition(rec, start, b_max):
    """One Jacobi step written out pixel by pixel in exact rationals."""
    H, W = start.shape
    X = start.astype(np.int64)
    out = np.full((H, W), -1, np.int64)

    def domain(x0, y0, B):
        dx = min(max(x0 - B // 2, 0), W - 2 * B)
        dy = min(max(y0 - B // 2, 0), H - 2 * B)
        big = X[dy:dy + 2 * B, dx:dx + 2 * B]
        return np.array([[int(Fraction(int(big[2 * a:2 * a + 2, 2 * b:2 * b + 2].sum()), 4) + Fraction(1, 2))
                          for b in range(B)] for a in range(B)])

    def paint(x0, y0, t, dsum, s, lum):
        B = t.shape[0]
        dbar = Fraction(int(dsum), B * B)
        for i in range(B):
            for j in range(B):
                v = s * (int(t[i, j]) - dbar) + lum
                out[y0 + i, x0 + j] = min(max(int(v + Fraction(1, 2)), 0), 255)

    for r in rec:
        B = b_max >> int(r["level"])
        x, y = int(r["x"]), int(r["y"])
        if int(r["flags"]) & 1 == 0:
            d = domain(x, y, B)
            paint(x, y, geometric_isometry(d, int(r["iso"])), d.sum(), Fraction(int(r["s_idx"]), 8), int(r["lum"]))
        else:
            b = B // 2
            m = int(r["lum"])
            O = [m + int(v) for v in r["dlum"]]
            O.append(4 * m - sum(O))                       # eq. (1)
            c1, c2 = mns.PHASE2_SETS[int(r["level"]) + 1]
            for c in range(4):
                cx, cy = x + (c % 2) * b, y + (c // 2) * b
                d = domain(cx, cy, b)
                s = Fraction([c1, c2][(int(r["s_idx"]) >> c) & 1], 20)
                paint(cx, cy, d, d.sum(), s, O[c])
    assert np.all(out >= 0), "records do not cover the image"
    return out


def test_decoder_one_step_by_definition(c1_stream):
    img, rec = c1_stream
    assert np.any(rec["flags"] & 1) and np.any(rec["iso"] >= 4)
    rng = np.random.default_rng(11)
    start = rng.integers(0, 256, (64, 64)).astype(np.uint8)
    want = _decode_step_by_definition(rec, start, 8)
    np.testing.assert_array_equal(decode.decode(rec, 64, 64, 8, 1, start=start).astype(np.int64), want)


def test_decoder_one_step_by_definition_2x2():
    # a tree down to 2 x 2 (odd domain origins, phase 2 over 2 x 2 sub-blocks)
    img = synth.workload("c1")
    rec = mns.encode(img, 8, 2, [600, 300])
    assert np.any(rec["level"] == 2) and np.any((rec["flags"] & 1) & (rec["level"] == 1))
    assert np.any(rec["dx"] % 2)
    rng = np.random.default_rng(12)
    start = rng.integers(0, 256, (64, 64)).astype(np.uint8)
    want = _decode_step_by_definition(rec, start, 8)
    np.testing.assert_array_equal(decode.decode(rec, 64, 64, 8, 1, start=start).astype(np.int64), want)
