"""Planted mistakes in the oracle, each of which some pin must catch.

Every case swaps one oracle function (or constant) for a plausible wrong
version -- a dropped term, a wrong sign, a transposed or mislabelled
operand, an off-by-one rounding -- runs the pins of test_oracle_pins, and
requires at least one of them to fail.  This is what makes the pins evidence
that the oracle follows the paper and not only itself.  CPU only.
"""
import json

import numpy as np
import pytest

import test_oracle_pins as pins
from oracle import decode, fullsearch, mns
from paper_1501_02894_amd import synth


def _golden():
    with open(pins.GOLDEN) as f:
        return json.load(f)


def _c1_stream():
    img = synth.workload("c1")
    return img, mns.encode(img, 8, 4, [600])


def _phase2_pins():
    g = _golden()
    pins.test_phase2_mean_difference_at_the_stored_width(g)
    pins.test_phase2_threshold_is_strict_at_the_worst_child(g)
    # a stream rich in phase 2: C2, 16 -> 4, every failed range decided by definition
    pins.test_phase2_decisions_by_definition(g, "c2", 16, 4, [300, 200])


# the pins, cheapest first; each is a zero-argument callable
PINS = [
    ("paper constants", lambda: pins.test_paper_constants(_golden())),
    ("isometry group", lambda: pins.test_isometry_table_is_the_square_group(8)),
    ("downsample", pins.test_downsample_round_half_up),
    ("co-centred domain", pins.test_domain_is_cocentred_and_inside),
    ("closed-form k", pins.test_closed_form_k_is_grid_argmin),
    ("fit vs brute force B=4", lambda: pins.test_fit_equals_bruteforce_grid(4)),
    ("affine images", lambda: [pins.test_exact_affine_image_of_each_isometry(e) for e in range(8)]),
    ("moments", pins.test_moments_bruteforce),
    ("ramp", pins.test_ramp_has_zero_error_everywhere),
    ("flat", pins.test_flat_image),
    ("decode step", lambda: pins.test_decoder_one_step_by_definition(_c1_stream())),
    ("stream c1", lambda: pins.test_stream_structure_and_decisions("c1", 8, 4, [600])),
    ("phase 2 by definition", _phase2_pins),
    ("full search tiny", pins.test_fullsearch_bruteforce_tiny),
]


def _caught():
    """Name of the first pin that fails, or None."""
    for name, fn in PINS:
        try:
            fn()
        except Exception:      # an assertion, or a crash the mistake causes
            return name
    return None


# ------------------------------------------------------------------ mutants
def _downsample_floor(img):
    I = np.asarray(img).astype(np.int64)
    return (I[0::2, 0::2] + I[0::2, 1::2] + I[1::2, 0::2] + I[1::2, 1::2]) // 4


def _domain_wrong_centre(p, B, extent):
    return np.clip(np.asarray(p, np.int64) - B, 0, extent - 2 * B)


def _domain_clamped_to_w_minus_b(p, B, extent):
    return np.clip(np.asarray(p, np.int64) - B // 2, 0, extent - B)


_orig_iso = mns.isometry_source


def _iso_swapped_rotations(e, B):
    return _orig_iso({5: 6, 6: 5}.get(e, e), B)


def _iso_transpose_is_identity(e, B):
    return _orig_iso(e - 4 if e >= 4 else e, B)


_orig_moments = mns.range_moments


def _moments_no_transposes(I, h0, xs, ys, B):
    out = _orig_moments(I, h0, xs, ys, B)
    out["srd"][:, 4:] = out["srd"][:, :4]
    return out


def _moments_sdd_plain(I, h0, xs, ys, B):
    out = _orig_moments(I, h0, xs, ys, B)
    out["sdd"] = out["sd"] * out["sd"] // (B * B)
    return out


def _fit_factory(drop_lum=False, flip_p=False, k_scale=16):
    def fit(mom, n):
        sr, srr, sd, sdd, srd = (mom[k] for k in ("sr", "srr", "sd", "sdd", "srd"))
        Q = n * sdd - sd * sd
        Rr = n * srr - sr * sr
        P = n * srd + (sr * sd)[:, None] if flip_p else n * srd - (sr * sd)[:, None]
        k = np.arange(8, dtype=np.int64)
        f = (k * k)[None, None, :] * Q[:, None, None] - k_scale * k[None, None, :] * P[:, :, None]
        flat = f.reshape(len(sr), 64)
        best = np.argmin(flat, axis=1)
        fmin = flat[np.arange(len(sr)), best]
        m = mns.quantised_mean(sr, n)
        S = fmin + 64 * Rr + (0 if drop_lum else 64 * (n * m - sr) ** 2)
        return best // 8, best % 8, m, S
    return fit


def _mean_floor(sr, n):
    return np.asarray(sr, np.int64) // n


def _children_n_order(xs, ys, B):
    b = B // 2
    ox = np.array([0, 0, b, b], np.int64)
    oy = np.array([0, b, 0, b], np.int64)
    return np.asarray(xs, np.int64)[:, None] + ox[None, :], np.asarray(ys, np.int64)[:, None] + oy[None, :]


def _key_swapped(x, y, width, b_max, b_min):
    x = np.asarray(x, np.int64)
    y = np.asarray(y, np.int64)
    L = mns.num_levels(b_max, b_min)
    tile = (y // b_max) * (width // b_max) + (x // b_max)
    lx = (x % b_max) // b_min
    ly = (y % b_max) // b_min
    code = np.zeros_like(x)
    for bit in range(L - 1):
        code |= ((ly >> bit) & 1) << (2 * bit)
        code |= ((lx >> bit) & 1) << (2 * bit + 1)
    return tile * (4 ** (L - 1)) + code


_orig_domain_blocks = decode._domain_blocks


def _decode_floor(x, dx, dy, B, rounded):
    v = _orig_domain_blocks(x, dx, dy, B, False)
    return np.floor(v).astype(np.int64) if rounded else v


def _closed_k_floor(P, Q):
    P = np.asarray(P, np.int64)
    Q = np.asarray(Q, np.int64)
    safeQ = np.where(Q > 0, Q, 1)
    k = np.clip((16 * P - Q) // (2 * safeQ), 0, 7)
    return np.where(Q > 0, k, 0)


def _all_domains_floor(img, B):
    I = np.asarray(img).astype(np.int64)
    H, W = I.shape
    M = (I[:-1, :-1] + I[:-1, 1:] + I[1:, :-1] + I[1:, 1:]) // 4
    win = np.lib.stride_tricks.sliding_window_view(M, (2 * B - 1, 2 * B - 1))
    win = win[: H - 2 * B + 1, : W - 2 * B + 1, ::2, ::2]
    return np.ascontiguousarray(win).reshape(-1, B * B)


def _fit2_factory(thr_minus=0, thr_scale=1, strict_delta=False):
    """Technique 1 with one plausible slip in its rejection rule."""
    def fit2(I, h0, xs, ys, B, level, m, t):
        b = B // 2
        nb = b * b
        c1, c2 = mns.PHASE2_SETS[level]
        delta = mns.PHASE2_DELTA[level]
        m = np.asarray(m, np.int64)
        cx, cy = mns.children_xy(xs, ys, B)
        mom = [mns.range_moments(I, h0, cx[:, c], cy[:, c], b) for c in range(4)]
        O = np.zeros((m.size, 4), np.int64)
        for c in range(3):
            O[:, c] = mns.quantised_mean(mom[c]["sr"], nb)
        O[:, 3] = 4 * m - O[:, 0] - O[:, 1] - O[:, 2]
        dev = np.abs(O - m[:, None])
        accept = np.all(dev < delta if strict_delta else dev <= delta, axis=1)
        accept &= (O[:, 3] >= 0) & (O[:, 3] <= 255)
        bits = np.zeros(m.size, np.int64)
        S = np.zeros((m.size, 4), np.int64)
        tt = (int(t) - thr_minus) * thr_scale
        for c in range(4):
            mc = mom[c]
            Q = nb * mc["sdd"] - mc["sd"] * mc["sd"]
            Rr = nb * mc["srr"] - mc["sr"] * mc["sr"]
            P = nb * mc["srd"][:, 0] - mc["sr"] * mc["sd"]
            f1 = c1 * c1 * Q - 40 * c1 * P
            f2 = c2 * c2 * Q - 40 * c2 * P
            use2 = f2 < f1
            S[:, c] = np.where(use2, f2, f1) + 400 * Rr + 400 * (nb * O[:, c] - mc["sr"]) ** 2
            bits |= use2.astype(np.int64) << c
            accept &= S[:, c] < 400 * nb * nb * tt
        return accept, O, bits, S
    return fit2


MUTANTS = {
    "downsample rounds down": (mns, "downsample", _downsample_floor),
    "domain centred at x - B": (mns, "domain_origin", _domain_wrong_centre),
    "domain clamped to W - B": (mns, "domain_origin", _domain_clamped_to_w_minus_b),
    "rotations 90 cw / ccw swapped": (mns, "isometry_source", _iso_swapped_rotations),
    "transposing isometries dropped": (mns, "isometry_source", _iso_transpose_is_identity),
    "moments: transposes not applied": (mns, "range_moments", _moments_no_transposes),
    "moments: sum d^2 from the mean": (mns, "range_moments", _moments_sdd_plain),
    "fit: luminance term dropped": (mns, "fit_phase1", _fit_factory(drop_lum=True)),
    "fit: wrong sign of the cross term": (mns, "fit_phase1", _fit_factory(flip_p=True)),
    "fit: contrast scale 1/4 instead of 1/8": (mns, "fit_phase1", _fit_factory(k_scale=8)),
    "mean rounds down": (mns, "quantised_mean", _mean_floor),
    "children in N order": (mns, "children_xy", _children_n_order),
    "Morton x bit above y": (mns, "stream_key", _key_swapped),
    "phase-2 set typo": (mns, "PHASE2_SETS", {1: (4, 10), 2: (8, 14), 3: (10, 18)}),
    "phase-2 bound off by one": (mns, "PHASE2_DELTA", {1: 16, 2: 32, 3: 32}),
    "phase-2 threshold t - 1": (mns, "fit_phase2", _fit2_factory(thr_minus=1)),
    "phase-2 threshold 0.9 t": (mns, "fit_phase2", _fit2_factory(thr_scale=0.9)),
    "phase-2 strict bound on the mean difference": (mns, "fit_phase2", _fit2_factory(strict_delta=True)),
    "decoder 2x2 mean rounds down": (decode, "_domain_blocks", _decode_floor),
    "full search: k rounds down": (fullsearch, "closed_form_k", _closed_k_floor),
    "full search: domains round down": (fullsearch, "all_domains", _all_domains_floor),
}


def test_unmutated_oracle_passes_every_pin():
    assert _caught() is None


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(monkeypatch, name):
    module, attr, value = MUTANTS[name]
    monkeypatch.setattr(module, attr, value)
    assert _caught() is not None, f"no pin catches: {name}"
