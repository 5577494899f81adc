"""Oracle: distortion measures of Sec. 4.

TEST INFRASTRUCTURE ONLY (see the package docstring).

MSE is the mean over all pixels of (x - x^)^2; PSNR = 10 log10(K^2 / MSE)
with K = 255 for 8-bit images, in dB (infinite when MSE = 0).
"""
from __future__ import annotations

import numpy as np

PEAK = 255.0


def mse(a: np.ndarray, b: np.ndarray) -> float:
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.mean((a - b) ** 2))


def psnr(a: np.ndarray, b: np.ndarray) -> float:
    e = mse(a, b)
    if e == 0.0:
        return float("inf")
    return 10.0 * np.log10(PEAK * PEAK / e)
