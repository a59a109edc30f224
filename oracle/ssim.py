"""Structural similarity (SSIM) -- TEST AND MEASUREMENT INFRASTRUCTURE ONLY.

The paper scores block-wise foveation against per-pixel ("perfect")
foveation with SSIM maps (Sec. 3, Fig. 3).  SSIM is the index of Wang, Bovik,
Sheikh and Simoncelli (2004): with local means mu, variances s^2 and covariance
s_xy taken under an 11-tap Gaussian window of sigma 1.5,

    SSIM = (2 mu_x mu_y + C1)(2 s_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(s_x^2 + s_y^2 + C2)),

C1 = (0.01 L)^2, C2 = (0.03 L)^2, L the dynamic range.  The window is applied
separably with scipy's Gaussian filter (radius 5, edges reflected).
"""
from __future__ import annotations

import numpy as np
from scipy import ndimage

K1, K2 = 0.01, 0.03
WIN_SIGMA = 1.5
WIN_RADIUS = 5


def _blur(a: np.ndarray) -> np.ndarray:
    return ndimage.gaussian_filter(a, WIN_SIGMA, mode="reflect", truncate=WIN_RADIUS / WIN_SIGMA)


def ssim_map(x: np.ndarray, y: np.ndarray, data_range: float = 255.0) -> np.ndarray:
    """Per-pixel SSIM of two 2-D images of the same shape."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    c1, c2 = (K1 * data_range) ** 2, (K2 * data_range) ** 2
    mx, my = _blur(x), _blur(y)
    sxx = _blur(x * x) - mx * mx
    syy = _blur(y * y) - my * my
    sxy = _blur(x * y) - mx * my
    return ((2 * mx * my + c1) * (2 * sxy + c2)) / ((mx * mx + my * my + c1) * (sxx + syy + c2))
