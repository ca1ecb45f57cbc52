"""FP64 oracle: dynamic range compression of a complex image for display.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Definition (Eqs. 11-12, Sec. II-E). I is the input image normalised to
[0, 1]; here the magnitude of the complex image divided by its maximum. The
output of each pixel is

    I_DRC = q I / ((q - 1) I + 1),

a bijection of [0, 1] onto itself, and q is chosen so that the median input
pixel maps to the requested output brightness b in (0, 1):

    q = (b - b I~) / (I~ - b I~),   I~ the median of I.

Readings where the paper is silent: the median of N pixels is the element of
rank floor((N - 1) / 2) in ascending order (the lower median for even N). An
all-zero image maps to zeros (q = 1). If I~ = 0 the limit q -> infinity maps
every non-zero pixel to 1; if I~ = 1 the limit q -> 0 maps every pixel below
the maximum to 0.
"""
from __future__ import annotations

import math

import numpy as np


def drc(image, brightness: float):
    """Returns (out float64 array shaped like image, params dict with max, median, q)."""
    if not (0.0 < brightness < 1.0):
        raise ValueError("brightness must lie in (0, 1)")
    mag = np.abs(np.asarray(image, dtype=np.complex128)).ravel()
    peak = float(mag.max()) if mag.size else 0.0
    if peak == 0.0:
        return np.zeros(np.shape(image)), {"max": 0.0, "median": 0.0, "q": 1.0}
    x = mag / peak
    k = (x.size - 1) // 2
    med = float(np.partition(x, k)[k])
    b = float(brightness)
    if med == 0.0:
        q = math.inf
        out = (x > 0.0).astype(np.float64)
    elif med == 1.0:
        q = 0.0
        out = (x >= 1.0).astype(np.float64)
    else:
        q = (b - b * med) / (med - b * med)
        out = q * x / ((q - 1.0) * x + 1.0)
    return out.reshape(np.shape(image)), {"max": peak, "median": med, "q": q}
