"""Error metrics between an image and its FP64 oracle (test infrastructure only).

rel-L2 = |I - I_ref|_2 / |I_ref|_2 over the compared pixels. The phase error is
|arg(I * conj(I_ref))|, maximised over pixels whose reference magnitude lies
within ``floor_db`` of the reference peak: phase is undefined at nulls.
"""
from __future__ import annotations

import numpy as np


def rel_l2(img, ref) -> float:
    a = np.asarray(img, dtype=np.complex128).ravel()
    b = np.asarray(ref, dtype=np.complex128).ravel()
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / den) if den > 0 else float(np.linalg.norm(a))


def phase_error_mrad(img, ref, floor_db: float = 30.0, stat: str = "max") -> float:
    a = np.asarray(img, dtype=np.complex128).ravel()
    b = np.asarray(ref, dtype=np.complex128).ravel()
    mag = np.abs(b)
    if mag.size == 0 or mag.max() == 0:
        return 0.0
    sel = mag >= mag.max() * 10.0 ** (-floor_db / 20.0)
    ph = np.abs(np.angle(a[sel] * np.conj(b[sel]))) * 1e3
    if stat == "p99":
        return float(np.percentile(ph, 99))
    return float(ph.max())
