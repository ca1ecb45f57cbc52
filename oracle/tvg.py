"""FP64 oracle: time-varying gain of an echo cube (Eq. 10, Sec. II-E).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Definition: for each sample time t, the population median power over every
(ping, element) of the batch, P~(t) = median |E[p, e, t]|^2, and its average
over the sample times, mean P~. The gain is

    G(t) = (alpha mean P~ + P~(t))^-1.

Readings where the paper is silent: the median of N values is the element of
rank floor((N - 1) / 2) in ascending order; G is a power gain, applied to the
complex echo as the amplitude factor sqrt(G(t)); a sample time whose gain is
not finite (alpha = 0 and a zero median) keeps its samples unchanged.
"""
from __future__ import annotations

import numpy as np


def tvg(echo, alpha: float):
    """Returns (conditioned echo complex128 [P, E, N_s], median power P~ [N_s], gain G [N_s])."""
    e = np.asarray(echo, dtype=np.complex128)
    P, E, Ns = e.shape
    power = (np.abs(e) ** 2).reshape(P * E, Ns)
    k = (P * E - 1) // 2
    med = np.partition(power, k, axis=0)[k]
    with np.errstate(divide="ignore"):
        G = 1.0 / (alpha * med.mean() + med)
    amp = np.where(np.isfinite(G), np.sqrt(np.where(np.isfinite(G), G, 1.0)), 1.0)
    return e * amp[None, None, :], med, G
