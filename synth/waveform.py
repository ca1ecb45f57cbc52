"""Seeded test signals for range compression: a linear-FM replica and raw
(uncompressed, analytic passband) echoes of point scatterers built from it.

Input generation only; shared by the tests and the benchmark.
"""
from __future__ import annotations

import numpy as np


def lfm_replica(bandwidth: float, duration: float, fs: float) -> np.ndarray:
    """Complex baseband linear-FM pulse q(t) = exp(j pi K (t - T/2)^2),
    K = B / T, sampled at t = m / f_s for m < round(T f_s): the sweep runs
    from -B/2 to +B/2."""
    M = int(round(duration * fs))
    T = M / fs
    K = bandwidth / T
    t = np.arange(M, dtype=np.float64) / fs
    return np.exp(1j * np.pi * K * (t - T / 2) ** 2)


def raw_echo(n_rows: int, n_sample: int, replica: np.ndarray, f_c: float, fs: float, t0: float,
             n_targets: int, seed: int, noise: float = 0.0) -> tuple:
    """Analytic passband rows x[k] = sum_s a_s q(t_k - tau_s) exp(j 2 pi f_c (t_k - tau_s)) (+ noise),
    with the replica delayed by whole samples (tau_s on the sample grid) so the
    rows are exact. Returns (echo complex128 [n_rows, n_sample], delays in
    samples [n_rows, n_targets], amplitudes [n_rows, n_targets])."""
    rng = np.random.default_rng(seed)
    M = replica.shape[0]
    x = np.zeros((n_rows, n_sample), dtype=np.complex128)
    d = rng.integers(0, max(1, n_sample - M // 2), size=(n_rows, n_targets))
    a = (rng.normal(size=(n_rows, n_targets)) + 1j * rng.normal(size=(n_rows, n_targets))) / np.sqrt(2)
    t = t0 + np.arange(n_sample) / fs
    for r in range(n_rows):
        for s in range(n_targets):
            k0 = int(d[r, s])
            k1 = min(n_sample, k0 + M)
            tau = t0 + k0 / fs
            x[r, k0:k1] += a[r, s] * replica[:k1 - k0] * np.exp(2j * np.pi * f_c * (t[k0:k1] - tau))
    if noise > 0:
        x += noise * (rng.normal(size=x.shape) + 1j * rng.normal(size=x.shape)) / np.sqrt(2)
    return x, d, a
