"""FP64 oracle: time-delay estimation between consecutive pings for the
displaced-phase-centre (DPC) motion estimate (Sec. II-D: the measured delay
delta(t) of Eq. 4, from overlapped coherent looks of the seafloor; coarse
delay by quadratic interpolation of the correlation magnitude, fine delay
from the phase of the correlation at the interpolated point).

TEST INFRASTRUCTURE ONLY (see the package docstring).

For ping pair (i, i + 1), a list of J element pairs (e1, e2) whose phase
centres overlap (element e1 of ping i, element e2 of ping i + 1), and window
k of W samples starting at sample k H (K = floor((N_s - W) / H) + 1 windows;
reference time t_k = t0 + (k H + W / 2) / f_s):

    r(l) = sum_j sum_{n in window} a_j[n] conj(b_j[n + l]),   |l| <= L
    a_j = echo[i, e1_j], b_j = echo[i + 1, e2_j], b = 0 outside the record
    rho(l) = |r(l)| / sqrt(sum_j sum_n |a_j[n]|^2 * sum_j sum_n |b_j[n + l]|^2)
    l* = argmax_{|l| < L} |r(l)| (first on ties)
    mu = (m_- - m_+) / (2 (m_- - 2 m_0 + m_+)),  m = |r| at l* - 1, l*, l* + 1
    coarse delay = (l* + mu) / f_s
    r_c = r(l*) + mu (r_+ - r_-) / 2 + mu^2 (r_+ - 2 r_0 + r_-) / 2,  phase = arg r_c

Readings where the paper is silent: the element pairs and window geometry
are inputs; pairs are summed coherently (one estimate per ping pair and
window); ping i + 1's return lagging ping i's by delta gives l ~ delta f_s,
and for baseband echoes of a common delayed return the phase is
2 pi f_c delta (mod 2 pi); the fine delay is (phase + 2 pi m) / (2 pi f_c)
with m the integer that brings it nearest a reference delay (the coarse
delay, or a prior from a first motion solution); the peak search excludes
the end lags so that both neighbours exist; a flat top (zero curvature)
gives mu = 0.
"""
from __future__ import annotations

import math

import numpy as np


def n_windows(n_sample: int, win: int, hop: int) -> int:
    return (n_sample - win) // hop + 1 if n_sample >= win else 0


def correlate(a, b, lags: int):
    """r(l) = sum_n a[n] conj(b[n + l]) for l = -lags..lags, b zero outside its
    array; a, b complex [J, n] with the window of a at b's index offset given
    by the caller (both already cut to the same window origin). Returns r
    [2 lags + 1] and the energies of a and of each shifted b."""
    J, W = a.shape
    Nb = b.shape[1]
    r = np.zeros(2 * lags + 1, dtype=np.complex128)
    eb = np.zeros(2 * lags + 1)
    for li, l in enumerate(range(-lags, lags + 1)):
        idx = np.arange(W) + l + lags
        ok = (idx >= 0) & (idx < Nb)
        bs = np.zeros((J, W), dtype=np.complex128)
        bs[:, ok] = b[:, idx[ok]]
        r[li] = np.sum(a * np.conj(bs))
        eb[li] = np.sum(np.abs(bs) ** 2)
    return r, float(np.sum(np.abs(a) ** 2)), eb


def peak(r, ea: float, eb):
    """Coarse lag (l* + mu), complex correlation at it, and rho(l*)."""
    L = (r.shape[0] - 1) // 2
    m = np.abs(r)
    inner = m[1:-1]
    ic = int(np.argmax(inner)) + 1          # first maximum among |l| < L
    m_, m0, mp = m[ic - 1], m[ic], m[ic + 1]
    den = m_ - 2.0 * m0 + mp
    mu = 0.0 if den == 0.0 else (m_ - mp) / (2.0 * den)
    r_, r0, rp = r[ic - 1], r[ic], r[ic + 1]
    rc = r0 + mu * (rp - r_) / 2.0 + mu * mu * (rp - 2.0 * r0 + r_) / 2.0
    d = math.sqrt(ea * eb[ic])
    rho = float(m0 / d) if d > 0.0 else 0.0
    return (ic - L) + mu, rc, rho, ic - L


def tde(echo, pairs, win: int, hop: int, max_lag: int, fs: float):
    """Per ping pair and window: coarse delay (s), phase (rad), rho, peak lag.
    Arrays [P - 1, K] (float64, float64, float64, int64)."""
    e = np.asarray(echo, dtype=np.complex128)
    P, E, Ns = e.shape
    pr = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    K = n_windows(Ns, win, hop)
    delay = np.zeros((P - 1, K))
    phase = np.zeros((P - 1, K))
    rho = np.zeros((P - 1, K))
    lag = np.zeros((P - 1, K), dtype=np.int64)
    L = max_lag
    for i in range(P - 1):
        for k in range(K):
            n0 = k * hop
            a = e[i, pr[:, 0], n0:n0 + win]
            # b over [n0 - L, n0 + win + L), zero outside the record
            b = np.zeros((pr.shape[0], win + 2 * L), dtype=np.complex128)
            lo, hi = max(0, n0 - L), min(Ns, n0 + win + L)
            b[:, lo - (n0 - L):hi - (n0 - L)] = e[i + 1, pr[:, 1], lo:hi]
            r, ea, eb = correlate(a, b, L)
            lc, rc, rh, l0 = peak(r, ea, eb)
            delay[i, k] = lc / fs
            phase[i, k] = math.atan2(rc.imag, rc.real)
            rho[i, k] = rh
            lag[i, k] = l0
    return delay, phase, rho, lag


def fine_delay(phase, reference_delay, fc: float):
    """(phase + 2 pi m) / (2 pi f_c) with m the integer nearest
    f_c reference - phase / (2 pi): the phase unwrapped around the reference."""
    ph = np.asarray(phase, dtype=np.float64)
    ref = np.asarray(reference_delay, dtype=np.float64)
    m = np.round(fc * ref - ph / (2.0 * math.pi))
    return (ph + 2.0 * math.pi * m) / (2.0 * math.pi * fc)
