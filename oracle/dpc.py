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


# ---------------------------------------------------------------------------
# Motion estimate from the measured delays (Eqs. 3-8, Sec. II-D).
#
# Unknowns: the sway and heave velocities v_y[i], v_z[i] of every ping; the
# surge v_x[i] is known (DVL or along-track estimate). Readings where the
# paper is silent or garbled:
#   * positions integrate the velocities, p_i(0) = p_0 + sum_{n<i} v_n dt_n,
#     and move on during reception, p_i(t) = p_i(0) + v_i t (Eq. 5's first-
#     order kinematics);
#   * Omega (attitude and lever arms) is a fixed attitude with lever arms:
#     TX_i = p_i(0) + l_T, RX_ie(t) = p_i(t) + l_e;
#   * the footprint p_s of window k of ping pair i is fixed in the world: the
#     point of the flat seafloor z = z_floor, abeam (same x) of the pairs' mean
#     phase centre of ping i on the look side, whose two-way time from that
#     phase centre is t_k under the nominal navigation (the caller's prior);
#   * the J element pairs enter one residual through the mean of their path
#     differences: g = c^-1 mean_j (path_1j - path_2j) + delta;
#   * h is the square (Eq. 5) or the Huber function of Eq. 3 of g / sigma;
#     residuals carry weights w (e.g. the correlation coefficients);
#   * Eq. 7 compares ping i's integrated depth with z_DVL[i] (the sum runs over
#     the intervals before ping i);
#   * the solve is Levenberg-Marquardt on the stacked residuals, the Huber
#     case by iteratively reweighted least squares.
# ---------------------------------------------------------------------------


def huber(a):
    """Eq. 3: a^2 / 2 for |a| <= 1, |a| - 1/2 beyond."""
    a = np.abs(np.asarray(a, dtype=np.float64))
    return np.where(a <= 1.0, 0.5 * a * a, a - 0.5)


def platform_positions(p0, vel, dt):
    """p_i(0) for every ping: p0 + sum_{n<i} v_n dt_n. vel [P, 3], dt [P - 1]."""
    vel = np.asarray(vel, dtype=np.float64)
    steps = vel[:-1] * np.asarray(dt, dtype=np.float64)[:, None]
    return np.asarray(p0, dtype=np.float64)[None, :] + np.concatenate([np.zeros((1, 3)), np.cumsum(steps, axis=0)])


def footprints(p0, vel_nominal, dt, lever_tx, lever_rx, pairs, t_ref, c, z_floor, look=1.0):
    """p_s [P - 1, K, 3] for every ping pair and window, from the nominal navigation."""
    pos = platform_positions(p0, vel_nominal, dt)
    pr = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    lt = np.asarray(lever_tx, dtype=np.float64)
    lr = np.asarray(lever_rx, dtype=np.float64)
    pc_off = 0.5 * (lt + lr[pr[:, 0]].mean(axis=0))
    t = np.asarray(t_ref, dtype=np.float64)
    out = np.zeros((pos.shape[0] - 1, t.size, 3))
    for i in range(pos.shape[0] - 1):
        pc = pos[i] + pc_off
        slant = 0.5 * c * t
        dz = z_floor - pc[2]
        ground = np.sqrt(np.maximum(slant * slant - dz * dz, 0.0))
        out[i, :, 0] = pc[0]
        out[i, :, 1] = pc[1] + look * ground
        out[i, :, 2] = z_floor
    return out


def residuals(vyz, vx, p0, dt, lever_tx, lever_rx, pairs, t_ref, ps, delay, c):
    """Eq. 4 for every ping pair i and window k: g[i, k] (seconds).
    vyz [P, 2] (v_y, v_z); vx [P]."""
    vyz = np.asarray(vyz, dtype=np.float64).reshape(-1, 2)
    vel = np.column_stack([np.asarray(vx, dtype=np.float64), vyz])
    pos = platform_positions(p0, vel, dt)
    pr = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    lt = np.asarray(lever_tx, dtype=np.float64)
    lr = np.asarray(lever_rx, dtype=np.float64)
    t = np.asarray(t_ref, dtype=np.float64)
    P = pos.shape[0]
    g = np.zeros((P - 1, t.size))
    for i in range(P - 1):
        s = ps[i]                                            # [K, 3]
        tx1, tx2 = pos[i] + lt, pos[i + 1] + lt
        d = np.zeros(t.size)
        for e1, e2 in pr:
            rx1 = pos[i][None, :] + vel[i][None, :] * t[:, None] + lr[e1]
            rx2 = pos[i + 1][None, :] + vel[i + 1][None, :] * t[:, None] + lr[e2]
            p1 = np.linalg.norm(tx1 - s, axis=1) + np.linalg.norm(s - rx1, axis=1)
            p2 = np.linalg.norm(tx2 - s, axis=1) + np.linalg.norm(s - rx2, axis=1)
            d += p1 - p2
        g[i] = d / (c * pr.shape[0]) + np.asarray(delay[i], dtype=np.float64)
    return g


def smooth_terms(vyz):
    """Second differences of v_y and v_z (the terms squared in Eq. 6)."""
    v = np.asarray(vyz, dtype=np.float64).reshape(-1, 2)
    return v[:-2] - 2.0 * v[1:-1] + v[2:]


def dvl_terms(vz, p0z, dt, z_dvl):
    """Eq. 7's bracket for every ping: integrated depth minus z_DVL."""
    z = p0z + np.concatenate([[0.0], np.cumsum(np.asarray(vz[:-1]) * np.asarray(dt))])
    return z - np.asarray(z_dvl, dtype=np.float64)


def loss(vyz, vx, p0, dt, lever_tx, lever_rx, pairs, t_ref, ps, delay, c, weights, sigma, lam1, lam2, z_dvl,
         robust=False):
    """Eq. 8: L_DPC + lambda_1 L_smooth + lambda_2 L_DVL."""
    g = residuals(vyz, vx, p0, dt, lever_tx, lever_rx, pairs, t_ref, ps, delay, c) / sigma
    w = np.asarray(weights, dtype=np.float64)
    l_dpc = np.sum(w * (huber(g) if robust else g * g))
    v = np.asarray(vyz, dtype=np.float64).reshape(-1, 2)
    l_s = np.sum(smooth_terms(v) ** 2)
    l_d = np.sum(dvl_terms(v[:, 1], p0[2], dt, z_dvl) ** 2)
    return l_dpc + lam1 * l_s + lam2 * l_d


def _stacked(vyz, args, wsqrt):
    (vx, p0, dt, lever_tx, lever_rx, pairs, t_ref, ps, delay, c, sigma, lam1, lam2, z_dvl) = args
    v = vyz.reshape(-1, 2)
    g = residuals(v, vx, p0, dt, lever_tx, lever_rx, pairs, t_ref, ps, delay, c) / sigma
    return np.concatenate([wsqrt * g.ravel(), math.sqrt(lam1) * smooth_terms(v).ravel(),
                           math.sqrt(lam2) * dvl_terms(v[:, 1], p0[2], dt, z_dvl)])


def solve(vyz0, vx, p0, dt, lever_tx, lever_rx, pairs, t_ref, ps, delay, c, weights, sigma, lam1, lam2, z_dvl,
          robust=False, iters=30, h=1e-6):
    """Levenberg-Marquardt over v_y, v_z of every ping (numerical Jacobian by
    central differences; dense normal equations). Returns (vyz [P, 2], loss)."""
    args = (vx, p0, dt, lever_tx, lever_rx, pairs, t_ref, ps, delay, c, sigma, lam1, lam2, z_dvl)
    x = np.asarray(vyz0, dtype=np.float64).ravel().copy()
    w = np.asarray(weights, dtype=np.float64)
    lam = 1e-3
    L = lambda xx: loss(xx.reshape(-1, 2), vx, p0, dt, lever_tx, lever_rx, pairs, t_ref, ps, delay, c, w, sigma,
                        lam1, lam2, z_dvl, robust)
    cur = L(x)
    for _ in range(iters):
        if robust:   # IRLS: h'(a) = omega a, so sqrt(w omega / 2) a has the gradient of w h(a)
            g = residuals(x.reshape(-1, 2), vx, p0, dt, lever_tx, lever_rx, pairs, t_ref, ps, delay, c) / sigma
            wi = 0.5 * w * np.where(np.abs(g) <= 1.0, 1.0, 1.0 / np.maximum(np.abs(g), 1e-300))
        else:
            wi = w
        ws = np.sqrt(wi).ravel()
        r = _stacked(x, args, ws)
        Jm = np.zeros((r.size, x.size))
        for q in range(x.size):
            xp, xm = x.copy(), x.copy()
            xp[q] += h
            xm[q] -= h
            Jm[:, q] = (_stacked(xp, args, ws) - _stacked(xm, args, ws)) / (2 * h)
        A = Jm.T @ Jm
        gvec = Jm.T @ r
        improved = False
        for _ in range(10):
            step = np.linalg.solve(A + lam * np.diag(np.diag(A) + 1e-12), -gvec)
            new = L(x + step)
            if new < cur:
                x, cur, lam = x + step, new, max(lam / 3.0, 1e-12)
                improved = True
                break
            lam *= 4.0
        if not improved or np.linalg.norm(step) < 1e-12 * (1 + np.linalg.norm(x)):
            break
    return x.reshape(-1, 2), cur
