"""FP64 oracle: backprojection image, gated-term count and geometry gradient.

TEST INFRASTRUCTURE ONLY (see the package docstring): nothing in the product
path imports this module.

Definition (Eq. 1 and its symbol list, Sec. II-A; per-ping integration with a
field-of-view test, Sec. II-C; transmitter and receiver tested separately, the
bistatic case of Sec. III-B). For a pixel centre p, ping i with transmitter T_i
and receiver element e at R_ie:

    d_T = |p - T_i|,   d_R = |p - R_ie|,   tau = (d_T + d_R) / c
    u   = (tau - t0) * f_s,  n = floor(u),  w = u - n
    L   = (1 - w) * E~[n] + w * E~[n+1]      E~[k] = echo[i, e, k] inside the record, else 0
    g   = [|p_x - T_x| <= sin(theta) d_T] * [|p_x - R_x| <= sin(theta) d_R]   (g = 1 without a gate)
    I(p) = sum_i sum_e  g * L * exp(+j 2 pi f_c tau)

Readings where the paper is silent: linear interpolation in sample index with
zero extension (a Hann-windowed sinc over 8 samples is available as a
variant of the image); t_k = t0 + k / f_s; echoes at complex baseband so the carrier
phase is re-applied; no amplitude weighting; positions fixed per ping.

Continuous motion (variant of the image; the receiver location x_RX(t) of
Eq. 1, with the transmitter stationary while it transmits): with a per-ping
velocity v_i the receivers move during reception, R_ie(t) = R_ie + v_i t
(t after transmit), and tau solves c tau = d_T + |p - R_ie - v_i tau|. With
a = p - R_ie this is the quadratic

    (c^2 - |v|^2) tau^2 - 2 (c d_T - a.v) tau + (d_T^2 - |a|^2) = 0,

whose larger root is the one with c tau - d_T >= 0 (``motion_delay``). The
beam gate keeps the ping-time positions.

Position table (the same variant with the sensor track up-sampled into a
table that is interpolated linearly at the query time, Sec. II-C): ping i's
receivers are displaced by Delta_i(t) from their ping-time positions,
R_ie(t) = R_ie + Delta_i(t), with Delta_i sampled at t_j = j h (j = 0..N - 1)
and linear between samples; before t_0 and after t_{N-1} the first and last
segments extend linearly. tau solves c tau = d_T + |p - R_ie - Delta_i(tau)|;
the right side changes more slowly than the left when the track's speed is
below c, so the root is unique, and ``track_delay`` brackets it by bisection.

Sediment refraction (variant of the image; Sec. III-B): the flat seafloor
z = z_int separates water (c, above; the array is in the water) from sediment
(c_sed, below). A leg from apex X to a pixel p below the interface crosses it
where the travel time |X - q| / c + |q - p| / c_sed is least; that point lies in
the vertical plane through X and p, at horizontal distance r from X where
Snell's law r / (c |X - q|) = (D - r) / (c_sed |q - p|) holds (D the horizontal
distance of X and p; the left side grows and the right side falls with r, so
the root is unique: ``refracted_leg`` brackets it by bisection). Legs to
pixels at or above the interface are straight. The beam gate keeps straight
lines.

Gradient (vector-Jacobian product) for a cotangent Gbar = dJ/dRe I + j dJ/dIm I:

    dJ/dtheta = sum_p Re( conj(Gbar(p)) * sum_ie g * D_ie(p) * dtau_ie/dtheta )
    D = [ f_s (E~[n+1] - E~[n]) + j 2 pi f_c L ] * exp(j 2 pi f_c tau)
    dtau/dT_i = (T_i - p) / (c d_T),  dtau/dR_ie = (R_ie - p) / (c d_R),  dtau/dc = -tau / c

The gate is held constant and the slope is that of the segment containing u.
"""
from __future__ import annotations

import math
import os

import numpy as np


def pixel_points(origin, spacing, n, index=None) -> np.ndarray:
    """Pixel centres [N,3] float64: origin + index * spacing per axis, x fastest."""
    nx, ny, nz = (int(v) for v in n)
    if index is None:
        index = np.arange(nx * ny * nz, dtype=np.int64)
    index = np.asarray(index, dtype=np.int64)
    ix = (index % nx).astype(np.float64)
    iy = ((index // nx) % ny).astype(np.float64)
    iz = (index // (nx * ny)).astype(np.float64)
    pts = np.empty((index.size, 3), dtype=np.float64)
    pts[:, 0] = origin[0] + ix * spacing[0]
    pts[:, 1] = origin[1] + iy * spacing[1]
    pts[:, 2] = origin[2] + iz * spacing[2]
    return pts


def _taps(row: np.ndarray, n: np.ndarray):
    """E~[n] and E~[n+1] with zero outside the record."""
    ns = row.shape[0]
    a = np.zeros(n.shape, dtype=np.complex128)
    b = np.zeros(n.shape, dtype=np.complex128)
    ia = (n >= 0) & (n < ns)
    ib = (n + 1 >= 0) & (n + 1 < ns)
    a[ia] = row[n[ia]]
    b[ib] = row[n[ib] + 1]
    return a, b


def _gate(dx: np.ndarray, d: np.ndarray, sin_g: float) -> np.ndarray:
    return np.abs(dx) <= sin_g * d


SINC_HALF = 4   # the windowed-sinc interpolator uses 2 * SINC_HALF taps


def sinc_kernel(t, half: int = SINC_HALF) -> np.ndarray:
    """Hann-windowed sinc: sinc(t) (1 + cos(pi t / half)) / 2 for |t| < half, 0 beyond."""
    t = np.asarray(t, dtype=np.float64)
    return np.where(np.abs(t) < half, np.sinc(t) * 0.5 * (1.0 + np.cos(np.pi * t / half)), 0.0)


def _sinc_interp(row: np.ndarray, u: np.ndarray, half: int = SINC_HALF) -> np.ndarray:
    """sum over m = floor(u) - half + 1 .. floor(u) + half of E~[m] h(u - m)."""
    n = np.floor(u).astype(np.int64)
    ns = row.shape[0]
    out = np.zeros(u.shape, dtype=np.complex128)
    for j in range(2 * half):
        m = n - half + 1 + j
        inside = (m >= 0) & (m < ns)
        v = np.zeros(u.shape, dtype=np.complex128)
        v[inside] = row[m[inside]]
        out += v * sinc_kernel(u - m, half)
    return out


def motion_delay(d_T, a, v, c):
    """Two-way delay with the receiver moving at v during reception: the root
    of c tau = d_T + |a - v tau| (a = p - R at transmit; a [N, 3], v [3])."""
    av = a @ v
    vv = float(v @ v)
    aa = np.sum(a * a, axis=1)
    A = c * c - vv
    Bh = c * d_T - av
    return (Bh + np.sqrt(Bh * Bh - A * (d_T * d_T - aa))) / A


def track_position(table, h, t):
    """Delta(t) of one ping's table [N, 3] (samples every h seconds from t = 0),
    linear between samples and extended linearly past both ends; t [M]."""
    table = np.asarray(table, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    n = table.shape[0]
    j = np.clip(np.floor(t / h), 0, n - 2).astype(np.int64)
    frac = t / h - j                        # outside [0, 1] on the extended end segments
    return table[j] + frac[:, None] * (table[j + 1] - table[j])


def track_delay(d_T, a, table, h, c):
    """Two-way delay with the receivers displaced by the table: the root of
    c tau = d_T + |a - Delta(tau)| (a = p - R at transmit, [M, 3]), by
    bisection on tau (100 halvings of a bracket that starts at 0)."""
    d_T = np.asarray(d_T, dtype=np.float64)
    a = np.asarray(a, dtype=np.float64)
    f = lambda tau: c * tau - d_T - np.linalg.norm(a - track_position(table, h, tau), axis=1)
    lo = np.zeros_like(d_T)
    hi = 2.0 * (d_T + np.linalg.norm(a, axis=1)) / c + h
    for _ in range(64):                      # widen until the bracket holds the root
        grow = f(hi) <= 0.0
        if not grow.any():
            break
        hi = np.where(grow, 2.0 * hi, hi)
    for _ in range(100):
        mid = 0.5 * (lo + hi)
        neg = f(mid) < 0.0
        lo = np.where(neg, mid, lo)
        hi = np.where(neg, hi, mid)
    return 0.5 * (lo + hi)


def refracted_leg(X, pts, c, c_sed, z_int):
    """One-way travel time from X [3] (in the water) to every point of pts [N, 3]."""
    X = np.asarray(X, dtype=np.float64)
    D = np.sqrt((pts[:, 0] - X[0]) ** 2 + (pts[:, 1] - X[1]) ** 2)
    h1 = z_int - X[2]
    h2 = pts[:, 2] - z_int
    below = h2 > 0
    lo, hi = np.zeros_like(D), D.copy()
    h2c = np.where(below, h2, 1.0)      # pixels at or above the interface take the straight path below
    for _ in range(100):                 # brackets D / 2^100: far below FP64 resolution
        r = 0.5 * (lo + hi)
        f = r / (c * np.sqrt(r * r + h1 * h1)) - (D - r) / (c_sed * np.sqrt((D - r) ** 2 + h2c * h2c))
        lo = np.where(f < 0, r, lo)
        hi = np.where(f < 0, hi, r)
    r = 0.5 * (lo + hi)
    t = np.sqrt(r * r + h1 * h1) / c + np.sqrt((D - r) ** 2 + h2c * h2c) / c_sed
    return np.where(below, t, np.sqrt(((pts - X) ** 2).sum(axis=1)) / c)


def _bp_chunk(echo, tx, rx, c, fc, fs, t0, pts, gate, interp="linear", vel=None, refr=None, track=None,
              track_h=None):
    P, E = rx.shape[0], rx.shape[1]
    acc = np.zeros(pts.shape[0], dtype=np.complex128)
    count = 0
    sin_g = math.sin(gate) if gate > 0 else None
    for i in range(P):
        dT = np.sqrt(((pts - tx[i]) ** 2).sum(axis=1))
        gT = _gate(pts[:, 0] - tx[i, 0], dT, sin_g) if sin_g is not None else None
        tT = None if refr is None else refracted_leg(tx[i], pts, c, refr[0], refr[1])
        for e in range(E):
            R = rx[i, e]
            dR = np.sqrt(((pts - R) ** 2).sum(axis=1))
            if refr is not None:
                tau = tT + refracted_leg(R, pts, c, refr[0], refr[1])
            elif track is not None:
                tau = track_delay(dT, pts - R, track[i], track_h, c)
            else:
                tau = (dT + dR) / c if vel is None else motion_delay(dT, pts - R, vel[i], c)
            u = (tau - t0) * fs
            if interp == "sinc":
                L = _sinc_interp(echo[i, e], u)
            else:
                nf = np.floor(u)
                w = u - nf
                a, b = _taps(echo[i, e], nf.astype(np.int64))
                L = (1.0 - w) * a + w * b
            term = L * np.exp(1j * 2.0 * np.pi * fc * tau)
            if sin_g is not None:
                g = gT & _gate(pts[:, 0] - R[0], dR, sin_g)
                term = np.where(g, term, 0.0)
                count += int(g.sum())
            else:
                count += pts.shape[0]
            acc += term
    return acc, count


def _worker(args):
    specs, sc, lo, hi = args
    from . import pool
    a = pool.attach(specs)
    return _bp_chunk(a["echo"], a["tx"], a["rx"], sc["c"], sc["fc"], sc["fs"], sc["t0"],
                     a["pts"][lo:hi], sc["gate"], sc["interp"], a["vel"], sc["refr"], a["track"], sc["track_h"])


def backproject(echo, tx, rx, c, fc, fs, t0, points, gate_half_angle=0.0,
                workers=1, chunk=4096, return_count=False, interp="linear", rx_vel=None, refraction=None,
                rx_track=None):
    """Backprojected complex values at arbitrary points [N,3] (float64 in, complex128 out).

    echo: complex [P,E,N_s]; tx: [P,3]; rx: [P,E,3]; gate_half_angle in radians
    (0 = no gate). ``workers`` > 1 splits the points over the worker pool of
    ``oracle.pool`` (arrays passed through shared memory).
    ``interp`` = "linear" (the definition above) or "sinc": the interpolation
    variant L = sum over the 2 SINC_HALF samples m around u of E~[m] h(u - m),
    h the Hann-windowed sinc of ``sinc_kernel``. ``rx_vel`` ([P, 3], m/s)
    selects continuous receiver motion (``motion_delay``); ``rx_track`` =
    (table [P, N, 3], h) the same with a position table (``track_delay``);
    ``refraction`` = (c_sed, z_int) the sediment interface (``refracted_leg``).
    """
    echo = np.asarray(echo)
    if echo.dtype not in (np.complex64, np.complex128):   # complex64 samples convert exactly per tap
        echo = echo.astype(np.complex128)
    echo = np.ascontiguousarray(echo)
    tx = np.asarray(tx, dtype=np.float64)
    rx = np.asarray(rx, dtype=np.float64)
    pts = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    vel = None if rx_vel is None else np.asarray(rx_vel, dtype=np.float64).reshape(-1, 3)
    track, track_h = (None, None) if rx_track is None else (np.ascontiguousarray(rx_track[0], dtype=np.float64),
                                                           float(rx_track[1]))
    N = pts.shape[0]
    spans = [(lo, min(N, lo + chunk)) for lo in range(0, N, chunk)]
    out = np.zeros(N, dtype=np.complex128)
    total = 0
    if workers <= 1 or len(spans) <= 1:
        for lo, hi in spans:
            v, cnt = _bp_chunk(echo, tx, rx, float(c), fc, fs, t0, pts[lo:hi], gate_half_angle, interp, vel,
                               refraction, track, track_h)
            out[lo:hi] = v
            total += cnt
    else:
        from . import pool
        workers_pool, _ = pool.get()
        sc = dict(c=float(c), fc=fc, fs=fs, t0=t0, gate=gate_half_angle, interp=interp, refr=refraction,
                  track_h=track_h)
        with pool.Shared(echo=echo, tx=tx, rx=rx, pts=pts, vel=vel, track=track) as sh:
            res = workers_pool.map(_worker, [(sh.specs, sc, lo, hi) for lo, hi in spans], chunksize=1)
        for (lo, hi), (v, cnt) in zip(spans, res):
            out[lo:hi] = v
            total += cnt
    return (out, total) if return_count else out


def backproject_image(echo, tx, rx, c, fc, fs, t0, origin, spacing, n, gate_half_angle=0.0,
                      workers=1, return_count=False, interp="linear", rx_vel=None, refraction=None, rx_track=None):
    """Full image [nz, ny, nx] complex128 on the grid origin + index * spacing."""
    pts = pixel_points(origin, spacing, n)
    r = backproject(echo, tx, rx, c, fc, fs, t0, pts, gate_half_angle, workers=workers,
                    return_count=return_count, interp=interp, rx_vel=rx_vel, refraction=refraction,
                    rx_track=rx_track)
    nx, ny, nz = (int(v) for v in n)
    if return_count:
        return r[0].reshape(nz, ny, nx), r[1]
    return r.reshape(nz, ny, nx)


def gated_term_count(tx, rx, points, gate_half_angle) -> int:
    """Number of (pixel, ping, element) terms with g = 1, testing every term."""
    tx = np.asarray(tx, dtype=np.float64)
    rx = np.asarray(rx, dtype=np.float64)
    pts = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    if gate_half_angle <= 0:
        return pts.shape[0] * rx.shape[0] * rx.shape[1]
    s = math.sin(gate_half_angle)
    total = 0
    for i in range(tx.shape[0]):
        dT = np.sqrt(((pts - tx[i]) ** 2).sum(axis=1))
        gT = _gate(pts[:, 0] - tx[i, 0], dT, s)
        for e in range(rx.shape[1]):
            dR = np.sqrt(((pts - rx[i, e]) ** 2).sum(axis=1))
            total += int((gT & _gate(pts[:, 0] - rx[i, e, 0], dR, s)).sum())
    return total


def gated_term_count_rows(tx, rx, origin, spacing, n, gate_half_angle) -> int:
    """Same count from per-row x-intervals of the cone (no per-term test).

    For a row of pixels at fixed (y, z), |x - X| <= sin(theta) sqrt((x-X)^2 + rho^2)
    is the interval |x - X| <= tan(theta) rho, with rho the (y, z) distance to X.
    """
    tx = np.asarray(tx, dtype=np.float64)
    rx = np.asarray(rx, dtype=np.float64)
    nx, ny, nz = (int(v) for v in n)
    if gate_half_angle <= 0:
        return nx * ny * nz * rx.shape[0] * rx.shape[1]
    t = math.tan(gate_half_angle)
    ys = origin[1] + np.arange(ny) * spacing[1]
    zs = origin[2] + np.arange(nz) * spacing[2]
    Y, Z = np.meshgrid(ys, zs, indexing="xy")
    Y, Z = Y.ravel(), Z.ravel()
    total = 0
    for i in range(tx.shape[0]):
        hT = t * np.hypot(Y - tx[i, 1], Z - tx[i, 2])
        loT, hiT = tx[i, 0] - hT, tx[i, 0] + hT
        for e in range(rx.shape[1]):
            R = rx[i, e]
            hR = t * np.hypot(Y - R[1], Z - R[2])
            lo = np.maximum(loT, R[0] - hR)
            hi = np.minimum(hiT, R[0] + hR)
            ilo = np.maximum(np.ceil((lo - origin[0]) / spacing[0]), 0)
            ihi = np.minimum(np.floor((hi - origin[0]) / spacing[0]), nx - 1)
            total += int(np.clip(ihi - ilo + 1, 0, None).sum())
    return total


def vjp(echo, tx, rx, c, fc, fs, t0, points, gbar, gate_half_angle=0.0):
    """Gradient of J w.r.t. (tx [P,3], rx [P,E,3], c) given Gbar at the points."""
    echo = np.asarray(echo).astype(np.complex128, copy=False)
    tx = np.asarray(tx, dtype=np.float64)
    rx = np.asarray(rx, dtype=np.float64)
    pts = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    gbar = np.asarray(gbar, dtype=np.complex128).reshape(-1)
    P, E = rx.shape[0], rx.shape[1]
    g_tx = np.zeros((P, 3))
    g_rx = np.zeros((P, E, 3))
    g_c = 0.0
    sin_g = math.sin(gate_half_angle) if gate_half_angle > 0 else None
    for i in range(P):
        dT = np.sqrt(((pts - tx[i]) ** 2).sum(axis=1))
        gT = _gate(pts[:, 0] - tx[i, 0], dT, sin_g) if sin_g is not None else None
        for e in range(E):
            R = rx[i, e]
            dR = np.sqrt(((pts - R) ** 2).sum(axis=1))
            tau = (dT + dR) / c
            u = (tau - t0) * fs
            nf = np.floor(u)
            w = u - nf
            a, b = _taps(echo[i, e], nf.astype(np.int64))
            L = (1.0 - w) * a + w * b
            ph = np.exp(1j * 2.0 * np.pi * fc * tau)
            D = (fs * (b - a) + 1j * 2.0 * np.pi * fc * L) * ph
            coef = np.real(np.conj(gbar) * D)
            if sin_g is not None:
                g = gT & _gate(pts[:, 0] - R[0], dR, sin_g)
                coef = np.where(g, coef, 0.0)
            g_tx[i] += ((coef / (c * dT))[:, None] * (tx[i] - pts)).sum(axis=0)
            g_rx[i, e] += ((coef / (c * dR))[:, None] * (R - pts)).sum(axis=0)
            g_c += float((coef * (-tau / c)).sum())
    return g_tx, g_rx, g_c


def vjp_segment_bound(echo, tx, rx, c, fc, fs, t0, points, gbar, gate_half_angle=0.0, delta=1e-4):
    """Largest change of ``vjp`` that choosing the other interpolation segment
    can make for terms whose sample position u lies within ``delta`` samples of
    an integer (the derivative of the linear interpolator jumps there, so an
    implementation whose u carries a rounding error up to ``delta`` may take
    either slope). Returns non-negative (b_tx [P,3], b_rx [P,E,3], b_c).

    For such a term with m = round(u), the slopes left and right of sample m
    are s_l = E~[m] - E~[m-1] and s_r = E~[m+1] - E~[m]; the two choices of D
    differ by at most f_s |s_r - s_l| + 2 pi f_c delta (|s_l| + |s_r|) (the
    second part bounds the change of L over the rounding interval). Each term's
    bound is |Gbar| times that, times |dtau/dtheta| per component.
    """
    echo = np.asarray(echo).astype(np.complex128, copy=False)
    tx = np.asarray(tx, dtype=np.float64)
    rx = np.asarray(rx, dtype=np.float64)
    pts = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    gbar = np.asarray(gbar, dtype=np.complex128).reshape(-1)
    P, E = rx.shape[0], rx.shape[1]
    b_tx = np.zeros((P, 3))
    b_rx = np.zeros((P, E, 3))
    b_c = 0.0
    sin_g = math.sin(gate_half_angle) if gate_half_angle > 0 else None
    for i in range(P):
        dT = np.sqrt(((pts - tx[i]) ** 2).sum(axis=1))
        gT = _gate(pts[:, 0] - tx[i, 0], dT, sin_g) if sin_g is not None else None
        for e in range(E):
            R = rx[i, e]
            dR = np.sqrt(((pts - R) ** 2).sum(axis=1))
            tau = (dT + dR) / c
            u = (tau - t0) * fs
            m = np.round(u)
            near = np.abs(u - m) < delta
            if sin_g is not None:
                near &= gT & _gate(pts[:, 0] - R[0], dR, sin_g)
            if not near.any():
                continue
            mi = m[near].astype(np.int64)
            em1, e0 = _taps(echo[i, e], mi - 1)
            _, e1 = _taps(echo[i, e], mi)
            sl, sr = e0 - em1, e1 - e0
            dD = fs * np.abs(sr - sl) + 2.0 * np.pi * fc * delta * (np.abs(sl) + np.abs(sr))
            q = np.abs(gbar[near]) * dD
            p = pts[near]
            b_tx[i] += ((q / (c * dT[near]))[:, None] * np.abs(tx[i] - p)).sum(axis=0)
            b_rx[i, e] += ((q / (c * dR[near]))[:, None] * np.abs(R - p)).sum(axis=0)
            b_c += float((q * tau[near] / c).sum())
    return b_tx, b_rx, b_c


def reproject(ybar, tx, rx, c, fc, fs, t0, points, n_sample, gate_half_angle=0.0):
    """Linear adjoint of the image with respect to the echo (reprojection).

    The image is complex-linear in the echo cube: I = A E, with one row of A
    per point and, per term (point p, ping i, element e) with g = 1, the entry
    (1 - w) exp(+j 2 pi f_c tau) on sample n = floor(u) of row (i, e) and
    w exp(+j 2 pi f_c tau) on sample n + 1 (samples outside the record have no
    entry: the zero extension). This returns A^H Y for Y at the points, an
    echo-shaped complex128 [P, E, n_sample]. For Y = Gbar (dJ/dRe I +
    j dJ/dIm I) it is the gradient of J with respect to the echo in the same
    convention.
    """
    tx = np.asarray(tx, dtype=np.float64)
    rx = np.asarray(rx, dtype=np.float64)
    pts = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    ybar = np.asarray(ybar, dtype=np.complex128).reshape(-1)
    P, E = rx.shape[0], rx.shape[1]
    out = np.zeros((P, E, int(n_sample)), dtype=np.complex128)
    sin_g = math.sin(gate_half_angle) if gate_half_angle > 0 else None
    for i in range(P):
        dT = np.sqrt(((pts - tx[i]) ** 2).sum(axis=1))
        gT = _gate(pts[:, 0] - tx[i, 0], dT, sin_g) if sin_g is not None else None
        for e in range(E):
            R = rx[i, e]
            dR = np.sqrt(((pts - R) ** 2).sum(axis=1))
            tau = (dT + dR) / c
            u = (tau - t0) * fs
            nf = np.floor(u)
            w = u - nf
            n = nf.astype(np.int64)
            v = np.exp(-1j * 2.0 * np.pi * fc * tau) * ybar
            if sin_g is not None:
                v = np.where(gT & _gate(pts[:, 0] - R[0], dR, sin_g), v, 0.0)
            row = out[i, e]
            lo = (n >= 0) & (n < n_sample)
            hi = (n + 1 >= 0) & (n + 1 < n_sample)
            np.add.at(row, n[lo], (1.0 - w[lo]) * v[lo])
            np.add.at(row, n[hi] + 1, w[hi] * v[hi])
    return out


def sharpness(img) -> float:
    """S = sum |I|^4 / (sum |I|^2)^2."""
    m2 = np.abs(np.asarray(img, dtype=np.complex128)) ** 2
    return float((m2 ** 2).sum() / m2.sum() ** 2)


def sharpness_cotangent(img) -> np.ndarray:
    """Gbar = dS/dRe I + j dS/dIm I = 4 I (|I|^2 / B^2 - A / B^3), A = sum|I|^4, B = sum|I|^2."""
    I = np.asarray(img, dtype=np.complex128)
    m2 = np.abs(I) ** 2
    A = (m2 ** 2).sum()
    B = m2.sum()
    return 4.0 * I * (m2 / B ** 2 - A / B ** 3)
