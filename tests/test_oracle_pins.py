"""Pins of the FP64 oracle to facts that do not come from the oracle itself.

The paper prints no worked numeric example for backprojection, so the oracle
is pinned to what the geometry and the mathematics fix (Eq. 1 and the
inversion statement of Sec. II-A; gate of Sec. II-C):

* P1  an independent brute-force evaluation at 30 significant digits (mpmath);
* P2  the closed form of a lone point scatterer focused at a pixel centre;
* P3  the focus lands on the pixel nearest an off-grid scatterer;
* P4  linearity in the echoes;
* P5  shift equivariance along a straight, sway-free track;
* P6  the interpolator on echoes where it is exact (linear, single impulse);
* P7  the analytic gradient against central finite differences, and the
      sharpness objective's identities;
* P8  the gated-term count from per-row cone intervals;
* P10 reprojection is the conjugate transpose of backprojection: the
      adjoint identity <A x, y> = <x, A^H y> and, element by element, the
      matrix A assembled column by column from the (pinned) backprojection;
* P11 the windowed-sinc interpolation variant: the brute-force evaluation at
      30 digits, and the lone-scatterer closed form, whose gain stays within
      0.3% of one where linear interpolation loses up to 2.6%.

A plausible slip anywhere in the oracle (a dropped path leg, a wrong phase
sign, transposed tx/rx, an off-by-one tap, a gate on the wrong axis) fails at
least one of these.
"""
import math

import mpmath
import numpy as np
import pytest
import torch

import oracle
from synth import make_config, synthesize_echo
from synth.echo import pulse
from synth.scenario import Grid, linear_array_rx


def _tiny_geometry(seed=7, P=4, E=2, ns=48, gate_deg=25.0, t0=1.5e-3):
    rng = np.random.default_rng(seed)
    tx = np.stack([np.arange(P) * 0.4 + rng.normal(0, 0.01, P),
                   rng.normal(0, 0.02, P), -3.0 + rng.normal(0, 0.02, P)], axis=1)
    rx = linear_array_rx(tx, E, 0.13)
    rx[:, :, 1] += 0.05 * np.arange(E)[None, :]        # break tx/rx symmetry
    echo = rng.normal(size=(P, E, ns)) + 1j * rng.normal(size=(P, E, ns))
    grid = Grid(n=(8, 8, 1), origin=(0.2, 2.0, 0.0), spacing=(0.11, 0.07, 1.0))
    return dict(echo=echo, tx=tx, rx=rx, c=1500.0, fc=9e3, fs=10e3, t0=t0,
                grid=grid, gate=math.radians(gate_deg))


def _brute_mp(g, pts):
    mpmath.mp.dps = 30
    echo, tx, rx = g["echo"], g["tx"], g["rx"]
    c, fc, fs, t0 = (mpmath.mpf(g[k]) for k in ("c", "fc", "fs", "t0"))
    sg = mpmath.sin(mpmath.mpf(g["gate"]))
    out = []
    for p in pts:
        pm = [mpmath.mpf(float(v)) for v in p]
        acc = mpmath.mpc(0)
        for i in range(tx.shape[0]):
            T = [mpmath.mpf(float(v)) for v in tx[i]]
            dT = mpmath.sqrt(sum((pm[k] - T[k]) ** 2 for k in range(3)))
            for e in range(rx.shape[1]):
                R = [mpmath.mpf(float(v)) for v in rx[i, e]]
                dR = mpmath.sqrt(sum((pm[k] - R[k]) ** 2 for k in range(3)))
                if g["gate"] > 0:
                    if not (abs(pm[0] - T[0]) <= sg * dT and abs(pm[0] - R[0]) <= sg * dR):
                        continue
                tau = (dT + dR) / c
                u = (tau - t0) * fs
                n = int(mpmath.floor(u))
                w = u - n
                ns = echo.shape[2]
                a = complex(echo[i, e, n]) if 0 <= n < ns else 0j
                b = complex(echo[i, e, n + 1]) if 0 <= n + 1 < ns else 0j
                L = (1 - w) * mpmath.mpc(a) + w * mpmath.mpc(b)
                acc += L * mpmath.expjpi(2 * fc * tau)
        out.append(complex(acc))
    return np.array(out)


# ------------------------------------------------------------------- P1 ----

@pytest.mark.parametrize("gate_deg,ns,t0", [(0.0, 36, 1.5e-3), (12.0, 36, 1.5e-3), (12.0, 48, 4.95e-3)])
def test_p1_brute_force_mpmath(gate_deg, ns, t0):
    g = _tiny_geometry(gate_deg=gate_deg, ns=ns, t0=t0)
    gr = g["grid"]
    pts = gr.points()
    ref = _brute_mp(g, pts)
    got, cnt = oracle.backproject(g["echo"], g["tx"], g["rx"], g["c"], g["fc"], g["fs"], g["t0"],
                                  pts, g["gate"], return_count=True)
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)
    # the case must exercise what it claims to: taps outside the record, and the gate
    dist = np.linalg.norm(pts[:, None] - g["tx"][None], axis=-1)
    u_max = (dist.max() * 2 / g["c"] - g["t0"]) * g["fs"]
    u_min = (dist.min() * 2 / g["c"] - g["t0"]) * g["fs"]
    assert u_max > g["echo"].shape[2] or u_min < 0
    if gate_deg > 0:
        assert 0 < cnt < pts.shape[0] * 8


# ------------------------------------------------------------------- P2 ----

def _lone(scn_kw, pix, amp=0.7 - 0.4j, bandwidth=None):
    scn = make_config("c1", n_scat=1, snr_db=None, **scn_kw)
    if bandwidth is not None:
        scn.bandwidth = bandwidth
    gr = scn.grid
    p = gr.points(np.array([pix]))[0]
    scn.scat_pos = p[None, :].copy()
    scn.scat_amp = np.array([amp])
    echo = synthesize_echo(scn, noise=False).numpy()
    return scn, p, echo


def test_p2_lone_scatterer_closed_form():
    kw = dict(n_ping=12, n_elem=4, nx=32, ny=32)
    amp = 0.7 - 0.4j
    scn, p, echo = _lone(kw, pix=17 * 32 + 9, amp=amp)
    got = oracle.backproject(echo, scn.tx, scn.rx, scn.c, scn.fc, scn.fs, scn.t0, p[None, :])[0]
    # closed form: each term contributes a * G(w), G(w) = (1-w) h(w) + w h(1-w),
    # w = frac of the geometric delay in samples, h the synthesized pulse
    dT = np.sqrt(((scn.tx - p) ** 2).sum(-1))
    dR = np.sqrt(((scn.rx - p) ** 2).sum(-1))
    u = ((dT[:, None] + dR) / scn.c - scn.t0) * scn.fs
    w = u - np.floor(u)
    h = lambda d: pulse(np.asarray(d, dtype=np.float64), scn.bandwidth, scn.fs, scn.taper_half)
    G = (1 - w) * h(w) + w * h(1 - w)
    want = amp * G.sum()
    # FP64 floor: the carrier argument 2 pi f_c tau is ~2e4 rad, so each term's
    # phase carries ~2e4 * 2^-53 ~ 3e-12 rad of rounding
    assert abs(got - want) <= 1e-11 * abs(want)
    assert abs(np.angle(got / amp)) < 1e-11        # zero residual phase
    assert 0.97 * G.size < G.sum() <= G.size        # G in [0.9745, 1] at B/f_s = 1/4


def test_p2_peak_is_N_times_amplitude_in_the_oversampled_limit():
    # with f_s / B -> infinity the interpolation loss vanishes: |I(p*)| -> P * E * |a|
    kw = dict(n_ping=10, n_elem=3, nx=16, ny=16)
    scn, p, echo = _lone(kw, pix=5 * 16 + 11, amp=1.3 + 0.2j, bandwidth=20.0)
    got = oracle.backproject(echo, scn.tx, scn.rx, scn.c, scn.fc, scn.fs, scn.t0, p[None, :])[0]
    N = scn.n_ping * scn.n_elem
    assert abs(abs(got) - N * abs(1.3 + 0.2j)) < 1e-6 * N
    assert abs(np.angle(got / (1.3 + 0.2j))) < 1e-9


# ------------------------------------------------------------------- P3 ----

@pytest.mark.parametrize("frac", [(0.2, -0.3), (-0.25, 0.15), (0.3, 0.3)])
def test_p3_focus_at_nearest_pixel(frac):
    scn = make_config("c1", n_scat=1, snr_db=None, n_ping=64, n_elem=8, nx=24, ny=24)
    gr = scn.grid
    ix, iy = 11, 13
    p = gr.points(np.array([iy * 24 + ix]))[0].copy()
    p[0] += frac[0] * gr.spacing[0]
    p[1] += frac[1] * gr.spacing[1]
    scn.scat_pos = p[None]
    scn.scat_amp = np.array([1.0 + 0j])
    echo = synthesize_echo(scn, noise=False).numpy()
    img = oracle.backproject_image(echo, scn.tx, scn.rx, scn.c, scn.fc, scn.fs, scn.t0,
                                   gr.origin, gr.spacing, gr.n)
    k = int(np.argmax(np.abs(img)))
    assert (k % 24, (k // 24) % 24) == (ix, iy)


# ------------------------------------------------------------------- P4 ----

def test_p4_linearity():
    g = _tiny_geometry(gate_deg=12.0)
    rng = np.random.default_rng(3)
    e2 = rng.normal(size=g["echo"].shape) + 1j * rng.normal(size=g["echo"].shape)
    al, be = 0.3 - 1.1j, -2.0 + 0.5j
    pts = g["grid"].points()
    args = (g["tx"], g["rx"], g["c"], g["fc"], g["fs"], g["t0"], pts, g["gate"])
    lhs = oracle.backproject(al * g["echo"] + be * e2, *args)
    rhs = al * oracle.backproject(g["echo"], *args) + be * oracle.backproject(e2, *args)
    assert np.linalg.norm(lhs - rhs) <= 1e-14 * 10 * np.linalg.norm(rhs)


# ------------------------------------------------------------------- P5 ----

def test_p5_shift_equivariance_along_track():
    k = 10     # pings of shift; 10 * 0.15 m = 1.5 m = 100 pixels of 1.5 cm
    base = dict(n_ping=120, n_elem=4, nx=12, ny=12, sway_sigma=0.0, gate_deg=10.0, n_sample=4096)
    imgs = []
    for shift in (0, k):
        scn = make_config("c1", n_scat=1, snr_db=None, **base)
        scn.grid.origin = (6.0 + shift * 0.15, 20.1, 0.0)
        scn.scat_pos = np.array([[6.0 + shift * 0.15 + 5.3 * 0.015, 20.1 + 6.6 * 0.015, 0.0]])
        scn.scat_amp = np.array([0.9 + 0.3j])
        echo = synthesize_echo(scn, noise=False).numpy()
        gr = scn.grid
        imgs.append(oracle.backproject_image(echo, scn.tx, scn.rx, scn.c, scn.fc, scn.fs, scn.t0,
                                             gr.origin, gr.spacing, gr.n, scn.gate_half_angle))
    a, b = imgs
    assert np.abs(a).max() > 10.0
    assert np.linalg.norm(a - b) <= 1e-9 * np.linalg.norm(a)


# ------------------------------------------------------------------- P6 ----

def test_p6_linear_echo_is_reproduced_exactly():
    g = _tiny_geometry(gate_deg=0.0, ns=4000)
    P, E, ns = g["echo"].shape
    rng = np.random.default_rng(11)
    al = rng.normal(size=(P, E)) + 1j * rng.normal(size=(P, E))
    be = (rng.normal(size=(P, E)) + 1j * rng.normal(size=(P, E))) * 1e-3
    echo = al[:, :, None] + be[:, :, None] * np.arange(ns)[None, None, :]
    pts = g["grid"].points()
    got = oracle.backproject(echo, g["tx"], g["rx"], g["c"], g["fc"], g["fs"], g["t0"], pts)
    want = np.zeros(pts.shape[0], dtype=np.complex128)
    for i in range(P):
        for e in range(E):
            tau = (np.linalg.norm(pts - g["tx"][i], axis=1) + np.linalg.norm(pts - g["rx"][i, e], axis=1)) / g["c"]
            u = (tau - g["t0"]) * g["fs"]
            assert u.min() > 0 and u.max() < ns - 1
            want += (al[i, e] + be[i, e] * u) * np.exp(2j * np.pi * g["fc"] * tau)
    assert np.linalg.norm(got - want) <= 1e-11 * np.linalg.norm(want)


def test_p6_single_impulse_gives_tent_ring():
    g = _tiny_geometry(gate_deg=0.0, ns=200)
    P, E, ns = g["echo"].shape
    nk = 37
    echo = np.zeros((P, E, ns), dtype=np.complex128)
    echo[:, :, nk] = 1.0
    pts = g["grid"].points()
    got = oracle.backproject(echo, g["tx"], g["rx"], g["c"], g["fc"], g["fs"], g["t0"], pts)
    want = np.zeros(pts.shape[0], dtype=np.complex128)
    for i in range(P):
        for e in range(E):
            tau = (np.linalg.norm(pts - g["tx"][i], axis=1) + np.linalg.norm(pts - g["rx"][i, e], axis=1)) / g["c"]
            u = (tau - g["t0"]) * g["fs"]
            want += np.maximum(0.0, 1.0 - np.abs(u - nk)) * np.exp(2j * np.pi * g["fc"] * tau)
    assert np.abs(want).max() > 0.5          # the ring crosses the grid
    assert np.linalg.norm(got - want) <= 1e-12 * np.linalg.norm(want)


# ------------------------------------------------------------------- P7 ----

def _smooth_case():
    scn = make_config("c5", n_ping=6, n_elem=3, nx=10, ny=10, n_scat=6, err_rms=0.0, snr_db=None)
    # put scatterers inside the small grid so the image is not empty
    gr = scn.grid
    rng = np.random.default_rng(5)
    scn.scat_pos = gr.points(rng.choice(100, 6, replace=False)) + rng.normal(0, 0.004, (6, 3)) * [1, 1, 0]
    echo = synthesize_echo(scn, noise=False).numpy()
    return scn, echo


def test_p7_gradient_matches_central_differences():
    scn, echo = _smooth_case()
    gr = scn.grid
    pts = gr.points()
    rng = np.random.default_rng(9)
    gbar = rng.normal(size=pts.shape[0]) + 1j * rng.normal(size=pts.shape[0])

    def J(tx, rx, c):
        I = oracle.backproject(echo, tx, rx, c, scn.fc, scn.fs, scn.t0, pts)
        return float(np.real(np.vdot(gbar, I)))

    g_tx, g_rx, g_c = oracle.vjp(echo, scn.tx, scn.rx, scn.c, scn.fc, scn.fs, scn.t0, pts, gbar)
    h = 1e-6
    fd_tx = np.zeros_like(scn.tx)
    for i in range(scn.tx.shape[0]):
        for a in range(3):
            tp, tm = scn.tx.copy(), scn.tx.copy()
            tp[i, a] += h
            tm[i, a] -= h
            fd_tx[i, a] = (J(tp, scn.rx, scn.c) - J(tm, scn.rx, scn.c)) / (2 * h)
    fd_rx = np.zeros_like(scn.rx)
    for i in range(scn.rx.shape[0]):
        for e in range(scn.rx.shape[1]):
            for a in range(3):
                rp, rm = scn.rx.copy(), scn.rx.copy()
                rp[i, e, a] += h
                rm[i, e, a] -= h
                fd_rx[i, e, a] = (J(scn.tx, rp, scn.c) - J(scn.tx, rm, scn.c)) / (2 * h)
    hc = 1e-4
    fd_c = (J(scn.tx, scn.rx, scn.c + hc) - J(scn.tx, scn.rx, scn.c - hc)) / (2 * hc)
    assert np.linalg.norm(g_tx - fd_tx) <= 1e-5 * np.linalg.norm(fd_tx)
    assert np.linalg.norm(g_rx - fd_rx) <= 1e-5 * np.linalg.norm(fd_rx)
    assert abs(g_c - fd_c) <= 1e-5 * abs(fd_c)
    assert np.linalg.norm(fd_tx) > 0 and abs(fd_c) > 0


def test_p7_gradient_with_gate_and_record_edge():
    g = _tiny_geometry(gate_deg=12.0, ns=36)
    pts = g["grid"].points()
    rng = np.random.default_rng(4)
    gbar = rng.normal(size=pts.shape[0]) + 1j * rng.normal(size=pts.shape[0])
    args = (g["c"], g["fc"], g["fs"], g["t0"], pts)

    def J(tx, rx):
        return float(np.real(np.vdot(gbar, oracle.backproject(g["echo"], tx, rx, *args, g["gate"]))))

    g_tx, g_rx, _ = oracle.vjp(g["echo"], g["tx"], g["rx"], *args, gbar, g["gate"])
    h = 1e-7     # small enough that no term crosses a gate edge or a tap boundary
    fd = np.zeros_like(g["tx"])
    for i in range(g["tx"].shape[0]):
        for a in range(3):
            tp, tm = g["tx"].copy(), g["tx"].copy()
            tp[i, a] += h
            tm[i, a] -= h
            fd[i, a] = (J(tp, g["rx"]) - J(tm, g["rx"])) / (2 * h)
    assert np.linalg.norm(g_tx - fd) <= 1e-4 * np.linalg.norm(fd)


def test_p7_segment_bound_equals_the_jump_at_a_sample():
    # One monostatic term with u on either side of sample m = 20; the echo is 0
    # at samples 19 and 20 and 1 at 21, so the slope is 0 left of m and 1 right
    # of it. With Gbar = exp(j 2 pi f_c tau), Re(conj(Gbar) D) jumps by exactly
    # f_s, so dJ/dc jumps by f_s tau / c and dJ/dT by f_s |T - p| / (c d_T).
    c, fc, fs = 1500.0, 9e3, 10e3
    echo = np.zeros((1, 1, 40), dtype=np.complex128)
    echo[0, 0, 21] = 1.0
    tx = np.zeros((1, 3))
    rx = np.zeros((1, 1, 3))
    m, eps = 20, 1e-7
    out = {}
    for side in (+1, -1):
        d = (m + side * eps) * c / (2.0 * fs)
        p = np.array([[0.0, d, 0.0]])
        tau = 2.0 * d / c
        gbar = np.array([np.exp(1j * 2.0 * np.pi * fc * tau)])
        out[side] = oracle.vjp(echo, tx, rx, c, fc, fs, 0.0, p, gbar)
        b = oracle.vjp_segment_bound(echo, tx, rx, c, fc, fs, 0.0, p, gbar, delta=1e-6)
        far = oracle.vjp_segment_bound(echo, tx, rx, c, fc, fs, 0.0, p + [0.0, 0.3 * c / (2.0 * fs), 0.0],
                                       gbar, delta=1e-6)
        assert np.all(far[0] == 0) and far[2] == 0.0
        tau_m = 2.0 * m / (2.0 * fs)
        assert b[2] == pytest.approx(fs * tau_m / c, rel=1e-4)
        assert b[0][0, 1] == pytest.approx(fs / c, rel=1e-4)
        assert b[1][0, 0, 1] == pytest.approx(fs / c, rel=1e-4)
    jump_c = abs(out[+1][2] - out[-1][2])
    jump_t = np.abs(out[+1][0] - out[-1][0])
    assert jump_c == pytest.approx(fs * (m / fs) / c, rel=1e-5)
    assert jump_t[0, 1] == pytest.approx(fs / c, rel=1e-5)
    assert jump_c <= b[2] * (1 + 1e-5)


def test_p7_sharpness_identities_and_cotangent():
    one = np.zeros(50, dtype=np.complex128)
    one[17] = 2.5 - 1j
    assert oracle.sharpness(one) == pytest.approx(1.0, rel=1e-15)
    rng = np.random.default_rng(2)
    uni = np.exp(1j * rng.uniform(0, 2 * np.pi, 40)) * 3.0
    assert oracle.sharpness(uni) == pytest.approx(1.0 / 40, rel=1e-13)
    I = rng.normal(size=30) + 1j * rng.normal(size=30)
    G = oracle.sharpness_cotangent(I)
    h = 1e-7
    for k in range(0, 30, 7):
        for unit in (1.0, 1j):
            Ip, Im = I.copy(), I.copy()
            Ip[k] += h * unit
            Im[k] -= h * unit
            fd = (oracle.sharpness(Ip) - oracle.sharpness(Im)) / (2 * h)
            an = G[k].real if unit == 1.0 else G[k].imag
            assert abs(fd - an) <= 1e-6 * abs(G).max()


# ------------------------------------------------------------------- P8 ----

@pytest.mark.parametrize("name", ["c2", "c4b:3"])
def test_p8_gated_count_from_row_intervals(name):
    scn = make_config(name, n_ping=40, n_elem=5, nx=70, ny=33, n_scat=1, snr_db=None)
    gr = scn.grid
    pts = gr.points()
    brute = oracle.gated_term_count(scn.tx, scn.rx, pts, scn.gate_half_angle)
    rows = oracle.gated_term_count_rows(scn.tx, scn.rx, gr.origin, gr.spacing, gr.n, scn.gate_half_angle)
    assert brute == rows
    assert 0 < brute < scn.nominal_updates()
    echo = np.zeros((scn.n_ping, scn.n_elem, 8), dtype=np.complex128)
    _, cnt = oracle.backproject(echo, scn.tx, scn.rx, scn.c, scn.fc, scn.fs, scn.t0, pts,
                                scn.gate_half_angle, return_count=True)
    assert cnt == brute


def test_p8_gated_count_3d_rows():
    # rows run along x at fixed (y, z): the interval form must hold off the z = 0 plane too
    scn = make_config("c3", n_ping=12, n_across=4, nx=20, ny=9, nz=5, n_seabed=0, n_surface=1,
                      n_buried=0, snr_db=None)
    gr = scn.grid
    gate = math.radians(10.0)
    brute = oracle.gated_term_count(scn.tx, scn.rx, gr.points(), gate)
    rows = oracle.gated_term_count_rows(scn.tx, scn.rx, gr.origin, gr.spacing, gr.n, gate)
    assert brute == rows and brute > 0


# ------------------------------------------------------------------ P10 ----

def _inner(a, b):
    return np.vdot(np.asarray(a).ravel(), np.asarray(b).ravel())


@pytest.mark.parametrize("gate_deg,t0", [(0.0, 1.5e-3), (12.0, 1.5e-3), (12.0, 4.95e-3)])
def test_p10_reprojection_satisfies_the_adjoint_identity(gate_deg, t0):
    # t0 = 4.95 ms puts part of the delays past the record end (taps dropped)
    g = _tiny_geometry(gate_deg=gate_deg, t0=t0, ns=48, P=4, E=3)
    pts = g["grid"].points()
    rng = np.random.default_rng(11)
    x = rng.normal(size=g["echo"].shape) + 1j * rng.normal(size=g["echo"].shape)
    y = rng.normal(size=pts.shape[0]) + 1j * rng.normal(size=pts.shape[0])
    ax = oracle.backproject(x, g["tx"], g["rx"], g["c"], g["fc"], g["fs"], g["t0"], pts, g["gate"])
    ahy = oracle.reproject(y, g["tx"], g["rx"], g["c"], g["fc"], g["fs"], g["t0"], pts, x.shape[2], g["gate"])
    lhs, rhs = _inner(ax, y), _inner(x, ahy)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs) and abs(lhs) > 0


def test_p10_reprojection_equals_the_assembled_conjugate_transpose():
    g = _tiny_geometry(gate_deg=12.0, t0=4.95e-3, ns=20, P=2, E=2)
    pts = g["grid"].points()[::3]
    P, E, ns = 2, 2, 20
    # column (i, e, n) of A is the image of a unit echo at that sample
    A = np.zeros((pts.shape[0], P * E * ns), dtype=np.complex128)
    for col in range(P * E * ns):
        unit = np.zeros((P, E, ns), dtype=np.complex128)
        unit.reshape(-1)[col] = 1.0
        A[:, col] = oracle.backproject(unit, g["tx"], g["rx"], g["c"], g["fc"], g["fs"], g["t0"], pts, g["gate"])
    assert np.count_nonzero(A) > 0
    y = np.random.default_rng(5).normal(size=(pts.shape[0], 2)) @ np.array([1.0, 1j])
    got = oracle.reproject(y, g["tx"], g["rx"], g["c"], g["fc"], g["fs"], g["t0"], pts, ns, g["gate"])
    want = (A.conj().T @ y).reshape(P, E, ns)
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


# ------------------------------------------------------------------ P11 ----

def _brute_mp_sinc(g, pts, half=4):
    mpmath.mp.dps = 30
    echo, tx, rx = g["echo"], g["tx"], g["rx"]
    c, fc, fs, t0 = (mpmath.mpf(g[k]) for k in ("c", "fc", "fs", "t0"))
    sg = mpmath.sin(mpmath.mpf(g["gate"]))
    ns = echo.shape[2]

    def h(t):
        if abs(t) >= half:
            return mpmath.mpf(0)
        s = mpmath.mpf(1) if t == 0 else mpmath.sin(mpmath.pi * t) / (mpmath.pi * t)
        return s * (1 + mpmath.cos(mpmath.pi * t / half)) / 2

    out = []
    for p in pts:
        pm = [mpmath.mpf(float(v)) for v in p]
        acc = mpmath.mpc(0)
        for i in range(tx.shape[0]):
            T = [mpmath.mpf(float(v)) for v in tx[i]]
            dT = mpmath.sqrt(sum((pm[k] - T[k]) ** 2 for k in range(3)))
            for e in range(rx.shape[1]):
                R = [mpmath.mpf(float(v)) for v in rx[i, e]]
                dR = mpmath.sqrt(sum((pm[k] - R[k]) ** 2 for k in range(3)))
                if g["gate"] > 0 and not (abs(pm[0] - T[0]) <= sg * dT and abs(pm[0] - R[0]) <= sg * dR):
                    continue
                tau = (dT + dR) / c
                u = (tau - t0) * fs
                n = int(mpmath.floor(u))
                L = mpmath.mpc(0)
                for m in range(n - half + 1, n + half + 1):
                    if 0 <= m < ns:
                        L += mpmath.mpc(complex(echo[i, e, m])) * h(u - m)
                acc += L * mpmath.expjpi(2 * fc * tau)
        out.append(complex(acc))
    return np.array(out)


@pytest.mark.parametrize("gate_deg,t0", [(12.0, 1.5e-3), (0.0, 4.95e-3)])
def test_p11_sinc_variant_brute_force_mpmath(gate_deg, t0):
    g = _tiny_geometry(gate_deg=gate_deg, t0=t0, ns=48, P=3, E=2)
    pts = g["grid"].points()[::2]
    got = oracle.backproject(g["echo"], g["tx"], g["rx"], g["c"], g["fc"], g["fs"], g["t0"], pts, g["gate"],
                             interp="sinc")
    ref = _brute_mp_sinc(g, pts)
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)
    lin = oracle.backproject(g["echo"], g["tx"], g["rx"], g["c"], g["fc"], g["fs"], g["t0"], pts, g["gate"])
    assert np.linalg.norm(got - lin) > 1e-3 * np.linalg.norm(ref)    # a different interpolator


def test_p11_sinc_kernel_interpolates_samples():
    k = np.arange(-6, 7, dtype=np.float64)
    h = oracle.sinc_kernel(k)
    assert h[6] == 1.0 and np.all(np.abs(np.delete(h, 6)) < 1e-15)
    assert oracle.sinc_kernel(np.array([4.0, -4.0, 4.5])).tolist() == [0.0, 0.0, 0.0]


def test_p11_sinc_variant_lone_scatterer_closed_form():
    kw = dict(n_ping=12, n_elem=4, nx=32, ny=32)
    amp = 0.7 - 0.4j
    scn, p, echo = _lone(kw, pix=17 * 32 + 9, amp=amp)
    got = oracle.backproject(echo, scn.tx, scn.rx, scn.c, scn.fc, scn.fs, scn.t0, p[None, :], interp="sinc")[0]
    # closed form: each term contributes a * G(w), G(w) = sum_j h_s(t_j) pulse(t_j)
    # over the taps t_j = w + 3 - j (j = 0..7), h_s the windowed sinc
    dT = np.sqrt(((scn.tx - p) ** 2).sum(-1))
    dR = np.sqrt(((scn.rx - p) ** 2).sum(-1))
    u = ((dT[:, None] + dR) / scn.c - scn.t0) * scn.fs
    w = u - np.floor(u)
    t = w[..., None] + 3.0 - np.arange(8)
    hp = pulse(t, scn.bandwidth, scn.fs, scn.taper_half)
    G = (oracle.sinc_kernel(t) * hp).sum(-1)
    want = amp * G.sum()
    assert abs(got - want) <= 1e-11 * abs(want)
    assert abs(np.angle(got / amp)) < 1e-11
    # the gain over all fractional delays: within 0.3% of one (linear: 2.55% worst)
    ws = np.linspace(0.0, 1.0, 201)[:, None] + 3.0 - np.arange(8)
    Gs = (oracle.sinc_kernel(ws) * pulse(ws, scn.bandwidth, scn.fs, scn.taper_half)).sum(-1)
    assert np.all(np.abs(Gs - 1.0) < 3e-3)


def test_multiprocess_oracle_matches_single():
    g = _tiny_geometry(gate_deg=12.0)
    pts = np.repeat(g["grid"].points(), 3, axis=0) + np.random.default_rng(1).normal(0, 0.01, (192, 3))
    args = (g["echo"], g["tx"], g["rx"], g["c"], g["fc"], g["fs"], g["t0"], pts, g["gate"])
    a = oracle.backproject(*args, workers=1, chunk=50)
    b = oracle.backproject(*args, workers=3, chunk=50)
    assert np.array_equal(a, b)
