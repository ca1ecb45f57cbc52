"""Pins of the continuous-motion variant of the oracle (the receiver location
x_RX(t) of Eq. 1 moving during reception, the transmitter stationary while
it transmits).

* P12a: a zero velocity gives the stop-and-hop image.
* P12b: ``motion_delay`` solves the defining equation c tau = d_T +
  |a - v tau|, checked against bisection on that equation (monotone in tau
  for |v| < c), for speeds up to 20 m/s in every direction.
* P12c: a lone scatterer at a pixel centre, its echo synthesized with the
  receivers moving (the synthesis finds each delay by fixed-point
  iteration), images to the P2 closed form a * sum G(w) with w taken from the
  bisection delays, with zero residual phase; the stop-and-hop image of the
  same echo does not.
"""
import importlib
import inspect
import types

import numpy as np
import pytest

import oracle
from synth import make_config, synthesize_echo, receiver_velocity, receiver_track
from synth.echo import pulse


def _bisect_delay(d_T, a, v, c):
    lo = np.zeros_like(d_T)
    hi = 2.0 * (d_T + np.linalg.norm(a, axis=1)) / c + 1.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        f = c * mid - d_T - np.linalg.norm(a - mid[:, None] * v[None, :], axis=1)
        lo = np.where(f < 0, mid, lo)
        hi = np.where(f < 0, hi, mid)
    return 0.5 * (lo + hi)


def test_p12a_zero_velocity_is_stop_and_hop():
    scn = make_config("c1", n_ping=6, n_elem=3, nx=24, ny=20)
    from synth import synthesize_echo as se
    echo = se(scn).numpy()
    pts = scn.grid.points()
    a = oracle.backproject(echo, scn.tx, scn.rx, scn.c, scn.fc, scn.fs, scn.t0, pts, scn.gate_half_angle)
    b = oracle.backproject(echo, scn.tx, scn.rx, scn.c, scn.fc, scn.fs, scn.t0, pts, scn.gate_half_angle,
                           rx_vel=np.zeros((scn.n_ping, 3)))
    # FP64 floor: the carrier argument is ~2e4 rad, the two delay formulas round differently
    assert np.linalg.norm(a - b) <= 1e-11 * np.linalg.norm(a)


def test_p12b_delay_solves_the_defining_equation():
    rng = np.random.default_rng(3)
    c = 1500.0
    for speed in (0.0, 0.3, 2.9, 20.0):
        a = rng.normal(size=(500, 3)) * rng.uniform(0.5, 80.0, size=(500, 1))
        d_T = np.linalg.norm(a + rng.normal(size=(500, 3)) * 0.2, axis=1)
        v = rng.normal(size=3)
        v *= speed / max(np.linalg.norm(v), 1e-300)
        tau = oracle.motion_delay(d_T, a, v, c)
        ref = _bisect_delay(d_T, a, v, c)
        assert np.max(np.abs(tau - ref) / ref) < 1e-13, speed
        resid = c * tau - d_T - np.linalg.norm(a - tau[:, None] * v[None, :], axis=1)
        assert np.max(np.abs(resid)) < 1e-10


def _lone_moving(pix, amp=0.7 - 0.4j):
    scn = make_config("c1", n_scat=1, snr_db=None, n_ping=12, n_elem=4, nx=32, ny=32)
    p = scn.grid.points(np.array([pix]))[0]
    scn.scat_pos = p[None, :].copy()
    scn.scat_amp = np.array([amp])
    vel = receiver_velocity(scn)
    echo = synthesize_echo(scn, noise=False, rx_vel=vel).numpy()
    return scn, p, vel, echo


def test_p12c_lone_scatterer_closed_form_with_motion():
    amp = 0.7 - 0.4j
    scn, p, vel, echo = _lone_moving(17 * 32 + 9, amp)
    got = oracle.backproject(echo, scn.tx, scn.rx, scn.c, scn.fc, scn.fs, scn.t0, p[None, :], rx_vel=vel)[0]
    d_T = np.sqrt(((scn.tx - p) ** 2).sum(-1))
    h = lambda d: pulse(np.asarray(d, dtype=np.float64), scn.bandwidth, scn.fs, scn.taper_half)
    G = []
    for i in range(scn.n_ping):
        tau = _bisect_delay(np.full(scn.n_elem, d_T[i]), p[None, :] - scn.rx[i], vel[i], scn.c)
        u = (tau - scn.t0) * scn.fs
        w = u - np.floor(u)
        G.append((1 - w) * h(w) + w * h(1 - w))
    G = np.concatenate(G)
    want = amp * G.sum()
    assert abs(got - want) <= 1e-10 * abs(want)
    assert abs(np.angle(got / amp)) < 1e-10
    # the receivers move by several centimetres: stop-and-hop loses the phase
    static = oracle.backproject(echo, scn.tx, scn.rx, scn.c, scn.fc, scn.fs, scn.t0, p[None, :])[0]
    assert abs(static) < 0.5 * abs(want) or abs(np.angle(static / amp)) > 0.3


MOTION_MUTATIONS = {
    "velocity_sign": ("Bh = c * d_T - av", "Bh = c * d_T + av"),
    "smaller_root": ("return (Bh + np.sqrt(", "return (Bh - np.sqrt("),
    "speed_term_dropped": ("A = c * c - vv", "A = c * c"),
}


@pytest.mark.parametrize("name", sorted(MOTION_MUTATIONS))
def test_p12_pins_reject_mutation(name):
    mod0 = importlib.import_module("oracle.tdbp")
    old, new = MOTION_MUTATIONS[name]
    src = inspect.getsource(mod0)
    assert src.count(old) == 1
    mod = types.ModuleType("tdbp_mutant")
    exec(compile(src.replace(old, new), "tdbp_mutant", "exec"), mod.__dict__)
    rng = np.random.default_rng(3)
    a = rng.normal(size=(200, 3)) * 30.0
    d_T = np.linalg.norm(a + 0.1, axis=1)
    v = np.array([2.9, 0.2, -0.1])
    ok = np.max(np.abs(mod.motion_delay(d_T, a, v, 1500.0) - _bisect_delay(d_T, a, v, 1500.0))) < 1e-15
    amp = 0.7 - 0.4j
    scn, p, vel, echo = _lone_moving(17 * 32 + 9, amp)
    got = mod.backproject(echo, scn.tx, scn.rx, scn.c, scn.fc, scn.fs, scn.t0, p[None, :], rx_vel=vel)[0]
    ok = ok and abs(np.angle(got / amp)) < 1e-10
    assert not ok, f"mutation {name} survived"


# ------------------------------------------------------------ position table
#
# P12d: with a table that samples a straight line, Delta(t) = v t, the table
#   delay (bisection) equals the closed-form root of the constant-velocity
#   quadratic (``motion_delay``, pinned by P12b).
# P12e: a lone scatterer whose echo is synthesized with a curved table (the
#   synthesis finds each delay by fixed-point iteration with its own
#   interpolation) images to the P2 closed form with zero residual phase; the
#   same echo imaged with the table shifted by one sample does not.
# P12f: the defining equation holds at the root, and the interpolation is
#   exact at the samples and linear between and past them.

def curved_track(scn, n_samp=40, h=2e-3, seed=5):
    return receiver_track(scn, n_samp, h, seed)


def test_p12d_straight_table_equals_constant_velocity_root():
    rng = np.random.default_rng(4)
    c = 1500.0
    for speed in (0.3, 2.9, 20.0):
        a = rng.normal(size=(400, 3)) * rng.uniform(0.5, 80.0, size=(400, 1))
        d_T = np.linalg.norm(a + rng.normal(size=(400, 3)) * 0.2, axis=1)
        v = rng.normal(size=3)
        v *= speed / np.linalg.norm(v)
        h = 1e-3
        table = np.arange(7)[:, None] * h * v[None, :]      # covers 6 ms; later delays use the extension
        got = oracle.track_delay(d_T, a, table, h, c)
        want = oracle.motion_delay(d_T, a, v, c)
        assert np.max(np.abs(got - want) / want) < 1e-13, speed


def test_p12f_interpolation_and_defining_equation():
    table = np.array([[0.0, 0.0, 0.0], [1.0, -2.0, 0.5], [1.5, -1.0, 0.5]])
    h = 0.5
    t = np.array([0.0, 0.5, 1.0, 0.25, 0.75, -0.5, 1.5])
    want = np.array([[0, 0, 0], [1, -2, 0.5], [1.5, -1, 0.5], [0.5, -1, 0.25], [1.25, -1.5, 0.5],
                     [-1, 2, -0.5], [2.0, 0.0, 0.5]])
    assert np.allclose(oracle.track_position(table, h, t), want, atol=1e-15)
    scn = make_config("c1", n_ping=2, n_elem=2)
    tab, hh = curved_track(scn)
    rng = np.random.default_rng(2)
    a = rng.normal(size=(200, 3)) * 30.0
    d_T = np.linalg.norm(a, axis=1) + rng.uniform(-0.5, 0.5, 200)
    tau = oracle.track_delay(d_T, a, tab[0], hh, 1500.0)
    resid = 1500.0 * tau - d_T - np.linalg.norm(a - oracle.track_position(tab[0], hh, tau), axis=1)
    assert np.max(np.abs(resid)) < 1e-10


def test_p12e_lone_scatterer_closed_form_with_a_table():
    amp = 0.6 + 0.5j
    scn = make_config("c1", n_scat=1, snr_db=None, n_ping=12, n_elem=4, nx=32, ny=32)
    p = scn.grid.points(np.array([11 * 32 + 20]))[0]
    scn.scat_pos = p[None, :].copy()
    scn.scat_amp = np.array([amp])
    tab, h = curved_track(scn)
    echo = synthesize_echo(scn, noise=False, rx_track=(tab, h)).numpy()
    got = oracle.backproject(echo, scn.tx, scn.rx, scn.c, scn.fc, scn.fs, scn.t0, p[None, :],
                             rx_track=(tab, h))[0]
    hfun = lambda d: pulse(np.asarray(d, dtype=np.float64), scn.bandwidth, scn.fs, scn.taper_half)
    want = 0.0
    for i in range(scn.n_ping):
        d_T = np.sqrt(((scn.tx[i] - p) ** 2).sum())
        for e in range(scn.n_elem):
            tau = oracle.track_delay(np.array([d_T]), (p - scn.rx[i, e])[None, :], tab[i], h, scn.c)[0]
            u = (tau - scn.t0) * scn.fs
            w = u - np.floor(u)
            want += (1 - w) * hfun(-w) + w * hfun(1 - w)
    want = amp * want
    assert abs(got - want) <= 1e-9 * abs(want)
    # the table shifted by one sample (a slip of the time origin) misses it
    shifted = np.concatenate([tab[:, 1:], 2 * tab[:, -1:] - tab[:, -2:-1]], axis=1)
    bad = oracle.backproject(echo, scn.tx, scn.rx, scn.c, scn.fc, scn.fs, scn.t0, p[None, :],
                             rx_track=(shifted, h))[0]
    assert abs(bad - want) > 1e-3 * abs(want)


TABLE_MUTATIONS = {
    "segment_off_by_one": ("j = np.clip(np.floor(t / h), 0, n - 2)", "j = np.clip(np.floor(t / h) + 1, 0, n - 2)"),
    "ends_clamped": ("frac = t / h - j ", "frac = np.clip(t / h - j, 0.0, 1.0) "),
    "slope_sign": ("return table[j] + frac[:, None] * (table[j + 1] - table[j])",
                   "return table[j] - frac[:, None] * (table[j + 1] - table[j])"),
    "bracket_direction": ("neg = f(mid) < 0.0", "neg = f(mid) > 0.0"),
}


@pytest.mark.parametrize("name", sorted(TABLE_MUTATIONS))
def test_p12_table_pins_reject_mutation(name):
    mod0 = importlib.import_module("oracle.tdbp")
    old, new = TABLE_MUTATIONS[name]
    src = inspect.getsource(mod0)
    assert src.count(old) == 1
    mod = types.ModuleType("tdbp_mutant")
    exec(compile(src.replace(old, new), "tdbp_mutant", "exec"), mod.__dict__)
    rng = np.random.default_rng(4)
    a = rng.normal(size=(200, 3)) * 30.0
    d_T = np.linalg.norm(a + 0.1, axis=1)
    v = np.array([2.9, 0.2, -0.1])
    h = 1e-3
    table = np.arange(7)[:, None] * h * v[None, :]
    ok = np.max(np.abs(mod.track_delay(d_T, a, table, h, 1500.0) - oracle.motion_delay(d_T, a, v, 1500.0))) < 1e-15
    amp = 0.6 + 0.5j
    scn = make_config("c1", n_scat=1, snr_db=None, n_ping=12, n_elem=4, nx=32, ny=32)
    p = scn.grid.points(np.array([11 * 32 + 20]))[0]
    scn.scat_pos = p[None, :].copy()
    scn.scat_amp = np.array([amp])
    tab, hh = curved_track(scn)
    echo = synthesize_echo(scn, noise=False, rx_track=(tab, hh)).numpy()
    got = mod.backproject(echo, scn.tx, scn.rx, scn.c, scn.fc, scn.fs, scn.t0, p[None, :], rx_track=(tab, hh))[0]
    ok = ok and abs(np.angle(got / amp)) < 1e-9
    assert not ok, f"mutation {name} survived"
