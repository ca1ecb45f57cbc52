"""Pins of the time-delay estimation oracle (DPC motion estimate, Sec. II-D).

Test signals are real Gaussian pulse trains a(t) = sum_s alpha_s
exp(-((t - c_s) / sigma)^2) (alpha_s real) and their copy delayed by delta
and brought to baseband, b(t) = a(t - delta) exp(-j 2 pi f_c delta): the
form two pings' returns from one patch take. Then r(l) = exp(j 2 pi f_c
delta) R(l - delta f_s) with R real, so

* the phase at the interpolated peak is exactly 2 pi f_c delta (mod 2 pi):
  it fixes which operand is conjugated and the lag direction;
* a whole-sample delay gives mu = 0 (R is even), a fractional one a coarse
  delay within 0.02 samples (quadratic fit of a Gaussian peak);
* the fine delay recovers delta to rounding once unwrapped around the coarse one;
* b = a gives rho = 1; rho <= 1 always (Cauchy-Schwarz);
* the quadratic step is exact on a parabola; coherent pairs add.
"""
import importlib
import inspect
import math
import types

import numpy as np
import pytest

import oracle
from oracle import dpc

FS, FC = 80e3, 100e3


def _pulses(n, centres, amps, shift=0.0, sigma=2.5):
    t = np.arange(n, dtype=np.float64)
    out = np.zeros(n)
    for c, a in zip(centres, amps):
        out += a * np.exp(-((t - c - shift) / sigma) ** 2)
    return out


WIN = 128   # windows do not overlap (hop = WIN) and every pulse lies 30 samples inside one


def _pair_cube(delta_samples, Ns=512, J=2, seed=0):
    rng = np.random.default_rng(seed)
    P, E = 2, 2 * J
    echo = np.zeros((P, E, Ns), dtype=np.complex128)
    pairs = []
    for j in range(J):
        cs = (np.arange(Ns // WIN)[:, None] * WIN + rng.uniform(30, WIN - 30, size=(Ns // WIN, 3))).ravel()
        am = rng.uniform(0.5, 1.5, size=cs.size)
        a = _pulses(Ns, cs, am)
        b = _pulses(Ns, cs, am, shift=delta_samples) * np.exp(-2j * np.pi * FC * delta_samples / FS)
        echo[0, j] = a
        echo[1, J + j] = b
        pairs.append((j, J + j))
    return echo, np.array(pairs)


@pytest.mark.parametrize("delta", [0.0, 3.0, -5.0, 2.37, -0.61, 7.5])
def test_delay_phase_and_fine_delay_of_a_delayed_copy(delta):
    echo, pairs = _pair_cube(delta)
    d, ph, rho, lag = dpc.tde(echo, pairs, win=WIN, hop=WIN, max_lag=12, fs=FS)
    want_ph = math.remainder(2 * math.pi * FC * delta / FS, 2 * math.pi)
    ok = rho[0] > 0.5                      # windows with signal
    assert ok.sum() == 4
    err_ph = np.abs(np.angle(np.exp(1j * (ph[0, ok] - want_ph))))
    assert err_ph.max() < 1e-9
    err = np.abs(d[0, ok] * FS - delta)
    if delta == round(delta):
        assert err.max() < 1e-9            # R is even: mu = 0
        assert np.all(lag[0, ok] == int(delta))
    else:
        assert err.max() < 0.02
    fine = dpc.fine_delay(ph[0, ok], d[0, ok], FC)
    assert np.abs(fine - delta / FS).max() < 1e-15


def test_identical_looks_have_unit_correlation_and_rho_bounded():
    echo, pairs = _pair_cube(0.0)
    echo[1, 2:] = echo[0, :2]
    d, ph, rho, lag = dpc.tde(echo, pairs, win=WIN, hop=WIN, max_lag=12, fs=FS)
    sig = np.abs(echo[0, 0]).max() > 0
    assert sig and np.allclose(rho[0], 1.0, atol=1e-12) and np.all(lag[0] == 0)
    rng = np.random.default_rng(1)
    noise = rng.normal(size=echo.shape) + 1j * rng.normal(size=echo.shape)
    _, _, rho2, _ = dpc.tde(noise, pairs, win=WIN, hop=WIN, max_lag=12, fs=FS)
    assert np.all((rho2 >= 0) & (rho2 <= 1 + 1e-12))


def test_quadratic_step_is_exact_on_a_parabola_and_pairs_add():
    L = 6
    vertex = 1.3
    lags = np.arange(-L, L + 1)
    m = 10.0 - 0.1 * (lags - vertex) ** 2
    r = m * np.exp(0.4j)
    lc, rc, rho, l0 = dpc.peak(r.astype(np.complex128), 1.0, np.ones(2 * L + 1))
    assert abs(lc - vertex) < 1e-12 and l0 == 1
    assert abs(np.angle(rc) - 0.4) < 1e-12 and abs(abs(rc) - 10.0) < 1e-12
    # two pairs carrying the same delayed look estimate the same delay
    e1, p1 = _pair_cube(2.37, J=1, seed=4)
    e2 = np.concatenate([e1, e1], axis=1)
    p2 = np.array([(0, 1), (2, 3)])
    a = dpc.tde(e1, p1, WIN, WIN, 12, FS)
    b = dpc.tde(e2, p2, WIN, WIN, 12, FS)
    assert np.allclose(a[0], b[0], rtol=0, atol=1e-15) and np.allclose(a[2], b[2], atol=1e-12)


DPC_MUTATIONS = {
    "conjugate_on_a": ("r[li] = np.sum(a * np.conj(bs))", "r[li] = np.sum(np.conj(a) * bs)"),
    "lag_direction": ("idx = np.arange(W) + l + lags", "idx = np.arange(W) - l + lags"),
    "mu_sign": ("mu = 0.0 if den == 0.0 else (m_ - mp) / (2.0 * den)",
                "mu = 0.0 if den == 0.0 else (mp - m_) / (2.0 * den)"),
    "rho_unnormalised": ("d = math.sqrt(ea * eb[ic])", "d = ea * eb[ic]"),
}


@pytest.mark.parametrize("name", sorted(DPC_MUTATIONS))
def test_pins_reject_mutation(name):
    mod0 = importlib.import_module("oracle.dpc")
    old, new = DPC_MUTATIONS[name]
    src = inspect.getsource(mod0)
    assert src.count(old) == 1
    mod = types.ModuleType("dpc_mutant")
    exec(compile(src.replace(old, new), "dpc_mutant", "exec"), mod.__dict__)
    ok = True
    for delta in (2.37, -5.0):
        echo, pairs = _pair_cube(delta)
        d, ph, rho, lag = mod.tde(echo, pairs, win=WIN, hop=WIN, max_lag=12, fs=FS)
        sig = rho[0] > 0.5
        want_ph = math.remainder(2 * math.pi * FC * delta / FS, 2 * math.pi)
        if sig.sum() != 4:
            ok = False
            continue
        ok &= bool(np.abs(np.angle(np.exp(1j * (ph[0, sig] - want_ph)))).max() < 1e-9)
        ok &= bool(np.abs(d[0, sig] * FS - delta).max() < 0.02)
    echo, pairs = _pair_cube(0.0)
    echo[1, 2:] = echo[0, :2]
    _, _, rho, _ = mod.tde(echo, pairs, win=WIN, hop=WIN, max_lag=12, fs=FS)
    ok &= bool(np.allclose(rho[0], 1.0, atol=1e-12))
    assert not ok, f"mutation {name} survived"
