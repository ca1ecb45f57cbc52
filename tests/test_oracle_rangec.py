"""Pins of the range-compression oracle (matched filter with Eq. 1's
waveform q, plus basebanding).

* A delayed linear-FM replica compresses to a closed form: the lag products
  q[m - l] conj(q[m]) of a quadratic-phase pulse form a geometric series in
  m, summed here in closed form over the overlap (the record end included),
  so the conjugated operand, the index direction, the normalisation and the
  zero extension are all fixed.
* A tone at f_c + delta with a one-tap replica basebands to the tone at
  delta: the sign and the time origin of the carrier mix.
* A raw point-scatterer echo compresses to exactly a exp(-j 2 pi f_c tau) at
  its delay (the baseband form the backprojection reads).
* Linearity and time-shift covariance away from the record end.
"""
import importlib
import inspect
import types

import numpy as np
import pytest

import oracle
from synth.waveform import lfm_replica, raw_echo

FC, FS, T0 = 100e3, 80e3, 0.0123457     # f_c t0 is not a whole number of cycles


def _lfm_closed_form(n, d, M, Ns, K, fs):
    """(1/M) sum_m q[n + m - d] conj(q[m]) for q[m] = exp(j pi K (m/fs - T/2)^2), by the geometric series."""
    T = M / fs
    lag = d - n                    # q[m - lag] conj(q[m])
    a = max(0, lag)
    b = min(M - 1, M - 1 + lag, Ns - 1 - n)
    if b < a:
        return 0.0
    h = lag / fs
    # (m/fs - h - T/2)^2 - (m/fs - T/2)^2 = h^2 - 2 h (m/fs - T/2)
    pre = np.exp(1j * np.pi * K * (h * h + 2 * h * T / 2))
    r = np.exp(-2j * np.pi * K * h / fs)
    cnt = b - a + 1
    s = cnt if abs(r - 1) < 1e-15 else r ** a * (1 - r ** cnt) / (1 - r)
    return pre * s / M


def test_lfm_compresses_to_the_geometric_closed_form():
    B, Tp = 20e3, 2.5e-3
    q = lfm_replica(B, Tp, FS)
    M = q.shape[0]
    K = B / (M / FS)
    Ns = 700
    for d in (0, 37, 450, Ns - M // 3):      # the last one runs off the record end
        x = np.zeros((1, 1, Ns), dtype=complex)
        k1 = min(Ns, d + M)
        x[0, 0, d:k1] = q[:k1 - d]
        y = oracle.range_compress(x, q, FC, FS, T0, mix=False)[0, 0]
        want = np.array([_lfm_closed_form(n, d, M, Ns, K, FS) for n in range(Ns)])
        assert np.max(np.abs(y - want)) < 1e-12, d
        if d + M <= Ns:
            assert abs(y[d] - 1.0) < 1e-13


def test_carrier_mix_sign_and_time_origin():
    Ns, delta, A = 333, 1.7e3, 0.3 - 1.1j
    t = T0 + np.arange(Ns) / FS
    x = (A * np.exp(2j * np.pi * (FC + delta) * t)).reshape(1, 1, Ns)
    y = oracle.range_compress(x, np.array([1.0 + 0j]), FC, FS, T0, mix=True)[0, 0]
    assert np.max(np.abs(y - A * np.exp(2j * np.pi * delta * t))) < 1e-10


def test_point_scatterer_compresses_to_baseband_peak():
    q = lfm_replica(20e3, 2e-3, FS)
    x, d, a = raw_echo(3, 600, q, FC, FS, T0, n_targets=1, seed=4)
    y = oracle.range_compress(x, q, FC, FS, T0, mix=True)
    for r in range(3):
        k = int(d[r, 0])
        tau = T0 + k / FS
        want = a[r, 0] * np.exp(-2j * np.pi * FC * tau)
        if k + q.shape[0] <= 600:
            assert abs(y[r, k] - want) < 1e-12
        assert int(np.argmax(np.abs(y[r]))) == k


def test_linear_and_shift_covariant():
    rng = np.random.default_rng(9)
    q = lfm_replica(20e3, 1e-3, FS)
    Ns, s = 400, 23
    x1 = rng.normal(size=(2, 1, Ns)) + 1j * rng.normal(size=(2, 1, Ns))
    x2 = rng.normal(size=(2, 1, Ns)) + 1j * rng.normal(size=(2, 1, Ns))
    y1 = oracle.range_compress(x1, q, FC, FS, T0, mix=False)
    y2 = oracle.range_compress(x2, q, FC, FS, T0, mix=False)
    y12 = oracle.range_compress(2.0 * x1 - 1j * x2, q, FC, FS, T0, mix=False)
    assert np.allclose(y12, 2.0 * y1 - 1j * y2, rtol=0, atol=1e-12)
    xs = np.zeros_like(x1)
    xs[..., s:] = x1[..., :-s]
    ys = oracle.range_compress(xs, q, FC, FS, T0, mix=False)
    lim = Ns - s - q.shape[0]       # outputs whose window stays inside the shifted record
    assert np.allclose(ys[..., s:s + lim], y1[..., :lim], rtol=0, atol=1e-12)


RANGEC_MUTATIONS = {
    "convolution_not_correlation": ('np.correlate(padded, q, mode="valid")',
                                    'np.convolve(padded, q, mode="valid")'),
    "conjugate_on_echo": ('np.correlate(padded, q, mode="valid")',
                          'np.correlate(np.conj(padded), np.conj(q), mode="valid")'),
    "mix_sign": ("np.exp(-2j * np.pi * f_c * t)", "np.exp(2j * np.pi * f_c * t)"),
    "mix_time_origin": ("t = t0 + np.arange", "t = np.arange"),
    "amplitude_normalised": ("energy = np.sum(np.abs(q) ** 2)", "energy = np.sqrt(np.sum(np.abs(q) ** 2))"),
}


def _pins_hold(mod) -> bool:
    q = lfm_replica(20e3, 2.5e-3, FS)
    M = q.shape[0]
    K = 20e3 / (M / FS)
    Ns, d = 700, 37
    x = np.zeros((1, 1, Ns), dtype=complex)
    x[0, 0, d:d + M] = q
    y = mod.range_compress(x, q, FC, FS, T0, mix=False)[0, 0]
    want = np.array([_lfm_closed_form(n, d, M, Ns, K, FS) for n in range(Ns)])
    if np.max(np.abs(y - want)) > 1e-12:
        return False
    t = T0 + np.arange(333) / FS
    xt = (np.exp(2j * np.pi * (FC + 1.7e3) * t)).reshape(1, 1, 333)
    yt = mod.range_compress(xt, np.array([1.0 + 0j]), FC, FS, T0, mix=True)[0, 0]
    return np.max(np.abs(yt - np.exp(2j * np.pi * 1.7e3 * t))) < 1e-10


@pytest.mark.parametrize("name", sorted(RANGEC_MUTATIONS))
def test_pins_reject_mutation(name):
    mod0 = importlib.import_module("oracle.rangec")
    assert _pins_hold(mod0)
    old, new = RANGEC_MUTATIONS[name]
    src = inspect.getsource(mod0)
    assert src.count(old) == 1
    mod = types.ModuleType("rangec_mutant")
    exec(compile(src.replace(old, new), "rangec_mutant", "exec"), mod.__dict__)
    assert not _pins_hold(mod), f"mutation {name} survived"
