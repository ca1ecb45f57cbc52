"""Pins of the time-varying gain oracle (Eq. 10, Sec. II-E).

With alpha = 0 the gain is the reciprocal median power, so after the gain the
median power of every sample time is exactly one: the defining property of
the correction. With alpha > 0 the corrected median power is
P~ / (alpha mean P~ + P~), below one and increasing with P~. For Rayleigh
amplitudes of scale s(t) the median power is 2 ln 2 s(t)^2 (the closed form
of the exponential distribution's median), which the estimate approaches.
"""
import importlib
import inspect
import types

import numpy as np
import pytest

import oracle


def _echo(P=24, E=9, Ns=300, seed=5):
    rng = np.random.default_rng(seed)
    s = np.exp(-np.linspace(0, 4, Ns))                      # spreading and absorption loss
    amp = rng.rayleigh(1.0, (P, E, Ns)) * s
    return amp * np.exp(1j * rng.uniform(0, 2 * np.pi, (P, E, Ns))), s


def _median_power(e):
    p = (np.abs(e) ** 2).reshape(-1, e.shape[2])
    k = (p.shape[0] - 1) // 2
    return np.partition(p, k, axis=0)[k]


def test_alpha_zero_flattens_the_median_power():
    e, _ = _echo()
    out, med, G = oracle.tvg(e, 0.0)
    assert np.allclose(_median_power(out), 1.0, rtol=1e-12, atol=0)


def test_alpha_positive_closed_form():
    e, _ = _echo()
    out, med, G = oracle.tvg(e, 0.5)
    want = med / (0.5 * med.mean() + med)
    assert np.allclose(_median_power(out), want, rtol=1e-12, atol=0)
    assert np.all(np.diff(want[np.argsort(med)]) >= -1e-15)


def test_median_power_tracks_the_rayleigh_closed_form():
    e, s = _echo(P=200, E=25, Ns=50)
    _, med, _ = oracle.tvg(e, 0.0)
    ratio = med / (2.0 * np.log(2.0) * s ** 2)
    assert np.all(np.abs(ratio - 1.0) < 0.15)             # 5000 samples per median
    assert abs(np.median(ratio) - 1.0) < 0.03


def test_zero_column_is_left_unchanged():
    e, _ = _echo()
    e[:, :, 7] = 0.0
    out, med, G = oracle.tvg(e, 0.0)
    assert med[7] == 0.0 and not np.isfinite(G[7]) and np.all(out[:, :, 7] == 0.0)


TVG_MUTATIONS = {
    "amplitude_not_root": ("return e * amp[None, None, :], med, G", "return e * amp[None, None, :] ** 2, med, G"),
    "upper_median": ("k = (P * E - 1) // 2", "k = (P * E) // 2"),
    "mean_of_power": ("G = 1.0 / (alpha * med.mean() + med)", "G = 1.0 / (alpha * power.mean() + med)"),
}


@pytest.mark.parametrize("name", sorted(TVG_MUTATIONS))
def test_pins_reject_mutation(name):
    mod0 = importlib.import_module("oracle.tvg")
    old, new = TVG_MUTATIONS[name]
    src = inspect.getsource(mod0)
    assert src.count(old) == 1
    mod = types.ModuleType("tvg_mutant")
    exec(compile(src.replace(old, new), "tvg_mutant", "exec"), mod.__dict__)
    e, _ = _echo(P=10, E=5)                                   # even population: the two medians differ
    rejected = False
    for a in (0.0, 0.5):
        out, med, G = mod.tvg(e, a)
        mp = _median_power(e)
        want = mp / (a * mp.mean() + mp)
        if not np.allclose(_median_power(out), want, rtol=1e-9, atol=0):
            rejected = True
    assert rejected, f"mutation {name} survived"
