"""Pins of the spectral whitening oracle (Eq. 9, Sec. II-E).

With gamma = 0 the gain is min P^ / P^(f), so the whitened cube's average
power spectrum is flat, equal to min P^ at every bin: the purpose of the
correction. A cube whose average spectrum is already flat is returned
unchanged for any gamma. The smallest attenuation is 0 dB (max G = 1), and
the gain is the closed form h(1 / (gamma mean P^ + P^)).
"""
import importlib
import inspect
import types

import numpy as np
import pytest

import oracle


def _coloured(P=12, E=5, Ns=256, seed=2):
    rng = np.random.default_rng(seed)
    w = rng.normal(size=(P, E, Ns)) + 1j * rng.normal(size=(P, E, Ns))
    shape = 0.2 + np.exp(-((np.fft.fftfreq(Ns) - 0.1) / 0.15) ** 2)   # a non-flat system response
    return np.fft.ifft(np.fft.fft(w, axis=-1) * shape, axis=-1)


def _avg_spectrum(e):
    return (np.abs(np.fft.fft(e, axis=-1)) ** 2).reshape(-1, e.shape[-1]).mean(axis=0)


def test_gamma_zero_flattens_the_average_spectrum():
    e = _coloured()
    out, Phat, G = oracle.whiten(e, 0.0)
    S = _avg_spectrum(out)
    assert np.allclose(S, Phat.min(), rtol=1e-10, atol=0)
    assert G.max() == 1.0


def test_gain_closed_form_and_flat_input_unchanged():
    e = _coloured()
    out, Phat, G = oracle.whiten(e, 0.7)
    g = 1.0 / (0.7 * Phat.mean() + Phat)
    assert np.allclose(G, g / g.max(), rtol=1e-14, atol=0)
    assert np.allclose(_avg_spectrum(out), Phat * G, rtol=1e-10, atol=0)
    # a single impulse per row has a flat spectrum: nothing to whiten
    imp = np.zeros((3, 2, 64), dtype=complex)
    imp[:, :, 5] = 1.0 + 0.5j
    out2, _, G2 = oracle.whiten(imp, 0.3)
    assert np.allclose(G2, 1.0) and np.allclose(out2, imp, atol=1e-14)


WHITEN_MUTATIONS = {
    "amplitude_gain_not_root": ("X * np.sqrt(G)[None, None, :]", "X * G[None, None, :]"),
    "normalised_by_min": ("G = G / G.max()", "G = G / G.min()"),
    "mean_over_rows_only": ("Phat = (np.abs(X) ** 2).reshape(-1, e.shape[-1]).mean(axis=0)",
                            "Phat = np.abs(X[0, 0]) ** 2"),
}


@pytest.mark.parametrize("name", sorted(WHITEN_MUTATIONS))
def test_pins_reject_mutation(name):
    mod0 = importlib.import_module("oracle.whiten")
    old, new = WHITEN_MUTATIONS[name]
    src = inspect.getsource(mod0)
    assert src.count(old) == 1
    mod = types.ModuleType("whiten_mutant")
    exec(compile(src.replace(old, new), "whiten_mutant", "exec"), mod.__dict__)
    e = _coloured()
    out, Phat, G = mod.whiten(e, 0.0)
    S = _avg_spectrum(out)
    ok = np.allclose(S, S.min(), rtol=1e-10, atol=0) and np.isclose(G.max(), 1.0) \
        and np.allclose(S, _avg_spectrum(e).min(), rtol=1e-10, atol=0)
    assert not ok, f"mutation {name} survived"
