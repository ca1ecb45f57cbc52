"""Pins of the dynamic range compression oracle (Eqs. 11-12, Sec. II-E).

The defining property of Eq. 12 is that the median input pixel maps to the
requested brightness: the median of the output equals b. The map of Eq. 11
is monotone, fixes 0 and 1, and is the identity when the median already
equals b.
"""
import numpy as np
import pytest

import oracle


def _image(n=10001, seed=3):
    rng = np.random.default_rng(seed)
    # speckle-like magnitudes spanning ~80 dB, plus a few bright points
    mag = rng.rayleigh(1.0, n) * 10 ** rng.uniform(-2, 2, n)
    mag[:5] *= 1e4
    return mag * np.exp(1j * rng.uniform(0, 2 * np.pi, n))


@pytest.mark.parametrize("b,n", [(0.25, 10001), (0.5, 10000), (0.7, 777)])
def test_output_median_is_the_requested_brightness(b, n):
    out, prm = oracle.drc(_image(n), b)
    k = (out.size - 1) // 2
    assert abs(np.partition(out.ravel(), k)[k] - b) <= 1e-12
    assert prm["q"] > 0 and 0 < prm["median"] < 1


def test_map_is_monotone_and_fixes_the_ends():
    img = _image()
    out, _ = oracle.drc(img, 0.4)
    order = np.argsort(np.abs(img))
    assert np.all(np.diff(out[order]) >= -1e-15)
    assert out[np.argmax(np.abs(img))] == pytest.approx(1.0, abs=1e-15)
    z = img.copy()
    z[17] = 0.0
    out0, _ = oracle.drc(z, 0.4)
    assert out0[17] == 0.0


def test_identity_when_median_already_equals_brightness():
    img = _image(2001)
    _, prm = oracle.drc(img, 0.4)
    out, prm2 = oracle.drc(img, prm["median"])
    assert prm2["q"] == pytest.approx(1.0, rel=1e-12)
    assert np.allclose(out, np.abs(img) / np.abs(img).max(), rtol=0, atol=1e-12)


def test_degenerate_images():
    out, prm = oracle.drc(np.zeros(10, dtype=complex), 0.5)
    assert np.all(out == 0) and prm["q"] == 1.0
    img = np.zeros(11, dtype=complex)
    img[:4] = [1, 2, 3, 4]                   # median 0: every non-zero pixel to 1
    out, prm = oracle.drc(img, 0.5)
    assert prm["q"] == np.inf and out.tolist() == [1, 1, 1, 1] + [0] * 7


DRC_MUTATIONS = {
    "q_inverted": ("q = (b - b * med) / (med - b * med)", "q = (med - b * med) / (b - b * med)"),
    "map_denominator": ("out = q * x / ((q - 1.0) * x + 1.0)", "out = q * x / ((q + 1.0) * x + 1.0)"),
    "upper_median": ("k = (x.size - 1) // 2", "k = x.size // 2"),
}


@pytest.mark.parametrize("name", sorted(DRC_MUTATIONS))
def test_median_pin_rejects_mutation(name):
    import importlib
    import inspect
    import types
    mod0 = importlib.import_module("oracle.drc")   # the module (oracle.drc is also the function's name)
    old, new = DRC_MUTATIONS[name]
    src = inspect.getsource(mod0)
    assert src.count(old) == 1
    mod = types.ModuleType("drc_mutant")
    exec(compile(src.replace(old, new), "drc_mutant", "exec"), mod.__dict__)
    out, _ = mod.drc(_image(10000), 0.3)
    k = (out.size - 1) // 2
    assert abs(np.partition(out.ravel(), k)[k] - 0.3) > 1e-9, f"mutation {name} survived"
