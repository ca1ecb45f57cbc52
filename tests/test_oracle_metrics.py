"""Pins of the error metrics every parity verdict goes through.

rel-L2 and the maximum phase error are checked on hand-computed cases:
a pixel exactly at the -30 dB amplitude floor counts and one just below it
does not, the floor is an amplitude (20 log10) floor and not a power one,
the norm is taken of the reference, and the phase is selected on the
reference's magnitude. Planted slips in private copies of the metrics module
(on the CPU) are each rejected.
"""
import inspect
import math
import types

import numpy as np
import pytest

import oracle.metrics as metrics


def test_rel_l2_hand_computed():
    img = np.array([1 + 1j, 2, 0])
    ref = np.array([1, 2, 1])
    # |img - ref| = |(1j, 0, -1)| = sqrt(2); |ref| = sqrt(6)
    assert metrics.rel_l2(img, ref) == pytest.approx(math.sqrt(2.0 / 6.0), rel=1e-15)
    # the norm is the reference's: swapping the arguments changes the value
    # (|img| = sqrt(6) as well here, so use a second case)
    a = np.array([3.0, 0.0])
    b = np.array([1.0, 0.0])
    assert metrics.rel_l2(a, b) == pytest.approx(2.0, rel=1e-15)
    assert metrics.rel_l2(b, a) == pytest.approx(2.0 / 3.0, rel=1e-15)
    # shapes are flattened; scaling both by a complex factor leaves it unchanged
    z = (0.3 - 2j)
    r2 = np.arange(12, dtype=complex).reshape(3, 4) * (1 + 0.5j)
    i2 = r2 + 0.01 * np.exp(1j * np.arange(12)).reshape(3, 4)
    assert metrics.rel_l2(z * i2, z * r2) == pytest.approx(metrics.rel_l2(i2, r2), rel=1e-12)
    assert metrics.rel_l2(i2.ravel(), r2.ravel()) == metrics.rel_l2(i2, r2)
    # identical images: zero; a zero reference: the norm of the image
    assert metrics.rel_l2(r2, r2) == 0.0
    assert metrics.rel_l2(np.array([3j, 4.0]), np.zeros(2)) == pytest.approx(5.0)


def _floor_case():
    """Reference: a peak of 1, one pixel exactly at -30 dB in amplitude
    (10^(-30/20)), one just below it, one above the -30 dB *power* floor
    (10^(-30/10) = 1e-3) but below the amplitude floor. Image phases are off
    by 0.5 rad at the floor pixel, 2.0 rad below it and 3.0 rad at the third."""
    f = 10.0 ** (-30.0 / 20.0)
    mag = np.array([1.0, f, f * (1.0 - 1e-9), 2e-3])
    err = np.array([0.1, 0.5, 2.0, 3.0])
    ref = mag.astype(complex)             # real references: |ref| is exactly mag
    img = mag * np.exp(1j * err)
    return img, ref


def test_phase_error_floor_hand_computed():
    img, ref = _floor_case()
    assert metrics.phase_error_mrad(img, ref) == pytest.approx(500.0, rel=1e-12)
    # a 0 dB floor keeps the peak alone
    assert metrics.phase_error_mrad(img, ref, floor_db=0.0) == pytest.approx(100.0, rel=1e-12)
    # a 60 dB floor takes all four pixels
    assert metrics.phase_error_mrad(img, ref, floor_db=60.0) == pytest.approx(3000.0, rel=1e-12)
    # wrapped differences: 2 pi + 0.25 rad counts as 0.25
    r = np.array([1.0 + 0j])
    assert metrics.phase_error_mrad(r * np.exp(1j * (2 * math.pi + 0.25)), r) == pytest.approx(250.0, rel=1e-9)
    # the selection uses the reference's magnitude: a large image value at a
    # reference null is not counted
    ref2 = np.array([1.0, 1e-6 + 0j])
    img2 = np.array([1.0, 5.0j])
    assert metrics.phase_error_mrad(img2, ref2) == 0.0
    # p99 over the selected pixels: 100 pixels with errors 0..99 mrad
    e = np.arange(100) * 1e-3
    assert metrics.phase_error_mrad(np.exp(1j * e), np.ones(100), stat="p99") == pytest.approx(
        np.percentile(np.arange(100.0), 99), rel=1e-9)
    assert metrics.phase_error_mrad(np.zeros(3), np.zeros(3)) == 0.0


SLIPS = {
    "power_floor": ("10.0 ** (-floor_db / 20.0)", "10.0 ** (-floor_db / 10.0)"),
    "strict_floor": ("sel = mag >= mag.max()", "sel = mag > mag.max()"),
    "norm_of_image": ("den = np.linalg.norm(b)", "den = np.linalg.norm(a)"),
    "select_on_image": ("mag = np.abs(b)", "mag = np.abs(a)"),
    "unsquared_norm_ratio": ("np.linalg.norm(a - b) / den", "np.linalg.norm(a - b) ** 2 / den ** 2"),
}


def _mutant(old, new):
    src = inspect.getsource(metrics)
    assert src.count(old) >= 1, old
    mod = types.ModuleType("metrics_mutant")
    exec(compile(src.replace(old, new), "metrics_mutant", "exec"), mod.__dict__)
    return mod


def _pins_hold(mod) -> bool:
    try:
        img, ref = _floor_case()
        assert mod.phase_error_mrad(img, ref) == pytest.approx(500.0, rel=1e-12)
        assert mod.rel_l2(np.array([1 + 1j, 2, 0]), np.array([1, 2, 1])) == pytest.approx(math.sqrt(1 / 3), rel=1e-15)
        assert mod.rel_l2(np.array([3.0, 0.0]), np.array([1.0, 0.0])) == pytest.approx(2.0, rel=1e-15)
        assert mod.phase_error_mrad(np.array([1.0, 5.0j]), np.array([1.0, 1e-6 + 0j])) == 0.0
    except AssertionError:
        return False
    return True


def test_unmutated_copy_passes():
    assert _pins_hold(_mutant("import numpy as np", "import numpy as np"))


@pytest.mark.parametrize("name", sorted(SLIPS))
def test_pins_reject_slip(name):
    assert not _pins_hold(_mutant(*SLIPS[name])), f"slip {name} survived the metric pins"
