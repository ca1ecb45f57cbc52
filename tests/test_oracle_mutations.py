"""The oracle's pins must reject plausible mistakes.

Each case plants one slip in a private copy of the oracle's source (on the
CPU, never in the HIP path) and checks that the brute-force pin (P1) rejects
the mutated backprojection, or that the adjoint identity against the
unmutated backprojection (P10) rejects the mutated reprojection.
"""
import inspect
import math
import types

import numpy as np
import pytest

import oracle.tdbp as tdbp
from tests.test_oracle_pins import _brute_mp, _tiny_geometry

MUTATIONS = {
    "phase_sign": ("np.exp(1j * 2.0 * np.pi * fc * tau)", "np.exp(-1j * 2.0 * np.pi * fc * tau)"),
    "dropped_tx_leg": ("tau = (dT + dR) / c", "tau = (2.0 * dR) / c"),
    "tap_off_by_one": ("b[ib] = row[n[ib] + 1]", "b[ib] = row[n[ib]]"),
    "swapped_weights": ("L = (1.0 - w) * a + w * b", "L = w * a + (1.0 - w) * b"),
    "gate_wrong_axis": ("g = gT & _gate(pts[:, 0] - R[0], dR, sin_g)", "g = gT & _gate(pts[:, 1] - R[1], dR, sin_g)"),
    "rx_transposed": ("R = rx[i, e]\n            dR", "R = rx[e % rx.shape[0], i % rx.shape[1]]\n            dR"),
    "t0_sign": ("u = (tau - t0) * fs", "u = (tau + t0) * fs"),
    "tx_gate_dropped": ("g = gT & _gate", "g = _gate"),
}


def _mutant(old, new):
    src = inspect.getsource(tdbp)
    assert src.count(old) >= 1, old
    mod = types.ModuleType("oracle_mutant")
    exec(compile(src.replace(old, new), "oracle_mutant", "exec"), mod.__dict__)
    return mod


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_reject_mutation(name):
    old, new = MUTATIONS[name]
    mod = _mutant(old, new)
    rejected = False
    for gate_deg, ns, t0 in [(12.0, 36, 1.5e-3), (12.0, 48, 4.95e-3)]:
        g = _tiny_geometry(gate_deg=gate_deg, ns=ns, t0=t0, P=4, E=3)
        pts = g["grid"].points()
        ref = _brute_mp(g, pts)
        got = mod.backproject(g["echo"], g["tx"], g["rx"], g["c"], g["fc"], g["fs"], g["t0"], pts, g["gate"])
        if np.linalg.norm(got - ref) > 1e-12 * np.linalg.norm(ref):
            rejected = True
            break
    assert rejected, f"mutation {name} survived the brute-force pin"


def test_unmutated_copy_passes():
    mod = _mutant("import math", "import math")
    g = _tiny_geometry(gate_deg=12.0, ns=36, P=4, E=3)
    pts = g["grid"].points()
    got = mod.backproject(g["echo"], g["tx"], g["rx"], g["c"], g["fc"], g["fs"], g["t0"], pts, g["gate"])
    assert np.linalg.norm(got - _brute_mp(g, pts)) <= 1e-12 * np.linalg.norm(got)


REPROJECT_MUTATIONS = {
    "phase_not_conjugated": ("v = np.exp(-1j * 2.0 * np.pi * fc * tau) * ybar",
                             "v = np.exp(1j * 2.0 * np.pi * fc * tau) * ybar"),
    "weights_swapped": ("np.add.at(row, n[lo], (1.0 - w[lo]) * v[lo])", "np.add.at(row, n[lo], w[lo] * v[lo])"),
    "upper_tap_off_by_one": ("np.add.at(row, n[hi] + 1, w[hi] * v[hi])", "np.add.at(row, n[hi], w[hi] * v[hi])"),
    "gate_ignored": ("v = np.where(gT & _gate(pts[:, 0] - R[0], dR, sin_g), v, 0.0)", "v = v"),
    "cotangent_conjugated": ("* ybar\n", "* np.conj(ybar)\n"),
}


@pytest.mark.parametrize("name", sorted(REPROJECT_MUTATIONS))
def test_adjoint_identity_rejects_reprojection_mutation(name):
    old, new = REPROJECT_MUTATIONS[name]
    mod = _mutant(old, new)
    g = _tiny_geometry(gate_deg=12.0, ns=48, t0=4.95e-3, P=4, E=3)
    pts = g["grid"].points()
    rng = np.random.default_rng(11)
    x = rng.normal(size=g["echo"].shape) + 1j * rng.normal(size=g["echo"].shape)
    y = rng.normal(size=pts.shape[0]) + 1j * rng.normal(size=pts.shape[0])
    ax = tdbp.backproject(x, g["tx"], g["rx"], g["c"], g["fc"], g["fs"], g["t0"], pts, g["gate"])
    ahy = mod.reproject(y, g["tx"], g["rx"], g["c"], g["fc"], g["fs"], g["t0"], pts, x.shape[2], g["gate"])
    lhs, rhs = np.vdot(ax, y), np.vdot(x.ravel(), ahy.ravel())
    assert abs(lhs - rhs) > 1e-9 * abs(lhs), f"mutation {name} survived the adjoint identity"


SINC_MUTATIONS = {
    "taps_shifted_by_one": ("m = n - half + 1 + j", "m = n - half + j"),
    "window_too_wide": ("np.cos(np.pi * t / half)", "np.cos(np.pi * t / (2 * half))"),
    "sinc_without_pi": ("np.sinc(t) * 0.5", "np.sinc(t / np.pi) * 0.5"),
}


@pytest.mark.parametrize("name", sorted(SINC_MUTATIONS))
def test_brute_force_rejects_sinc_variant_mutation(name):
    from tests.test_oracle_pins import _brute_mp_sinc
    old, new = SINC_MUTATIONS[name]
    mod = _mutant(old, new)
    g = _tiny_geometry(gate_deg=12.0, ns=48, P=3, E=2)
    pts = g["grid"].points()[::2]
    got = mod.backproject(g["echo"], g["tx"], g["rx"], g["c"], g["fc"], g["fs"], g["t0"], pts, g["gate"],
                          interp="sinc")
    ref = _brute_mp_sinc(g, pts)
    assert np.linalg.norm(got - ref) > 1e-9 * np.linalg.norm(ref), f"mutation {name} survived"
