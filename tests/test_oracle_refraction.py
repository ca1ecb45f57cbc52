"""Pins of the sediment-refraction variant of the oracle (Sec. III-B: a
sediment-water interface refraction model in the propagation time).

* Equal sound speeds give straight paths (the stop-and-hop oracle's image).
* The crossing point obeys Snell's law, sin(theta_1) / c = sin(theta_2) / c_sed.
* Fermat: no point of a fine two-dimensional grid on the interface (off the
  vertical plane too) gives a shorter time; the grid's best is within its
  resolution.
* Pixels at or above the interface take straight paths.
* A buried scatterer whose echo is synthesized with refraction (golden-section
  search in the synthesis, an independent route) images with zero phase to
  a sum G(w), w from the synthesis-side travel times; straight-path imaging
  of that echo does not.
"""
import importlib
import inspect
import types

import numpy as np
import pytest
import torch

import oracle
from synth import make_config, synthesize_echo
from synth.echo import pulse, _leg_time

C, CS, ZI = 1500.0, 1650.0, 5.5


def test_equal_speeds_are_straight_and_above_interface_is_straight():
    rng = np.random.default_rng(1)
    X = np.array([0.3, -0.2, 0.1])
    p = np.column_stack([rng.uniform(-2, 2, 200), rng.uniform(-2, 2, 200), rng.uniform(4.0, 7.0, 200)])
    straight = np.linalg.norm(p - X, axis=1) / C
    assert np.allclose(oracle.refracted_leg(X, p, C, C, ZI), straight, rtol=1e-14, atol=0)
    t = oracle.refracted_leg(X, p, C, CS, ZI)
    above = p[:, 2] <= ZI
    assert np.array_equal(t[above], straight[above])
    assert np.all(t[~above] < straight[~above])        # sound is faster in the sediment


def test_snell_and_fermat():
    X = np.array([0.0, 0.0, 0.2])
    pts = np.array([[1.1, 0.4, 6.3], [0.0, 0.0, 6.0], [2.5, -1.5, 5.6]])
    t = oracle.refracted_leg(X, pts, C, CS, ZI)
    for p, tp in zip(pts, t):
        D = np.hypot(*(p[:2] - X[:2]))
        h1, h2 = ZI - X[2], p[2] - ZI
        # recover the crossing distance from the time by a fine 1D scan, then check Snell there
        r = np.linspace(0, D, 200001)
        tt = np.sqrt(r * r + h1 * h1) / C + np.sqrt((D - r) ** 2 + h2 * h2) / CS
        k = np.argmin(tt)
        assert abs(tt[k] - tp) < 1e-12
        if D > 0:
            s1 = r[k] / np.hypot(r[k], h1)
            s2 = (D - r[k]) / np.hypot(D - r[k], h2)
            assert abs(s1 / C - s2 / CS) < 1e-4 / C        # scan resolution D / 2e5
        # Fermat over a 2D grid of interface points around the vertical plane
        gx, gy = np.meshgrid(np.linspace(-1, 3, 401), np.linspace(-2, 1, 301))
        q = np.column_stack([gx.ravel(), gy.ravel(), np.full(gx.size, ZI)])
        tq = np.linalg.norm(q - X, axis=1) / C + np.linalg.norm(q - p, axis=1) / CS
        assert tq.min() >= tp - 1e-15
        assert tq.min() - tp < 1e-7


def test_buried_scatterer_focuses_with_refraction():
    scn = make_config("c3", n_ping=12, n_across=4, nx=24, ny=20, nz=12, n_seabed=0, n_surface=0, n_buried=0,
                      n_sample=2048, snr_db=None)
    pix = 5 + 24 * (7 + 20 * 9)                   # z index 9: 5.18 m ... use a deeper voxel below
    p = scn.grid.points(np.array([pix]))[0]
    p = p + np.array([0.0, 0.0, 0.7])            # 0.88 m below the seafloor
    scn.scat_pos = p[None, :].copy()
    amp = 0.6 + 0.3j
    scn.scat_amp = np.array([amp])
    refr = (CS, ZI)
    echo = synthesize_echo(scn, noise=False, refraction=refr).numpy()
    got = oracle.backproject(echo, scn.tx, scn.rx, scn.c, scn.fc, scn.fs, scn.t0, p[None, :], refraction=refr)[0]
    tT = _leg_time(torch.as_tensor(scn.tx), torch.as_tensor(p)[None, :], scn.c, refr).numpy()      # [P]
    tR = _leg_time(torch.as_tensor(scn.rx), torch.as_tensor(p)[None, None, :], scn.c, refr).numpy()  # [P, E]
    u = (tT[:, None] + tR - scn.t0) * scn.fs
    w = u - np.floor(u)
    h = lambda d: pulse(np.asarray(d, dtype=np.float64), scn.bandwidth, scn.fs, scn.taper_half)
    G = (1 - w) * h(w) + w * h(1 - w)
    want = amp * G.sum()
    assert abs(got - want) <= 1e-9 * abs(want)
    assert abs(np.angle(got / amp)) < 1e-9
    straight = oracle.backproject(echo, scn.tx, scn.rx, scn.c, scn.fc, scn.fs, scn.t0, p[None, :])[0]
    assert abs(straight) < 0.5 * abs(want)


MUTATIONS = {
    "speeds_swapped": ("f = r / (c * np.sqrt(r * r + h1 * h1)) - (D - r) / (c_sed * np.sqrt((D - r) ** 2 + h2c * h2c))",
                       "f = r / (c_sed * np.sqrt(r * r + h1 * h1)) - (D - r) / (c * np.sqrt((D - r) ** 2 + h2c * h2c))"),
    "bracket_direction": ("lo = np.where(f < 0, r, lo)\n        hi = np.where(f < 0, hi, r)",
                          "lo = np.where(f > 0, r, lo)\n        hi = np.where(f > 0, hi, r)"),
    "straight_in_sediment": ("return np.where(below, t, np.sqrt(((pts - X) ** 2).sum(axis=1)) / c)",
                             "return np.sqrt(((pts - X) ** 2).sum(axis=1)) / c"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_reject_mutation(name):
    mod0 = importlib.import_module("oracle.tdbp")
    old, new = MUTATIONS[name]
    src = inspect.getsource(mod0)
    assert src.count(old) == 1
    mod = types.ModuleType("tdbp_mutant")
    exec(compile(src.replace(old, new), "tdbp_mutant", "exec"), mod.__dict__)
    saved = oracle.refracted_leg
    import oracle.tdbp as ot
    saved_t = ot.refracted_leg
    try:
        oracle.refracted_leg = mod.refracted_leg
        ot.refracted_leg = mod.refracted_leg
        failed = False
        for fn in (test_equal_speeds_are_straight_and_above_interface_is_straight, test_snell_and_fermat):
            try:
                fn()
            except AssertionError:
                failed = True
        assert failed, f"mutation {name} survived"
    finally:
        oracle.refracted_leg = saved
        ot.refracted_leg = saved_t
