"""The motion estimate (Eqs. 3-8) through the C ABI against the oracle: the
Eq. 4 residuals and their derivatives on the GPU (against the oracle's
residuals and its central differences), and the Levenberg-Marquardt solve,
checked as a minimiser of the oracle's loss (Eq. 8), not as a copy of the
oracle's iteration.

Bounds: residuals within 1e-14 s (FP64 path differences); derivatives within
1e-6 relative to their largest entry (central differences with a 1e-6 m/s
step carry about that). The solve: its loss, evaluated by the oracle, at most
1e-9 above the oracle solve's, and the oracle loss's gradient at the GPU
solution below 1e-3 of the data term's (the two cancel at a minimiser).
"""
import numpy as np
import pytest

from oracle import dpc
from tests.test_oracle_dpc_motion import STATIONARY, _noisy_problem, _problem, loss_gradients

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    import paper_2101_05888_amd as m
    return m


def _desc(api, kw, P, K, robust=False):
    return api.dpc_desc(P, K, len(kw["pairs"]), kw["lever_rx"].shape[0], kw["c"], kw["sigma"], kw["lam1"],
                        kw["lam2"], kw["p0"], kw["lever_tx"], robust, 60)


@pytest.mark.parametrize("P,K", [(10, 6), (24, 12)])
def test_residuals_and_derivatives_match_oracle(api, P, K):
    kw, true = _problem(P=P, K=K)
    v = true + 0.01 * np.random.default_rng(5).normal(size=true.shape)
    vel = np.column_stack([kw["vx"], v])
    d = _desc(api, kw, P, K)
    pos, rows = api.sas_bp_dpc_residual(d, vel, kw["dt"], kw["lever_rx"], kw["pairs"], kw["t_ref"], kw["ps"],
                                        kw["delay"])
    rows = rows.cpu().numpy()
    args = (kw["vx"], kw["p0"], kw["dt"], kw["lever_tx"], kw["lever_rx"], kw["pairs"], kw["t_ref"], kw["ps"],
            kw["delay"], kw["c"])
    g = dpc.residuals(v, *args)
    assert np.abs(rows[..., 0] - g).max() < 1e-14
    assert np.abs(pos.cpu().numpy() - dpc.platform_positions(kw["p0"], vel, kw["dt"])).max() < 1e-12
    # assembled analytic derivatives vs central differences of the oracle's residuals
    h = 1e-6
    num = np.zeros(g.shape + (P, 2))
    for n in range(P):
        for c in range(2):
            vp, vm = v.copy(), v.copy()
            vp[n, c] += h
            vm[n, c] -= h
            num[..., n, c] = (dpc.residuals(vp, *args) - dpc.residuals(vm, *args)) / (2 * h)
    ana = np.zeros_like(num)
    for i in range(P - 1):
        for n in range(i):
            ana[i, :, n, :] = kw["dt"][n] * rows[i, :, 1:3]
        ana[i, :, i, :] = rows[i, :, 3:5]
        ana[i, :, i + 1, :] = rows[i, :, 5:7]
    err = np.abs(ana - num).max() / np.abs(num).max()
    print(f"[dpc residual P={P} K={K}] max|dg| {np.abs(rows[..., 0] - g).max():.2e} s, derivative rel {err:.2e}",
          flush=True)
    assert err < 1e-6


@pytest.mark.parametrize("robust", [False, True])
def test_solve_reaches_the_minimum(api, robust):
    kw, true = _noisy_problem(robust)
    P, K = true.shape[0], kw["t_ref"].size
    d = _desc(api, kw, P, K, robust)
    v, loss = api.sas_bp_dpc_solve(d, kw["vx"], kw["dt"], kw["lever_rx"], kw["pairs"], kw["t_ref"], kw["ps"],
                                   kw["delay"], kw["weights"], kw["z_dvl"], np.zeros_like(true))
    lg = dpc.loss(v, robust=robust, **kw)
    vo, lo = dpc.solve(np.zeros_like(true), robust=robust, iters=60, **kw)
    g, gd = loss_gradients(kw, v, robust)
    ratio = np.abs(g).max() / np.abs(gd).max()
    print(f"[dpc solve robust={robust}] loss {lg:.9e} (native {loss:.9e}) vs oracle solve {lo:.9e}, "
          f"|grad L| / |grad data| {ratio:.2e}, |v - oracle| {np.abs(v - vo).max():.2e} m/s", flush=True)
    assert abs(loss - lg) <= 1e-9 * abs(lg)
    assert lg <= lo * (1.0 + 1e-9)
    assert ratio <= STATIONARY


def test_solve_recovers_a_longer_track(api):
    kw, true = _problem(P=64, K=16, seed=3)
    kw["lam1"] = 1e-8
    P, K = true.shape[0], kw["t_ref"].size
    d = _desc(api, kw, P, K)
    v, loss = api.sas_bp_dpc_solve(d, kw["vx"], kw["dt"], kw["lever_rx"], kw["pairs"], kw["t_ref"], kw["ps"],
                                   kw["delay"], kw["weights"], kw["z_dvl"], np.zeros_like(true))
    print(f"[dpc solve P=64] |v - true| {np.abs(v - true).max():.2e} m/s", flush=True)
    assert np.abs(v - true).max() < 1e-6
