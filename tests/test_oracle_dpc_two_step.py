"""The two-step DPC motion estimate of Sec. II-D in the oracle, end to end, on
echoes synthesized along a known track (``synth.dpc_track``: smooth sway and
heave velocities, receivers moving during reception, 16 pings of the
operational array geometry over a speckle seafloor, 20 dB SNR).

Steps, as the paper orders them: time-delay estimation between consecutive
pings; a first Levenberg-Marquardt solve on the coarse delays; the correlation
phase unwrapped around the delay that first solution predicts; a second solve
on the unwrapped fine delays.

Pins, from the generator's truth rather than the oracle itself:

* the phase unwrapped around the first solution takes the same cycle count as
  the phase unwrapped around the true track, on every weighted window (the
  first solution is within half a carrier cycle, which is the point of the
  first step);
* the fine residuals at the true track are about ten times smaller than the
  coarse ones (the fine delay carries the carrier phase);
* the second solve puts every ping within lambda / 16 of the true track in y
  and z, and at least three times closer than the first solve.

Element pairs: e + 16 of ping i with e of ping i + 1 for e = 6..9, the pairs
whose transmitter-to-receiver offsets are nearly equal in length. Pairs are
summed coherently, and a pair whose two offsets differ by d1^2 - d2^2 carries
a bistatic path offset near (d1^2 - d2^2) / (4 R); over all sixteen pairs that
spreads their phases by several radians at 15 m and cancels most of the sum
(rho near 0.2 instead of 0.9).
"""
import math

import numpy as np
import pytest
import torch

from oracle import dpc
from synth import dpc_track, synthesize_echo

PAIRS = np.array([(e + 16, e) for e in range(6, 10)], dtype=np.int32)
WIN, HOP, LAG = 128, 64, 16
SIGMA_COARSE, SIGMA_FINE = 1e-6, 3e-8     # s: Huber thresholds of the two solves
LAM_SMOOTH, LAM_DVL = 1e4, 1.0
RHO_MIN = 0.5
LAMBDA = 1500.0 / 100e3


def problem(track, n_window):
    """Everything the two solves share: known surge, lever arms, window times,
    footprints from the straight nominal track, DVL depths of the true track."""
    scn = track.scn
    P = scn.n_ping
    vx = track.vel[:, 0].copy()
    lever_rx = np.asarray(scn.rx[0] - scn.tx[0], dtype=np.float64)
    t_ref = scn.t0 + (np.arange(n_window) * HOP + WIN / 2) / scn.fs
    nominal = np.column_stack([vx, np.zeros(P), np.zeros(P)])
    ps = dpc.footprints(track.p0, nominal, track.dt, np.zeros(3), lever_rx, PAIRS, t_ref, scn.c, 0.0)
    z_dvl = np.asarray(scn.true_tx[:, 2], dtype=np.float64)
    return dict(vx=vx, p0=track.p0, dt=track.dt, lever_tx=np.zeros(3), lever_rx=lever_rx, pairs=PAIRS,
                t_ref=t_ref, ps=ps, c=scn.c, z_dvl=z_dvl), nominal


def model_delay(kw, vyz):
    """The delay a motion solution predicts for every window: -g at zero measured delay."""
    args = {k: kw[k] for k in ("vx", "p0", "dt", "lever_tx", "lever_rx", "pairs", "t_ref", "ps", "c")}
    return -dpc.residuals(vyz, delay=np.zeros((kw["ps"].shape[0], kw["ps"].shape[1])), **args)


def positions(kw, vyz):
    return dpc.platform_positions(kw["p0"], np.column_stack([kw["vx"], vyz]), kw["dt"])


def oracle_two_step(track, echo):
    scn = track.scn
    d, ph, rho, _ = dpc.tde(np.asarray(echo).astype(np.complex64).astype(np.complex128), PAIRS, WIN, HOP, LAG,
                            scn.fs)
    kw, _ = problem(track, d.shape[1])
    w = np.where(rho > RHO_MIN, rho, 0.0)
    P = scn.n_ping
    v1, _ = dpc.solve(np.zeros((P, 2)), delay=d, weights=w, sigma=SIGMA_COARSE, lam1=LAM_SMOOTH, lam2=LAM_DVL,
                      robust=True, iters=40, **kw)
    fine = dpc.fine_delay(ph, model_delay(kw, v1), scn.fc)
    v2, _ = dpc.solve(v1, delay=fine, weights=w, sigma=SIGMA_FINE, lam1=LAM_SMOOTH, lam2=LAM_DVL, robust=True,
                      iters=40, **kw)
    return dict(kw=kw, delay=d, phase=ph, rho=rho, weight=w, v1=v1, fine=fine, v2=v2)


@pytest.fixture(scope="module")
def run():
    track = dpc_track()
    echo = synthesize_echo(track.scn, dtype=torch.complex64, rx_vel=track.vel).numpy()
    return track, oracle_two_step(track, echo)


def test_unwrap_around_first_solution_matches_truth(run):
    track, r = run
    kw = r["kw"]
    truth = track.vel[:, 1:]
    fc = track.scn.fc
    m_first = np.round(fc * model_delay(kw, r["v1"]) - r["phase"] / (2 * math.pi))
    m_truth = np.round(fc * model_delay(kw, truth) - r["phase"] / (2 * math.pi))
    sel = r["weight"] > 0
    assert sel.sum() >= 0.4 * sel.size
    assert np.array_equal(m_first[sel], m_truth[sel])


def test_fine_delays_fit_the_true_track_better(run):
    track, r = run
    kw = r["kw"]
    w = r["weight"]
    args = {k: kw[k] for k in ("vx", "p0", "dt", "lever_tx", "lever_rx", "pairs", "t_ref", "ps", "c")}
    g_c = dpc.residuals(track.vel[:, 1:], delay=r["delay"], **args)
    g_f = dpc.residuals(track.vel[:, 1:], delay=r["fine"], **args)
    rms_c = math.sqrt(np.sum(w * g_c ** 2) / w.sum())
    rms_f = math.sqrt(np.sum(w * g_f ** 2) / w.sum())
    print(f"[dpc two-step oracle] residual rms at the true track: coarse {rms_c:.3e} s, fine {rms_f:.3e} s")
    assert rms_f < 0.2 * rms_c


def test_second_solve_reaches_lambda_over_16(run):
    track, r = run
    kw = r["kw"]
    true_pos = np.asarray(track.scn.true_tx)
    e1 = np.abs(positions(kw, r["v1"]) - true_pos).max(axis=0)
    e2 = np.abs(positions(kw, r["v2"]) - true_pos).max(axis=0)
    print(f"[dpc two-step oracle] max position error y/z: coarse {e1[1] * 1e3:.3f}/{e1[2] * 1e3:.3f} mm, "
          f"fine {e2[1] * 1e3:.3f}/{e2[2] * 1e3:.3f} mm")
    assert e2[1] < LAMBDA / 16 and e2[2] < LAMBDA / 16
    assert 3.0 * e2[1] < e1[1] and 3.0 * e2[2] < e1[2]
