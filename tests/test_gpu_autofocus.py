"""Sharpness autofocus on the differentiable workload (256 pings x 16
receivers, 4096 samples, 1024 x 1024 px at 1.5 cm; echoes synthesized on a
track with a smooth 1 cm RMS sway/heave error the imager does not know).

The workload's target is a detrended RMS position error below lambda/16 =
0.94 mm in both y and z (a constant offset or linear trend of the track only
moves or tilts the image, so it is removed before comparing). It is checked
as stated and is not met: see ``test_autofocus_meets_lambda_over_16_in_y_and_z``.
What is met: the error along the line of sight, which sets the ranges and so
the focus, falls below lambda/16; y and z both shrink; and the estimate is at
least as sharp as the truth moved by the estimate's own trend (the optimiser
reached the objective's maximum, not a wrapped neighbour). Convergence has no
closed form to pin it: these are seeded empirical results.
"""
import numpy as np
import pytest
import torch

from synth import make_config, synthesize_echo
from tests.helpers import desc_for

pytestmark = pytest.mark.gpu

LAMBDA = 1500.0 / 100e3


@pytest.fixture(scope="module")
def run():
    import paper_2101_05888_amd as api
    from paper_2101_05888_amd.autofocus import autofocus, default_stages, detrended_rms, line_of_sight_frame
    print("case c5 autofocus", flush=True)
    scn = make_config("c5")
    g = scn.grid
    echo = synthesize_echo(scn, device="cuda", dtype=torch.complex64, noise_on_device=True)
    plan = api.sas_bp_plan([desc_for(api, scn)])
    tx0 = torch.as_tensor(scn.tx, device="cuda")
    rx0 = torch.as_tensor(scn.rx, device="cuda")
    buf = api.SwathBuffers(echo=echo, tx=tx0.clone(), rx=rx0.clone(),
                           c=torch.tensor([scn.c], dtype=torch.float64, device="cuda"),
                           image=torch.empty((1, g.n[1], g.n[0]), dtype=torch.complex64, device="cuda"))
    truth = scn.true_tx - scn.tx
    centre = [g.origin[0] + 0.5 * (g.n[0] - 1) * g.spacing[0], g.origin[1] + 0.5 * (g.n[1] - 1) * g.spacing[1], 0.0]
    R = line_of_sight_frame(scn.tx, centre)
    res = autofocus(default_stages(plan, buf), tx0, rx0, truth=truth, frame=R)
    err = res.offsets - truth

    def sharp(off):
        o = torch.as_tensor(off, device="cuda")
        buf.tx.copy_(tx0 + o)
        buf.rx.copy_(rx0 + o[:, None, :])
        S = torch.zeros(1, dtype=torch.float64, device="cuda")
        api.sas_bp_image(plan, [buf])
        api.sas_bp_sharpness(plan, buf.image, S)
        return float(S.item())

    n = truth.shape[0]
    A = np.stack([np.ones(n), np.arange(n, dtype=np.float64)], axis=1)
    trend = A @ np.linalg.lstsq(A, err, rcond=None)[0]
    out = dict(
        los0=detrended_rms((truth @ R[1])[:, None])[0], los=detrended_rms((err @ R[1])[:, None])[0],
        yz0=detrended_rms(truth[:, 1:]), yz=detrended_rms(err[:, 1:]),
        S_nom=sharp(np.zeros_like(truth)), S_est=sharp(res.offsets), S_truth=sharp(truth + trend))
    print(f"[autofocus] S {out['S_nom']:.3e} -> {out['S_est']:.3e} (trend-aligned truth {out['S_truth']:.3e}); "
          f"line-of-sight error {out['los0'] * 1e3:.2f} -> {out['los'] * 1e3:.3f} mm; "
          f"y {out['yz0'][0] * 1e3:.2f} -> {out['yz'][0] * 1e3:.2f} mm, "
          f"z {out['yz0'][1] * 1e3:.2f} -> {out['yz'][1] * 1e3:.2f} mm", flush=True)
    return out


def test_autofocus_reaches_lambda_over_16_along_line_of_sight(run):
    assert run["los"] < LAMBDA / 16
    assert run["yz"][0] < 0.5 * run["yz0"][0] and run["yz"][1] < 0.5 * run["yz0"][1]
    assert run["S_est"] >= run["S_truth"] * (1.0 - 1e-3)


@pytest.mark.xfail(strict=False, reason=(
    "not met: the image plane is seen from look angles 16 to 27 deg, so an offset perpendicular to the "
    "line of sight changes ranges about 18x less than one along it; with the line-of-sight error at "
    "0.14 mm, z stays near 2.7 mm (y 0.8 mm), and the estimate is already sharper than the trend-aligned truth"))
def test_autofocus_meets_lambda_over_16_in_y_and_z(run):
    assert run["yz"][0] < LAMBDA / 16 and run["yz"][1] < LAMBDA / 16
