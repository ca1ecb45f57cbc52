"""Input generator checks: pulse shape, seeding, noise level, quantisation."""
import math

import numpy as np
import pytest
import torch

from synth import make_config, synthesize_echo, quantize_echo, dequantize_echo, subset_indices
from synth.echo import pulse


def test_pulse_is_unit_sinc_with_flat_top():
    B, fs, H = 20e3, 80e3, 64
    d = np.array([0.0, 4.0, 8.0, -12.0, 0.37])
    h = pulse(d, B, fs, H)
    assert h[0] == 1.0
    assert np.allclose(h[1:4], 0.0, atol=1e-15)           # nulls every f_s/B = 4 samples
    assert h[4] == pytest.approx(np.sinc(0.37 / 4.0), rel=1e-15)  # flat top: exact sinc
    assert pulse(np.array([64.0, 70.0]), B, fs, H).tolist() == [0.0, 0.0]


def test_scenario_layout_c1():
    scn = make_config("c1")
    assert scn.tx.shape == (64, 3) and scn.rx.shape == (64, 8, 3)
    gr = scn.grid
    assert gr.n == (256, 256, 1)
    assert gr.origin[1] == 20.0 and gr.axis(1)[-1] == pytest.approx(23.825)
    assert 0.5 * (gr.axis(0)[0] + gr.axis(0)[-1]) == pytest.approx(4.725)
    # receivers on a line along x about the transmitter, 3.75 cm pitch
    d = scn.rx[:, :, 0] - scn.tx[:, None, 0]
    assert np.allclose(np.diff(d, axis=1), 0.0375)
    assert np.allclose(d.mean(axis=1), 0.0)
    assert abs(scn.tx[:, 2].mean() + 10.0) < 0.1


def test_seeds_are_reproducible():
    a = make_config("c2", n_ping=8, n_elem=4, nx=64, ny=64, n_scat=5, n_speckle=7)
    b = make_config("c2", n_ping=8, n_elem=4, nx=64, ny=64, n_scat=5, n_speckle=7)
    assert np.array_equal(a.tx, b.tx) and np.array_equal(a.scat_pos, b.scat_pos)
    assert np.array_equal(a.scat_amp, b.scat_amp)
    ea = synthesize_echo(a)
    eb = synthesize_echo(b)
    assert torch.equal(ea, eb)
    assert np.array_equal(subset_indices(a, 100), subset_indices(b, 100))


def test_noise_level_matches_snr():
    scn = make_config("c1", n_ping=8, n_elem=4, nx=64, ny=64)
    clean = synthesize_echo(scn, noise=False)
    noisy = synthesize_echo(scn, noise=True)
    p_sig = float((clean.abs() ** 2).mean())
    p_noise = float(((noisy - clean).abs() ** 2).mean())
    assert p_noise == pytest.approx(p_sig / 100.0, rel=0.02)


@pytest.mark.parametrize("kind,u", [("f16", 2.0 ** -11), ("bf16", 2.0 ** -8)])
def test_quantiser_round_trip(kind, u):
    scn = make_config("c1", n_ping=6, n_elem=4, nx=32, ny=32)
    e = synthesize_echo(scn)
    q, scale = quantize_echo(e, kind)
    assert q.shape == (6, 4, scn.n_sample, 2) and scale.shape == (6,)
    assert torch.isfinite(q.float()).all()
    d = dequantize_echo(q, scale)
    er = torch.view_as_real(e)
    peak = er.abs().reshape(6, -1).amax(1)
    err = (torch.view_as_real(d) - er).abs().reshape(6, -1).amax(1)
    assert bool((err <= peak * u * 1.0001).all())        # at most half an ulp of the ping's peak
    if kind == "f16":
        assert float(q.float().abs().max()) <= 2.0 ** 15


def test_gate_applied_in_synthesis():
    scn = make_config("c2", n_ping=24, n_elem=2, nx=32, ny=32, n_scat=1, n_speckle=0, snr_db=None)
    scn.scat_pos = np.array([[scn.tx[0, 0] + 30.0, 40.0, 0.0]])   # far outside every ping's +-10 deg cone
    scn.scat_amp = np.array([1.0 + 0j])
    assert float(synthesize_echo(scn).abs().max()) == 0.0
