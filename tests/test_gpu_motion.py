"""Continuous receiver motion during reception (desc.motion = 1) through the
C ABI against the FP64 oracle's exact delay root, on echoes synthesized with
the same motion. Bound: the FP32 image bound of the stop-and-hop path (1e-4
relative L2, 10 mrad over pixels within 30 dB of the peak).

Velocities: central differences of the navigated track over a ping
repetition interval of one record (2.9 m/s along-track on workload 1, with
the sway and heave rates of its random walk), so the receivers move by
several centimetres (several wavelengths) while a ping's echo arrives.
"""
import numpy as np
import pytest
import torch

import oracle
from synth import make_config, synthesize_echo, subset_indices, receiver_velocity
from tests.helpers import FP32_REL_L2, FP32_PHASE_MRAD, desc_for, buffers_for, gpu_image, oracle_image, report

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    import paper_2101_05888_amd as m
    return m


CASES = {
    "c1_ragged": ("c1", dict(n_ping=16, n_elem=4, nx=100, ny=77)),
    "c2_small": ("c2", dict(n_ping=64, n_elem=8, nx=333, ny=129, n_sample=4096, n_scat=40, n_speckle=400)),
    "c3_small": ("c3", dict(n_ping=16, n_across=4, nx=40, ny=24, nz=10, n_seabed=300, n_surface=8,
                            n_buried=4, n_sample=2048)),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_motion_image_matches_oracle(api, case):
    name, kw = CASES[case]
    print(f"case motion {case}", flush=True)
    scn = make_config(name, **kw)
    vel = receiver_velocity(scn)
    echo = synthesize_echo(scn, dtype=torch.complex64, rx_vel=vel)
    img, plan, _ = gpu_image(api, scn, echo, rx_vel=vel)
    ref = oracle_image(scn, echo.numpy(), rx_vel=vel).reshape(img.shape)
    r, ph = report(f"motion {case}", img, ref)
    assert r <= FP32_REL_L2 and ph <= FP32_PHASE_MRAD
    # the case exercises the motion: stop-and-hop imaging of the same echo is far off
    static = oracle_image(scn, echo.numpy()).reshape(img.shape)
    assert oracle.rel_l2(static, ref) > 0.1


def test_zero_velocity_equals_stop_and_hop(api):
    scn = make_config("c1", n_ping=16, n_elem=4, nx=100, ny=77)
    echo = synthesize_echo(scn, dtype=torch.complex64)
    img_m, _, _ = gpu_image(api, scn, echo, rx_vel=np.zeros((scn.n_ping, 3)))
    img_s, _, _ = gpu_image(api, scn, echo)
    r, ph = report("motion v=0 vs stop-and-hop", img_m, img_s)
    assert r <= 1e-5


def test_motion_plans_refuse_the_adjoint_and_bad_arguments(api):
    scn = make_config("c1", n_ping=8, n_elem=4, nx=64, ny=32)
    vel = receiver_velocity(scn)
    echo = synthesize_echo(scn, dtype=torch.complex64, rx_vel=vel)
    img, plan, buf = gpu_image(api, scn, echo, rx_vel=vel)
    f64 = dict(dtype=torch.float64, device="cuda")
    with pytest.raises(RuntimeError):
        api.sas_bp_adjoint(plan, [buf], [torch.zeros_like(buf.image)], [torch.zeros((scn.n_ping, 3), **f64)],
                           [torch.zeros((scn.n_ping, scn.n_elem, 3), **f64)], [torch.zeros(1, **f64)])
    with pytest.raises(RuntimeError):
        api.sas_bp_reproject(plan, [buf], [buf.image], [torch.zeros_like(buf.echo)])
    with pytest.raises(RuntimeError):   # windowed sinc with motion is not built
        api.sas_bp_plan([desc_for(api, scn, interp="sinc8", motion=True)])
    # a speed of c/2 or more is refused on the device like bad navigation
    fast = buffers_for(api, scn, echo, rx_vel=np.tile([900.0, 0.0, 0.0], (scn.n_ping, 1)))
    api.sas_bp_image(plan, [fast])
    torch.cuda.synchronize()
    assert plan.status() == 5
    assert np.isfinite(fast.image.cpu().numpy()).all()


def test_full_size_operational_swath_motion_sampled(api):
    """The operational swath (512 pings x 32 receivers, 4096 x 4096 pixels,
    +-10 deg gate) with the receivers moving at 1.46 m/s along-track during
    reception, in the launch configuration the benchmark times, on a seeded
    pixel subset."""
    print("case motion c2 full size", flush=True)
    scn = make_config("c2")
    vel = receiver_velocity(scn)
    echo = synthesize_echo(scn, device="cuda", dtype=torch.complex64, rx_vel=vel)
    plan = api.sas_bp_plan([desc_for(api, scn, motion=True)])
    buf = buffers_for(api, scn, echo, rx_vel=vel)
    api.sas_bp_image(plan, [buf])
    torch.cuda.synchronize()
    assert plan.status() == 0
    idx = subset_indices(scn, 1024)
    img = buf.image.reshape(-1)[torch.as_tensor(idx, device="cuda")].cpu().numpy()
    echo_np = echo.cpu().numpy()
    del echo, buf
    ref = oracle_image(scn, echo_np, idx, rx_vel=vel)
    r, ph = report("motion c2-full-subset", img, ref)
    assert r <= FP32_REL_L2 and ph <= FP32_PHASE_MRAD


# ------------------------------------------------------------ position table
#
# The receivers displaced along an up-sampled position table (samples every
# 2 ms, linear between them; sinusoidal sway and heave accelerations up to
# about 0.9 m/s^2 on a 1.5 m/s surge, zero at transmit), the echoes
# synthesized with the same table (fixed-point delays), the image against the
# oracle's bisection root. Same FP32 bounds. The kernel follows each ping's
# table on the straight line of the segment that holds the tile centre's
# delay, and certifies the departure below 2e-6 m (about 1 mrad of phase).

from tests.test_oracle_motion import curved_track


@pytest.mark.parametrize("case", sorted(CASES))
def test_table_motion_image_matches_oracle(api, case):
    name, kw = CASES[case]
    print(f"case table motion {case}", flush=True)
    scn = make_config(name, **kw)
    tab, h = curved_track(scn)
    echo = synthesize_echo(scn, dtype=torch.complex64, rx_track=(tab, h))
    img, plan, _ = gpu_image(api, scn, echo, rx_track=(tab, h))
    ref = oracle_image(scn, echo.numpy(), rx_track=(tab, h), chunk=512).reshape(img.shape)
    r, ph = report(f"table motion {case}", img, ref)
    assert r <= FP32_REL_L2 and ph <= FP32_PHASE_MRAD
    static = oracle_image(scn, echo.numpy()).reshape(img.shape)
    assert oracle.rel_l2(static, ref) > 0.1


def test_straight_table_equals_velocity_mode(api):
    # a table that samples R + v t exactly is the constant-velocity model
    scn = make_config("c2", n_ping=24, n_elem=8, nx=150, ny=70, n_sample=4096, n_scat=30, n_speckle=100)
    vel = receiver_velocity(scn)
    h = 1e-3
    n = 60
    tab = np.arange(n)[None, :, None] * h * vel[:, None, :]
    echo = synthesize_echo(scn, dtype=torch.complex64, rx_vel=vel)
    img_v, _, _ = gpu_image(api, scn, echo, rx_vel=vel)
    img_t, _, _ = gpu_image(api, scn, echo, rx_track=(tab, h))
    r, ph = report("straight table vs velocity", img_t, img_v)
    assert r <= 1e-5


def test_table_with_velocity_jumps_is_refused(api):
    # velocity changes of 0.5 m/s between 1 ms segments depart from any one
    # segment's line by far more than the certified 2e-6 m inside a tile
    scn = make_config("c1", n_ping=6, n_elem=4, nx=64, ny=32)
    h = 1e-3
    n = 60
    rng = np.random.default_rng(1)
    vel = np.cumsum(rng.choice([-0.5, 0.5], size=(scn.n_ping, n, 3)), axis=1)
    tab = np.concatenate([np.zeros((scn.n_ping, 1, 3)), np.cumsum(vel[:, :-1] * h, axis=1)], axis=1)
    echo = synthesize_echo(scn, dtype=torch.complex64)
    plan = api.sas_bp_plan([desc_for(api, scn, motion="table", track=(n, h))])
    buf = buffers_for(api, scn, echo, rx_track=tab)
    api.sas_bp_image(plan, [buf])
    torch.cuda.synchronize()
    assert plan.status() == 5
    # a table that is not finite is refused the same way
    bad = tab.copy()
    bad[2, 5, 1] = np.nan
    plan2 = api.sas_bp_plan([desc_for(api, scn, motion="table", track=(n, h))])
    buf2 = buffers_for(api, scn, echo, rx_track=bad)
    api.sas_bp_image(plan2, [buf2])
    torch.cuda.synchronize()
    assert plan2.status() == 5
    with pytest.raises(RuntimeError):   # a table of one sample
        api.sas_bp_plan([desc_for(api, scn, motion="table", track=(1, h))])
    with pytest.raises(ValueError):     # a table of the wrong shape
        api.sas_bp_image(plan, [buffers_for(api, scn, echo, rx_track=tab[:, :-1])])


def test_full_size_operational_swath_table_sampled(api):
    """The operational swath in the benchmark's launch configuration with the
    receivers on a position table (2 ms samples over the 205 ms record), on a
    seeded pixel subset."""
    print("case table motion c2 full size", flush=True)
    scn = make_config("c2")
    tab, h = curved_track(scn, n_samp=110)
    echo = synthesize_echo(scn, device="cuda", dtype=torch.complex64, rx_track=(tab, h))
    plan = api.sas_bp_plan([desc_for(api, scn, motion="table", track=(tab.shape[1], h))])
    buf = buffers_for(api, scn, echo, rx_track=tab)
    api.sas_bp_image(plan, [buf])
    torch.cuda.synchronize()
    assert plan.status() == 0
    idx = subset_indices(scn, 512)
    img = buf.image.reshape(-1)[torch.as_tensor(idx, device="cuda")].cpu().numpy()
    echo_np = echo.cpu().numpy()
    del echo, buf
    ref = oracle_image(scn, echo_np, idx, rx_track=(tab, h), chunk=32)
    r, ph = report("table motion c2-full-subset", img, ref)
    assert r <= FP32_REL_L2 and ph <= FP32_PHASE_MRAD
