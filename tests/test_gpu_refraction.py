"""Sediment-water interface refraction (desc.refract = 1) through the C ABI
against the oracle, on echoes synthesized with the same interface (the
synthesis finds each crossing by golden-section search, the oracle by
bisection on Snell's law, the kernel by bracketed Newton steps). Bound: the
FP32 image bound (1e-4 relative L2, 10 mrad over pixels within 30 dB of the
peak).

The near-field volume (array at the surface, seabed at 5.5 m, sand at
1650 m/s): voxels from 5.0 m, buried scatterers to 1 m below the seabed.
"""
import numpy as np
import pytest
import torch

import oracle
from synth import make_config, synthesize_echo, subset_indices
from tests.helpers import (FP32_REL_L2, FP32_PHASE_MRAD, desc_for, buffers_for, gpu_image, oracle_image, report,
                           volume_subset)

pytestmark = pytest.mark.gpu

REFR = (1650.0, 5.5)


@pytest.fixture(scope="module")
def api():
    import paper_2101_05888_amd as m
    return m


def _scene(**kw):
    # voxels from 5.3 m to 5.88 m: across the seabed at 5.5 m
    base = dict(n_ping=16, n_across=4, nx=40, ny=24, nz=30, z0=5.3, n_seabed=300, n_surface=8, n_buried=12,
                n_sample=2048)
    base.update(kw)
    return make_config("c3", **base)


@pytest.mark.parametrize("c_sed", [1650.0, 1450.0])
def test_refraction_image_matches_oracle(api, c_sed):
    # sand (faster than water: a critical crossing bounds the bracket) and
    # mud (slower: no critical crossing)
    print(f"case refraction c3 small c_sed {c_sed}", flush=True)
    refr = (c_sed, REFR[1])
    scn = _scene()
    echo = synthesize_echo(scn, dtype=torch.complex64, refraction=refr)
    img, plan, _ = gpu_image(api, scn, echo, refraction=refr)
    ref = oracle_image(scn, echo.numpy(), refraction=refr).reshape(img.shape)
    r, ph = report(f"refraction c3 small c_sed {c_sed}", img, ref)
    assert r <= FP32_REL_L2 and ph <= FP32_PHASE_MRAD
    # the case exercises the interface: straight-path imaging of this echo is far off
    straight = oracle_image(scn, echo.numpy()).reshape(img.shape)
    assert oracle.rel_l2(straight, ref) > 0.1


@pytest.mark.parametrize("offset", [1e-5, 1e-4])
def test_voxels_just_below_the_interface_beyond_the_critical_distance(api, offset):
    # a voxel plane 1e-5 or 1e-4 m below a shallow interface (0.96 m under the
    # array, sand at 1650 m/s: the critical crossing is 2.09 m out), pings up
    # to 4 m away along the track: the sediment legs of that plane are almost
    # horizontal and their crossing lies just inside the critical distance
    print(f"case refraction near interface offset {offset}", flush=True)
    scn = _scene(n_ping=80, nz=6, z0=0.9, seabed_z=0.96, n_seabed=200, n_surface=10, n_buried=6, bury_max=0.05)
    refr = (1650.0, 0.96 - offset)
    echo = synthesize_echo(scn, dtype=torch.complex64, refraction=refr)
    img, plan, _ = gpu_image(api, scn, echo, refraction=refr)   # also asserts a clean status (every leg converged)
    ref = oracle_image(scn, echo.numpy(), refraction=refr).reshape(img.shape)
    r, ph = report(f"refraction near interface {offset}", img, ref)
    plane = ref[3]
    r3 = oracle.rel_l2(img[3], plane)
    print(f"  the plane below the interface: rel_l2 {r3:.3e}", flush=True)
    assert r <= FP32_REL_L2 and ph <= FP32_PHASE_MRAD
    assert r3 <= FP32_REL_L2


def test_more_receivers_than_one_reference_chunk(api):
    # 80 receivers (2 x 40) and 3D tiles of four voxel levels: a ping's
    # references span two chunks (the transmitter and 64 elements at four
    # levels fill one), so the transmitter leg's offsets carry over into the
    # second and each reference slot starts its crossing from another element
    print("case refraction 80 receivers", flush=True)
    scn = _scene(n_ping=8, n_across=40, nx=24, ny=16, nz=16)
    echo = synthesize_echo(scn, dtype=torch.complex64, refraction=REFR)
    img, plan, _ = gpu_image(api, scn, echo, refraction=REFR)
    assert scn.n_elem == 80 and plan.info()["tile_z"] == 4
    ref = oracle_image(scn, echo.numpy(), refraction=REFR).reshape(img.shape)
    r, ph = report("refraction 80 receivers", img, ref)
    assert r <= FP32_REL_L2 and ph <= FP32_PHASE_MRAD


def test_nonfinite_receiver_sets_status_and_zero_image(api):
    # a receiver position that is not finite: the plan reports bad navigation
    # and every tile (each one's pings include it: no gate) comes out zero
    print("case refraction non-finite receiver", flush=True)
    scn = _scene(n_ping=6, nx=16, ny=8, nz=8)
    echo = synthesize_echo(scn, dtype=torch.complex64, refraction=REFR)
    rx = scn.rx.copy()
    rx[2, 3, 0] = np.nan
    plan = api.sas_bp_plan([desc_for(api, scn, refraction=REFR)])
    buf = buffers_for(api, scn, echo, rx=rx)
    buf.image.fill_(3.0)
    api.sas_bp_image(plan, [buf])
    torch.cuda.synchronize()
    assert plan.status() == 5
    assert np.count_nonzero(buf.image.cpu().numpy()) == 0


def test_gated_2d_with_an_interface(api):
    # the stripmap geometry with a gate, pixels 0.2 m below an interface at z = -0.2
    print("case refraction gated 2D", flush=True)
    scn = make_config("c2", n_ping=32, n_elem=8, nx=160, ny=64, n_sample=4096, n_scat=20, n_speckle=100)
    refr = (1620.0, -0.2)
    echo = synthesize_echo(scn, dtype=torch.complex64, refraction=refr)
    img, plan, _ = gpu_image(api, scn, echo, refraction=refr)
    ref = oracle_image(scn, echo.numpy(), refraction=refr).reshape(img.shape)
    r, ph = report("refraction gated 2D", img, ref)
    assert r <= FP32_REL_L2 and ph <= FP32_PHASE_MRAD


def test_equal_speeds_match_the_straight_kernel(api):
    scn = _scene()
    echo = synthesize_echo(scn, dtype=torch.complex64)
    img_r, _, _ = gpu_image(api, scn, echo, refraction=(scn.c, 5.5))
    img_s, _, _ = gpu_image(api, scn, echo)
    r, ph = report("refraction c_sed = c vs straight kernel", img_r, img_s)
    assert r <= 2e-5


def test_refraction_plans_refuse_other_paths(api):
    scn = _scene(n_ping=4, nx=16, ny=8, nz=8)
    echo = synthesize_echo(scn, dtype=torch.complex64, refraction=REFR)
    img, plan, buf = gpu_image(api, scn, echo, refraction=REFR)
    with pytest.raises(RuntimeError):
        api.sas_bp_reproject(plan, [buf], [buf.image], [torch.zeros_like(buf.echo)])
    with pytest.raises(RuntimeError):
        api.sas_bp_plan([desc_for(api, scn, interp="sinc8", refraction=REFR)])
    with pytest.raises(RuntimeError):
        api.sas_bp_plan([desc_for(api, scn, refraction=(0.0, 5.5))])


@pytest.fixture(scope="module")
def full_volume(api):
    """The 3D workload at full size (256 pings x 64 receivers, 8192 samples,
    512 x 512 x 128 voxels) with the sediment interface, imaged once in the
    default launch configuration; 4096 seeded voxels weighted towards the
    seabed and large horizontal offsets are kept for the oracle."""
    print("case refraction c3 full size", flush=True)
    scn = make_config("c3", n_seabed=5000)
    echo = synthesize_echo(scn, device="cuda", dtype=torch.complex64, noise_on_device=True, refraction=REFR)
    plan = api.sas_bp_plan([desc_for(api, scn, refraction=REFR)])
    buf = buffers_for(api, scn, echo)
    api.sas_bp_image(plan, [buf])
    torch.cuda.synchronize()
    status = plan.status()
    idx = volume_subset(scn, 4096, REFR[1])
    img = buf.image.reshape(-1)[torch.as_tensor(idx, device="cuda")].cpu().numpy()
    echo_np = echo.cpu().numpy()
    del echo, buf
    plan.destroy()
    torch.cuda.empty_cache()
    return scn, echo_np, idx, img, status


@pytest.mark.parametrize("part", range(4))
def test_full_size_volume_refraction_sampled(full_volume, part):
    # the oracle's voxels in four parts of about 1024 (its bisection per leg
    # makes each part some 15 s of host time)
    scn, echo_np, idx, img, status = full_volume
    assert status == 0
    sel = slice(part * idx.size // 4, (part + 1) * idx.size // 4)
    ref = oracle_image(scn, echo_np, idx[sel], refraction=REFR, chunk=64)
    r, ph = report(f"refraction c3-full-subset part {part} ({ref.size} voxels)", img[sel], ref)
    assert r <= FP32_REL_L2 and ph <= FP32_PHASE_MRAD
