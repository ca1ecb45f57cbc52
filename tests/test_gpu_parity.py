"""HIP path vs the FP64 oracle, element by element, through the C ABI.

Every case synthesizes one echo cube (complex64), hands the same cube to the
GPU and to the oracle, and compares the images. The FP32 bound is 1e-4
relative L2 and 10 mrad maximum phase error over pixels within 30 dB of the
peak. Sizes are chosen so the oracle finishes in seconds while the image
spans several tiles with a ragged tail.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from synth import make_config, synthesize_echo, quantize_echo, dequantize_echo, subset_indices
from tests.helpers import (FP32_REL_L2, FP32_PHASE_MRAD, F16_REL_L2, F16_PHASE_MRAD, BF16_REL_L2,
                           BF16_PHASE_MRAD, desc_for, buffers_for, gpu_image, oracle_image, report,
                           volume_subset)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    import paper_2101_05888_amd as m
    return m


def _case(name, **kw):
    scn = make_config(name, **kw)
    echo = synthesize_echo(scn, dtype=torch.complex64)
    return scn, echo


CASES = {
    # 2D stripmap, workload 1 at full size
    "c1_full": ("c1", {}),
    # ragged 2D image, few pings
    "c1_ragged": ("c1", dict(n_ping=16, n_elem=4, nx=100, ny=77)),
    # gated operational geometry, scaled down, ragged
    "c2_small": ("c2", dict(n_ping=64, n_elem=8, nx=333, ny=129, n_sample=4096, n_scat=40, n_speckle=400)),
    # 3D volume below a downward-looking planar array
    "c3_small": ("c3", dict(n_ping=16, n_across=4, nx=40, ny=24, nz=10, n_seabed=300, n_surface=8,
                            n_buried=4, n_sample=2048)),
    # far pings beyond the record (out-of-record taps), no gate
    "c5_small": ("c5", dict(n_ping=64, n_elem=4, nx=128, ny=96, n_scat=30)),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_image_matches_oracle(api, case):
    name, kw = CASES[case]
    print(f"case {case}", flush=True)
    scn, echo = _case(name, **kw)
    img, plan, _ = gpu_image(api, scn, echo)
    ref = oracle_image(scn, echo.numpy()).reshape(img.shape)
    r, ph = report(case, img, ref)
    assert np.abs(ref).max() > 0
    assert r <= FP32_REL_L2
    assert ph <= FP32_PHASE_MRAD
    plan.destroy()


def test_lone_scatterer_peak_closed_form(api):
    # GPU counterpart of the oracle pin: a scatterer on a pixel centre focuses
    # to a * sum G(w) with zero phase
    scn = make_config("c1", n_scat=1, snr_db=None, n_ping=32, n_elem=8, nx=64, ny=64)
    p = scn.grid.points(np.array([37 * 64 + 21]))[0]
    scn.scat_pos = p[None]
    scn.scat_amp = np.array([0.8 + 0.6j])
    echo = synthesize_echo(scn, dtype=torch.complex64)
    img, plan, _ = gpu_image(api, scn, echo)
    ref = oracle_image(scn, echo.numpy(), np.array([37 * 64 + 21]))[0]
    got = img[0, 37, 21]
    assert abs(got - ref) <= 1e-4 * abs(ref)
    assert abs(np.angle(got / (0.8 + 0.6j))) < 1e-3
    assert int(np.argmax(np.abs(img))) == 37 * 64 + 21


@pytest.mark.parametrize("tile_x", [16, 32, 64])
def test_tile_shapes_agree(api, tile_x):
    scn, echo = _case("c2", n_ping=48, n_elem=6, nx=150, ny=70, n_sample=4096, n_scat=30, n_speckle=0)
    img, plan, _ = gpu_image(api, scn, echo, tile=(tile_x, 0, 0))
    ref = oracle_image(scn, echo.numpy()).reshape(img.shape)
    r, ph = report(f"tile{tile_x}", img, ref)
    assert r <= FP32_REL_L2 and ph <= FP32_PHASE_MRAD


@pytest.mark.parametrize("cp", [1, 3])
def test_ping_chunking_is_bitwise_neutral_within_a_tiling(api, cp):
    scn, echo = _case("c1", n_ping=20, n_elem=5, nx=70, ny=40)
    a, _, _ = gpu_image(api, scn, echo, pings_per_chunk=cp)
    b, _, _ = gpu_image(api, scn, echo, pings_per_chunk=2)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("epc", [3, 4, 7])
def test_element_chunks_are_bitwise_neutral_and_match_oracle(api, epc):
    # chunks of 3 and 7 records straddle pings (8 elements each), 4 split one
    # ping in two; gated geometry so that partially gated rows cross chunks
    print(f"elements per chunk {epc}", flush=True)
    scn, echo = _case("c2", n_ping=24, n_elem=8, nx=150, ny=70, n_sample=4096, n_scat=30, n_speckle=100)
    a, plan, _ = gpu_image(api, scn, echo, elems_per_chunk=epc)
    assert plan.info()["records_per_chunk"] == epc
    b, _, _ = gpu_image(api, scn, echo, pings_per_chunk=1)
    assert np.array_equal(a, b)
    ref = oracle_image(scn, echo.numpy()).reshape(a.shape)
    r, ph = report(f"epc{epc}", a, ref)
    assert r <= FP32_REL_L2 and ph <= FP32_PHASE_MRAD


def test_graph_replay_equals_direct_launch_and_is_deterministic(api):
    scn, echo = _case("c2", n_ping=40, n_elem=4, nx=96, ny=64, n_sample=4096, n_scat=20, n_speckle=50)
    a, plan, buf = gpu_image(api, scn, echo, use_graph=True)
    b, _, _ = gpu_image(api, scn, echo, use_graph=False)
    assert np.array_equal(a, b)
    # replays: image overwritten each time, identical bits, with eager work between
    for _ in range(3):
        buf.image.fill_(1.0 + 1.0j)
        api.sas_bp_image(plan, [buf])
        torch.cuda.synchronize()
        assert np.array_equal(buf.image.cpu().numpy(), a)


def test_kernel_timing_brackets_each_launch(api):
    scn, echo = _case("c1", n_ping=12, n_elem=4, nx=64, ny=48)
    ref, plan, buf = gpu_image(api, scn, echo)
    api.sas_bp_set_kernel_timing(plan, True)
    for _ in range(3):
        buf.image.fill_(0)
        api.sas_bp_image(plan, [buf])
    ms, n = api.sas_bp_kernel_time(plan)
    assert n == 3 and ms > 0.0
    assert np.array_equal(buf.image.cpu().numpy(), ref)     # direct launches, same bits
    assert api.sas_bp_kernel_time(plan) == (0.0, 0)         # the read starts a new count
    api.sas_bp_set_kernel_timing(plan, False)
    api.sas_bp_image(plan, [buf])
    assert api.sas_bp_kernel_time(plan) == (0.0, 0)         # graph replays are not timed


def test_autotune_choice_is_a_valid_tiling_and_cached(api):
    scn, echo = _case("c2", n_ping=48, n_elem=6, nx=200, ny=96, n_sample=4096, n_scat=20, n_speckle=100)
    d = desc_for(api, scn)
    buf = buffers_for(api, scn, echo)
    best = api.sas_bp_autotune([d], [buf], reps=2)
    assert best["ms"] > 0.0 and best["pings_per_chunk"] in (0, 1, 2, 4, 8)
    again = api.sas_bp_autotune([d], [buf], reps=2)
    assert again["ms"] == 0.0 and {k: v for k, v in again.items() if k != "ms"} == \
        {k: v for k, v in best.items() if k != "ms"}
    kw = {k: v for k, v in best.items() if k != "ms"}
    img, plan, _ = gpu_image(api, scn, echo, **kw)
    info = plan.info()
    assert (info["tile_x"], info["tile_y"], info["tile_z"]) == tuple(best["tile"])
    assert info["threads"] == best["threads"] and info["workgroups_per_cu"] >= 1
    ppc, epc = best["pings_per_chunk"], best["elems_per_chunk"]
    if 0 < epc < d.n_elem:
        assert info["records_per_chunk"] == epc
    elif ppc > 0:
        assert info["pings_per_chunk"] == ppc and info["records_per_chunk"] == ppc * d.n_elem
    r, ph = report("autotuned", img, oracle_image(scn, echo.numpy()).reshape(img.shape))
    assert r <= FP32_REL_L2 and ph <= FP32_PHASE_MRAD


def test_graph_sees_new_navigation_and_sound_speed(api):
    scn, echo = _case("c1", n_ping=12, n_elem=4, nx=48, ny=40)
    img, plan, buf = gpu_image(api, scn, echo)
    tx2 = scn.tx.copy()
    tx2[:, 1] += 0.003
    rx2 = scn.rx.copy()
    rx2[:, :, 1] += 0.003
    buf.tx.copy_(torch.as_tensor(tx2))
    buf.rx.copy_(torch.as_tensor(rx2))
    buf.c.fill_(1490.0)
    api.sas_bp_image(plan, [buf])
    torch.cuda.synchronize()
    got = buf.image.cpu().numpy()
    g = scn.grid
    pts = oracle.pixel_points(g.origin, g.spacing, g.n)
    ref = oracle.backproject(echo.numpy(), tx2, rx2, 1490.0, scn.fc, scn.fs, scn.t0, pts).reshape(got.shape)
    r, ph = report("renav", got, ref)
    assert r <= FP32_REL_L2 and ph <= FP32_PHASE_MRAD


def test_batched_plan_equals_separate_plans(api):
    scns = [make_config(f"c4b:{k}", nx=nx, ny=ny, n_ping=np_, n_elem=ne, n_scat=10, n_sample=4096)
            for k, (nx, ny, np_, ne) in enumerate([(70, 40, 30, 5), (33, 90, 24, 7), (128, 17, 40, 4)])]
    echoes = [synthesize_echo(s, dtype=torch.complex64) for s in scns]
    plan = api.sas_bp_plan([desc_for(api, s) for s in scns], tile=(32, 0, 0))
    bufs = [buffers_for(api, s, e) for s, e in zip(scns, echoes)]
    api.sas_bp_image(plan, bufs)
    torch.cuda.synchronize()
    for s, e, b in zip(scns, echoes, bufs):
        alone, _, _ = gpu_image(api, s, e, tile=(32, 0, 0))
        assert np.array_equal(b.image.cpu().numpy(), alone)
        ref = oracle_image(s, e.numpy()).reshape(alone.shape)
        r, ph = report(s.name, alone, ref)
        assert r <= FP32_REL_L2 and ph <= FP32_PHASE_MRAD


@pytest.mark.parametrize("kind", ["f16", "bf16"])
def test_sixteen_bit_echoes(api, kind):
    scn = make_config("c1")
    echo = synthesize_echo(scn, dtype=torch.complex64)
    q, scale = quantize_echo(echo, kind)
    img, _, _ = gpu_image(api, scn, q, echo_dtype=kind, echo_scale=scale)
    # compute-only error: oracle on the dequantised echo meets the FP32 bounds
    deq = dequantize_echo(q, scale).numpy()
    r1, p1 = report(f"{kind}-compute", img, oracle_image(scn, deq).reshape(img.shape))
    assert r1 <= FP32_REL_L2 and p1 <= FP32_PHASE_MRAD
    # storage + compute error against the original echo
    r2, p2 = report(f"{kind}-storage", img, oracle_image(scn, echo.numpy()).reshape(img.shape))
    lim_r, lim_p = (F16_REL_L2, F16_PHASE_MRAD) if kind == "f16" else (BF16_REL_L2, BF16_PHASE_MRAD)
    assert r2 <= lim_r and p2 <= lim_p


def test_useful_updates_count_matches_oracle(api):
    scn, echo = _case("c2", n_ping=48, n_elem=6, nx=150, ny=70, n_sample=4096, n_scat=5, n_speckle=0)
    plan = api.sas_bp_plan([desc_for(api, scn)])
    buf = buffers_for(api, scn, echo)
    got = api.sas_bp_useful_updates(plan, [buf])[0]
    g = scn.grid
    want = oracle.gated_term_count(scn.tx, scn.rx, g.points(), scn.gate_half_angle)
    assert got == want and 0 < got < scn.nominal_updates()


def test_degenerate_sizes(api):
    # one pixel, one ping, one element
    scn, echo = _case("c1", n_ping=1, n_elem=1, nx=1, ny=1, n_scat=3)
    img, _, _ = gpu_image(api, scn, echo)
    ref = oracle_image(scn, echo.numpy()).reshape(img.shape)
    assert abs(img.ravel()[0] - ref.ravel()[0]) <= 1e-4 * max(abs(ref.ravel()[0]), 1e-12)


def test_all_terms_outside_record_give_zero_image(api):
    scn, echo = _case("c1", n_ping=8, n_elem=2, nx=20, ny=20, n_sample=64)
    img, _, _ = gpu_image(api, scn, echo)
    assert np.count_nonzero(img) == 0


def test_bad_sound_speed_sets_status_and_zero_image(api):
    scn, echo = _case("c1", n_ping=8, n_elem=2, nx=20, ny=20)
    plan = api.sas_bp_plan([desc_for(api, scn)])
    buf = buffers_for(api, scn, echo, c=900.0)      # below the default c_min of 1400 m/s
    buf.image.fill_(3.0)
    api.sas_bp_image(plan, [buf])
    torch.cuda.synchronize()
    assert plan.status() == 5
    assert np.count_nonzero(buf.image.cpu().numpy()) == 0
    assert plan.status() == 0                       # cleared on read


def test_nonfinite_navigation_sets_status(api):
    scn, echo = _case("c1", n_ping=8, n_elem=2, nx=20, ny=20)
    tx = scn.tx.copy()
    tx[3, 1] = np.nan
    plan = api.sas_bp_plan([desc_for(api, scn)])
    buf = buffers_for(api, scn, echo, tx=tx)
    api.sas_bp_image(plan, [buf])
    torch.cuda.synchronize()
    assert plan.status() == 5
    assert np.isfinite(buf.image.cpu().numpy()).all()


def test_full_size_operational_swath_sampled(api):
    # the throughput workload at its full size (512 pings x 32 receivers,
    # 4096 x 4096 pixels, +-10 deg gate), in the launch configuration the
    # benchmark times, compared on a seeded pixel subset
    print("case c2 full size", flush=True)
    scn = make_config("c2")
    echo = synthesize_echo(scn, device="cuda", dtype=torch.complex64)
    plan = api.sas_bp_plan([desc_for(api, scn)])
    buf = buffers_for(api, scn, echo)
    api.sas_bp_image(plan, [buf])
    torch.cuda.synchronize()
    assert plan.status() == 0
    idx = subset_indices(scn, 2048)
    img = buf.image.reshape(-1)[torch.as_tensor(idx, device="cuda")].cpu().numpy()
    echo_np = echo.cpu().numpy()
    del echo, buf
    ref = oracle_image(scn, echo_np, idx)
    r, ph = report("c2-full-subset", img, ref)
    assert r <= FP32_REL_L2 and ph <= FP32_PHASE_MRAD


def test_full_size_volume_sampled(api):
    # the 3D workload at its full size (256 pings x 64 receivers, 8192
    # samples, 512 x 512 x 128 voxels) in the default launch configuration,
    # compared on 4096 seeded voxels weighted towards the seabed and large
    # horizontal offsets; the seabed carries 5000 weak scatterers instead of
    # 1e5 to keep the synthesis short (the content does not change the work
    # or the arithmetic)
    print("case c3 full size", flush=True)
    scn = make_config("c3", n_seabed=5000)
    echo = synthesize_echo(scn, device="cuda", dtype=torch.complex64, noise_on_device=True)
    plan = api.sas_bp_plan([desc_for(api, scn)])
    buf = buffers_for(api, scn, echo)
    api.sas_bp_image(plan, [buf])
    torch.cuda.synchronize()
    assert plan.status() == 0
    idx = volume_subset(scn, 4096, 5.5)
    img = buf.image.reshape(-1)[torch.as_tensor(idx, device="cuda")].cpu().numpy()
    echo_np = echo.cpu().numpy()
    del echo, buf
    ref = oracle_image(scn, echo_np, idx, chunk=256)
    r, ph = report(f"c3-full-subset ({idx.size} voxels)", img, ref)
    assert r <= FP32_REL_L2 and ph <= FP32_PHASE_MRAD


def test_wide_tile_without_adjoint_still_images(api):
    # 64 receivers and a 64 x 8 x 4 voxel tile: one ping's windows need more
    # LDS than a workgroup has, so the plan images in element chunks and the
    # adjoint (which stages whole pings) is refused with EUNSUPPORTED
    from paper_2101_05888_amd._native import SasBpError, SAS_BP_EUNSUPPORTED
    scn, echo = _case("c3", n_ping=6, n_across=32, nx=70, ny=16, nz=9, n_seabed=100, n_surface=6, n_buried=2,
                      n_sample=2048)
    img, plan, buf = gpu_image(api, scn, echo, tile=(64, 8, 4), threads=256)
    info = plan.info()
    assert info["records_per_chunk"] < scn.n_elem
    ref = oracle_image(scn, echo.numpy()).reshape(img.shape)
    r, ph = report("wide-tile", img, ref)
    assert r <= FP32_REL_L2 and ph <= FP32_PHASE_MRAD
    g = torch.zeros_like(buf.image)
    gtx = torch.zeros((scn.n_ping, 3), dtype=torch.float64, device="cuda")
    grx = torch.zeros((scn.n_ping, scn.n_elem, 3), dtype=torch.float64, device="cuda")
    gc = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(SasBpError) as ei:
        api.sas_bp_adjoint(plan, [buf], [g], [gtx], [grx], [gc])
    assert ei.value.status == SAS_BP_EUNSUPPORTED


# ------------------------------------------------- windowed-sinc variant ---

@pytest.mark.parametrize("case", ["c1_ragged", "c2_small", "c3_small", "c5_small"])
def test_sinc_image_matches_oracle(api, case):
    name, kw = CASES[case]
    print(f"sinc case {case}", flush=True)
    scn, echo = _case(name, **kw)
    img, plan, _ = gpu_image(api, scn, echo, interp="sinc8")
    ref = oracle_image(scn, echo.numpy(), interp="sinc8").reshape(img.shape)
    r, ph = report(f"sinc-{case}", img, ref)
    assert np.abs(ref).max() > 0
    assert r <= FP32_REL_L2 and ph <= FP32_PHASE_MRAD
    lin = oracle_image(scn, echo.numpy()).reshape(img.shape)
    assert oracle.rel_l2(img, lin) > 10 * FP32_REL_L2      # a different interpolator


@pytest.mark.parametrize("kw", [dict(elems_per_chunk=3), dict(tile=(64, 0, 0)), dict(pings_per_chunk=2)])
def test_sinc_tilings_match_oracle(api, kw):
    scn, echo = _case("c2", n_ping=24, n_elem=8, nx=150, ny=70, n_sample=4096, n_scat=30, n_speckle=100)
    img, _, _ = gpu_image(api, scn, echo, interp="sinc8", **kw)
    ref = oracle_image(scn, echo.numpy(), interp="sinc8").reshape(img.shape)
    r, ph = report(f"sinc-{kw}", img, ref)
    assert r <= FP32_REL_L2 and ph <= FP32_PHASE_MRAD


def test_sinc_sixteen_bit_storage(api):
    scn, echo = _case("c1", n_ping=16, n_elem=4, nx=100, ny=77)
    q, scale = quantize_echo(echo, "f16")
    deq = dequantize_echo(q, scale)
    img, _, _ = gpu_image(api, scn, q, echo_dtype="f16", echo_scale=scale, interp="sinc8")
    ref = oracle_image(scn, deq.numpy(), interp="sinc8").reshape(img.shape)
    r, ph = report("sinc-f16-compute", img, ref)
    assert r <= FP32_REL_L2 and ph <= FP32_PHASE_MRAD


def test_sinc_plan_refuses_adjoint_and_reprojection(api):
    from paper_2101_05888_amd._native import SasBpError, SAS_BP_EUNSUPPORTED
    scn, echo = _case("c1", n_ping=8, n_elem=4, nx=48, ny=40)
    img, plan, buf = gpu_image(api, scn, echo, interp="sinc8")
    g = torch.zeros_like(buf.image)
    with pytest.raises(SasBpError) as ei:
        api.sas_bp_adjoint(plan, [buf], [g], [torch.zeros((8, 3), dtype=torch.float64, device="cuda")],
                           [torch.zeros((8, 4, 3), dtype=torch.float64, device="cuda")],
                           [torch.zeros(1, dtype=torch.float64, device="cuda")])
    assert ei.value.status == SAS_BP_EUNSUPPORTED
    with pytest.raises(SasBpError) as ei:
        api.sas_bp_reproject(plan, [buf], [g], [torch.zeros_like(buf.echo)])
    assert ei.value.status == SAS_BP_EUNSUPPORTED


def test_full_size_sinc_sampled(api):
    # the windowed-sinc variant on the operational swath at full size, default
    # launch configuration, compared with the oracle's variant on 256 pixels
    print("case c2 full size sinc", flush=True)
    scn = make_config("c2")
    echo = synthesize_echo(scn, device="cuda", dtype=torch.complex64)
    plan = api.sas_bp_plan([desc_for(api, scn, interp="sinc8")])
    buf = buffers_for(api, scn, echo)
    api.sas_bp_image(plan, [buf])
    torch.cuda.synchronize()
    assert plan.status() == 0
    idx = subset_indices(scn, 256)
    img = buf.image.reshape(-1)[torch.as_tensor(idx, device="cuda")].cpu().numpy()
    echo_np = echo.cpu().numpy()
    del echo, buf
    ref = oracle_image(scn, echo_np, idx, interp="sinc8")
    r, ph = report("c2-full-sinc-subset", img, ref)
    assert r <= FP32_REL_L2 and ph <= FP32_PHASE_MRAD
