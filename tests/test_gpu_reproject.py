"""Reprojection (linear adjoint of the image in the echo) through the C ABI
against the FP64 oracle's reprojection, element by element over the echo
cube, and the adjoint identity between the GPU's own forward and adjoint.

The cotangent images are seeded complex Gaussian fields. Bound: 1e-4
relative L2 over the whole cube (the FP32 image bound; each output sample is
a sum of weighted terms whose FP32 delays, weights and phasors carry the same
errors as the image's).
"""
import numpy as np
import pytest
import torch

import oracle
from synth import make_config, synthesize_echo
from tests.helpers import FP32_REL_L2, desc_for, buffers_for, gpu_image, workers

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    import paper_2101_05888_amd as m
    return m


def _y(scn, seed=3):
    g = scn.grid
    rng = np.random.default_rng(seed)
    n = g.n[2] * g.n[1] * g.n[0]
    return (rng.normal(size=n) + 1j * rng.normal(size=n)).reshape(g.n[2], g.n[1], g.n[0])


def _gpu_reproject(api, scn, echo, y, **plan_kw):
    plan = api.sas_bp_plan([desc_for(api, scn)], **plan_kw)
    buf = buffers_for(api, scn, echo)
    yin = torch.as_tensor(y, dtype=torch.complex64, device="cuda").contiguous()
    out = torch.full((scn.n_ping, scn.n_elem, scn.n_sample), complex(7.0, -7.0), dtype=torch.complex64,
                     device="cuda")   # overwritten
    api.sas_bp_reproject(plan, [buf], [yin], [out])
    torch.cuda.synchronize()
    assert plan.status() == 0
    return out.cpu().numpy(), plan


def _oracle_reproject(scn, y):
    g = scn.grid
    pts = oracle.pixel_points(g.origin, g.spacing, g.n)
    return oracle.reproject(y.reshape(-1), scn.tx, scn.rx, scn.c, scn.fc, scn.fs, scn.t0, pts, scn.n_sample,
                            scn.gate_half_angle)


CASES = {
    "c1_ragged": ("c1", dict(n_ping=12, n_elem=4, nx=100, ny=77)),
    "c2_gated": ("c2", dict(n_ping=32, n_elem=8, nx=200, ny=96, n_sample=4096, n_scat=10, n_speckle=0)),
    "c3_volume": ("c3", dict(n_ping=8, n_across=4, nx=40, ny=24, nz=10, n_seabed=50, n_surface=4, n_buried=2,
                             n_sample=2048)),
    "c5_off_record": ("c5", dict(n_ping=32, n_elem=4, nx=128, ny=96, n_scat=10)),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_reprojection_matches_oracle(api, case):
    name, kw = CASES[case]
    print(f"reprojection case {case}", flush=True)
    scn = make_config(name, **kw)
    echo = synthesize_echo(scn, dtype=torch.complex64)
    y = _y(scn)
    got, _ = _gpu_reproject(api, scn, echo, y)
    ref = _oracle_reproject(scn, y)
    r = oracle.rel_l2(got, ref)
    print(f"[{case}] reprojection rel_l2={r:.3e} nonzero={np.count_nonzero(ref)}", flush=True)
    assert np.abs(ref).max() > 0 and r <= FP32_REL_L2
    # samples no term reaches are exactly zero
    assert np.all(got[ref == 0] == 0)


@pytest.mark.parametrize("kw", [dict(tile=(64, 0, 0)), dict(elems_per_chunk=3), dict(pings_per_chunk=2)])
def test_reprojection_tilings_match_oracle(api, kw):
    scn = make_config("c2", n_ping=24, n_elem=8, nx=150, ny=70, n_sample=4096, n_scat=10, n_speckle=0)
    echo = synthesize_echo(scn, dtype=torch.complex64)
    y = _y(scn, seed=4)
    got, _ = _gpu_reproject(api, scn, echo, y, **kw)
    r = oracle.rel_l2(got, _oracle_reproject(scn, y))
    print(f"[{kw}] reprojection rel_l2={r:.3e}", flush=True)
    assert r <= FP32_REL_L2


def test_adjoint_identity_on_the_gpu(api):
    # <A x, y> from the GPU image and <x, A^H y> from the GPU reprojection
    scn = make_config("c2", n_ping=32, n_elem=8, nx=200, ny=96, n_sample=4096, n_scat=30, n_speckle=100)
    echo = synthesize_echo(scn, dtype=torch.complex64)
    y = _y(scn, seed=9)
    img, _, _ = gpu_image(api, scn, echo)
    ahy, _ = _gpu_reproject(api, scn, echo, y)
    lhs = np.vdot(img.astype(np.complex128).ravel(), y.ravel())
    rhs = np.vdot(echo.numpy().astype(np.complex128).ravel(), ahy.astype(np.complex128).ravel())
    rel = abs(lhs - rhs) / abs(lhs)
    print(f"adjoint identity: |<Ax,y> - <x,A^H y>| / |<Ax,y>| = {rel:.3e}", flush=True)
    assert rel <= 1e-4


def test_reprojection_overwrites_and_repeats(api):
    scn = make_config("c1", n_ping=8, n_elem=4, nx=48, ny=40)
    echo = synthesize_echo(scn, dtype=torch.complex64)
    y = _y(scn, seed=2)
    a, plan = _gpu_reproject(api, scn, echo, y)
    buf = buffers_for(api, scn, echo)
    yin = torch.as_tensor(y, dtype=torch.complex64, device="cuda").contiguous()
    out = torch.full((scn.n_ping, scn.n_elem, scn.n_sample), complex(1.0, 1.0), dtype=torch.complex64, device="cuda")
    api.sas_bp_reproject(plan, [buf], [yin], [out])
    api.sas_bp_reproject(plan, [buf], [yin], [out])
    torch.cuda.synchronize()
    b = out.cpu().numpy()
    assert oracle.rel_l2(b, a) <= 1e-6


def test_autograd_echo_gradient_is_the_reprojection(api):
    # the image is linear in the echo, so for J = sum |I|^2 the echo gradient
    # in PyTorch's convention is A^H (2 I)
    from paper_2101_05888_amd.autograd import tdbp_image
    scn = make_config("c5", n_ping=16, n_elem=4, nx=64, ny=48, n_scat=12)
    echo = synthesize_echo(scn, dtype=torch.complex64).cuda().requires_grad_(True)
    plan = api.sas_bp_plan([desc_for(api, scn)])
    tx = torch.as_tensor(scn.tx, device="cuda")
    rx = torch.as_tensor(scn.rx, device="cuda")
    c = torch.tensor([scn.c], dtype=torch.float64, device="cuda")
    img = tdbp_image(plan, echo, tx, rx, c)
    (torch.view_as_real(img) ** 2).sum().backward()
    got = echo.grad.cpu().numpy()
    ref = _oracle_reproject(scn, 2.0 * img.detach().cpu().numpy().astype(np.complex128))
    r = oracle.rel_l2(got, ref)
    print(f"autograd echo gradient rel_l2={r:.3e}", flush=True)
    assert r <= FP32_REL_L2


def test_full_size_adjoint_identity(api):
    # the operational swath at full size (512 pings x 32 receivers, 16384
    # samples, 4096 x 4096 pixels, gate): <A x, y> = <x, A^H y> between the
    # GPU image and the GPU reprojection, a property that holds at any size
    print("case c2 full size adjoint identity", flush=True)
    scn = make_config("c2")
    echo = synthesize_echo(scn, device="cuda", dtype=torch.complex64, noise_on_device=True)
    plan = api.sas_bp_plan([desc_for(api, scn)])
    buf = buffers_for(api, scn, echo)
    api.sas_bp_image(plan, [buf])
    gen = torch.Generator(device="cuda").manual_seed(17)
    y = torch.randn(buf.image.shape, dtype=torch.complex64, device="cuda", generator=gen)
    out = torch.empty_like(buf.echo)
    api.sas_bp_reproject(plan, [buf], [y], [out])
    torch.cuda.synchronize()
    assert plan.status() == 0
    lhs = torch.vdot(buf.image.reshape(-1).to(torch.complex128), y.reshape(-1).to(torch.complex128)).item()
    rhs = torch.vdot(buf.echo.reshape(-1).to(torch.complex128), out.reshape(-1).to(torch.complex128)).item()
    rel = abs(lhs - rhs) / abs(lhs)
    print(f"full-size adjoint identity {rel:.3e}", flush=True)
    assert rel <= 1e-4
