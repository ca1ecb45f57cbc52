"""Geometry adjoint, sharpness and autograd on the GPU against the FP64 oracle.

The adjoint (vector-Jacobian product of the image with respect to the
transmitter and receiver positions and the sound speed) is compared with the
oracle's analytic gradient in every lane layout and at the autofocus
workload's full size, and with central finite differences of the GPU's and
the oracle's forward images; the sharpness objective and its cotangent with
the oracle's.
Bounds: the gradient sums many FP32 terms of both signs, so its error is
measured relative to the gradient's norm (GRAD_REL). On top of that, the
interpolator's slope jumps at every sample: a term whose sample position lies
within FP32 rounding of a sample may take the other slope. The oracle bounds
what such choices can change (``vjp_segment_bound`` over terms within
SEG_DELTA samples of a sample), and only the excess over that bound counts.
SEG_DELTA = 1e-4 samples is about twice the worst FP32 error of the sample
position: the position is rounded once where its magnitude is below 256
samples (half an ulp, 1.5e-5) and its delay offset carries a few ulps of a
sub-metre distance (under 1e-5 samples at 53 samples per metre).
"""
import numpy as np
import pytest
import torch

import oracle
from synth import make_config, synthesize_echo
from tests.helpers import desc_for, buffers_for

pytestmark = pytest.mark.gpu

GRAD_REL = 2e-4
SEG_DELTA = 1e-4


@pytest.fixture(scope="module")
def api():
    import paper_2101_05888_amd as m
    return m


def _grad_case(api, name, seed=3, tile=(0, 0, 0), **kw):
    scn = make_config(name, **kw)
    echo = synthesize_echo(scn, dtype=torch.complex64)
    plan = api.sas_bp_plan([desc_for(api, scn)], tile=tile)
    buf = buffers_for(api, scn, echo)
    g = scn.grid
    rng = np.random.default_rng(seed)
    gbar = (rng.normal(size=(g.n[2], g.n[1], g.n[0])) + 1j * rng.normal(size=(g.n[2], g.n[1], g.n[0])))
    gbar_t = torch.as_tensor(gbar.astype(np.complex64), device="cuda")
    gtx = torch.zeros((scn.n_ping, 3), dtype=torch.float64, device="cuda")
    grx = torch.zeros((scn.n_ping, scn.n_elem, 3), dtype=torch.float64, device="cuda")
    gc = torch.zeros(1, dtype=torch.float64, device="cuda")
    api.sas_bp_adjoint(plan, [buf], [gbar_t], [gtx], [grx], [gc])
    torch.cuda.synchronize()
    assert plan.status() == 0
    return scn, echo, plan, buf, gbar_t, gtx.cpu().numpy(), grx.cpu().numpy(), float(gc.cpu()[0])


def _rel(a, b):
    a, b = np.ravel(a), np.ravel(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


C5_SMALL = dict(n_ping=24, n_elem=4, nx=70, ny=50, n_scat=20)
C2_SMALL = dict(n_ping=40, n_elem=6, nx=90, ny=40, n_sample=4096, n_scat=20, n_speckle=100)
C3_SMALL = dict(n_ping=10, n_across=4, nx=24, ny=20, nz=6, n_seabed=200, n_surface=6, n_buried=2, n_sample=2048)


# every lane layout the adjoint runs: 16 x 32 (small images), 32 x 32, and the
# 64 x 32, 8 pixels per lane, of large images such as the autofocus workload;
# 32 x 8 x 4 and 64 x 8 x 4 voxels for volumes
@pytest.mark.parametrize("name,kw,tile", [
    ("c5", C5_SMALL, (0, 0, 0)), ("c5", C5_SMALL, (32, 0, 0)), ("c5", C5_SMALL, (64, 0, 0)),
    ("c2", C2_SMALL, (0, 0, 0)), ("c2", C2_SMALL, (32, 0, 0)), ("c2", C2_SMALL, (64, 0, 0)),
    ("c3", C3_SMALL, (0, 0, 0)), ("c3", C3_SMALL, (64, 0, 0)),
])
def test_adjoint_matches_oracle_gradient(api, name, kw, tile):
    print(f"case {name} tile {tile}", flush=True)
    scn, echo, plan, buf, gbar, gtx, grx, gc = _grad_case(api, name, tile=tile, **kw)
    info = plan.info()
    assert tile[0] == 0 or info["tile_x"] == tile[0]
    g = scn.grid
    pts = oracle.pixel_points(g.origin, g.spacing, g.n)
    args = (echo.numpy(), scn.tx, scn.rx, scn.c, scn.fc, scn.fs, scn.t0, pts, gbar.cpu().numpy().ravel(),
            scn.gate_half_angle)
    otx, orx, oc = oracle.vjp(*args)
    btx, brx, bc = oracle.vjp_segment_bound(*args, delta=SEG_DELTA)
    r_tx, r_rx, r_c = _rel(gtx, otx), _rel(grx, orx), abs(gc - oc) / abs(oc)
    # error beyond what segment choices at samples can explain
    x_tx = np.linalg.norm(np.maximum(np.abs(gtx - otx) - btx, 0.0)) / np.linalg.norm(otx)
    x_rx = np.linalg.norm(np.maximum(np.abs(grx - orx) - brx, 0.0)) / np.linalg.norm(orx)
    x_c = max(abs(gc - oc) - bc, 0.0) / abs(oc)
    print(f"[{name} {info['tile_x']}x{info['tile_y']}x{info['tile_z']}] grad rel: tx {r_tx:.2e} rx {r_rx:.2e} "
          f"c {r_c:.2e}; beyond segment bound "
          f"tx {x_tx:.2e} rx {x_rx:.2e} c {x_c:.2e} (bound/|g|: tx {np.linalg.norm(btx) / np.linalg.norm(otx):.1e})",
          flush=True)
    assert np.linalg.norm(otx) > 0
    assert x_tx <= GRAD_REL and x_rx <= GRAD_REL and x_c <= GRAD_REL


def test_adjoint_matches_finite_differences(api):
    # central differences with the workload's 1e-4 m step, of the GPU's own
    # forward image and of the FP64 oracle's, against the GPU's analytic
    # gradient. The interpolator's slope jumps at every sample, so even exact
    # differences differ from the analytic gradient wherever a step crosses a
    # sample: the oracle's own difference measures that (``kink``), and the
    # GPU gradient may differ from the oracle's difference by that plus FD_TOL.
    # The GPU's difference differs from the oracle's only by FP32 rounding of
    # the two images.
    scn, echo, plan, buf, gbar, gtx, grx, gc = _grad_case(api, "c5", n_ping=16, n_elem=4, nx=64, ny=48,
                                                        n_scat=15)
    gb = gbar.cpu().numpy().astype(np.complex128).ravel()
    g = scn.grid
    pts = oracle.pixel_points(g.origin, g.spacing, g.n)
    echo_np = echo.numpy()

    def J_gpu(tx, rx, c):
        b = buffers_for(api, scn, echo, tx=tx, rx=rx, c=c)
        api.sas_bp_image(plan, [b])
        torch.cuda.synchronize()
        return float(np.real(np.vdot(gb, b.image.cpu().numpy().astype(np.complex128).ravel())))

    def J_ora(tx, rx, c):
        return float(np.real(np.vdot(gb, oracle.backproject(echo_np, tx, rx, c, scn.fc, scn.fs, scn.t0, pts))))

    otx, orx, oc = oracle.vjp(echo_np, scn.tx, scn.rx, scn.c, scn.fc, scn.fs, scn.t0, pts, gb)
    scale = np.abs(otx).max()
    FD_TOL = 2e-4
    h = 1e-4   # metres, as the workload specifies
    rng = np.random.default_rng(1)
    for _ in range(6):
        i, a = int(rng.integers(scn.n_ping)), int(rng.integers(3))
        tp, tm = scn.tx.copy(), scn.tx.copy()
        tp[i, a] += h
        tm[i, a] -= h
        fd_g = (J_gpu(tp, scn.rx, scn.c) - J_gpu(tm, scn.rx, scn.c)) / (2 * h)
        fd_o = (J_ora(tp, scn.rx, scn.c) - J_ora(tm, scn.rx, scn.c)) / (2 * h)
        kink = abs(fd_o - otx[i, a])
        print(f"[fd tx {i},{a}] analytic {gtx[i, a]:.6e} oracle {otx[i, a]:.6e} fd gpu {fd_g:.6e} fd oracle "
              f"{fd_o:.6e}; |fd gpu - fd oracle| {abs(fd_g - fd_o) / scale:.1e}, kink {kink / scale:.1e} of max|g|",
              flush=True)
        assert abs(fd_g - fd_o) <= FD_TOL * scale
        assert abs(gtx[i, a] - fd_o) <= kink + FD_TOL * scale
    hc = 1e-2
    fdc_g = (J_gpu(scn.tx, scn.rx, scn.c + hc) - J_gpu(scn.tx, scn.rx, scn.c - hc)) / (2 * hc)
    fdc_o = (J_ora(scn.tx, scn.rx, scn.c + hc) - J_ora(scn.tx, scn.rx, scn.c - hc)) / (2 * hc)
    print(f"[fd c] analytic {gc:.6e} oracle {oc:.6e} fd gpu {fdc_g:.6e} fd oracle {fdc_o:.6e}", flush=True)
    assert abs(fdc_g - fdc_o) <= FD_TOL * abs(oc)
    assert abs(gc - fdc_o) <= abs(fdc_o - oc) + FD_TOL * abs(oc)


def test_full_size_autofocus_gradient(api):
    # the autofocus workload at full size (256 pings x 16 receivers, 4096
    # samples, 1024 x 1024 pixels), in the 64 x 32 tiling its plan picks: the
    # cotangent lives on a seeded 2048-pixel subset, so the oracle's gradient
    # needs only those pixels; all 769 values of the autofocus parameters (the
    # per-ping platform position of a rigid array, dJ/dT_i + sum_e dJ/dR_ie,
    # and c) are compared, beyond the segment-choice bound
    from synth import subset_indices
    print("case c5 full size gradient", flush=True)
    scn = make_config("c5")
    echo = synthesize_echo(scn, device="cuda", dtype=torch.complex64)
    plan = api.sas_bp_plan([desc_for(api, scn)])
    info = plan.info()
    assert (info["tile_x"], info["tile_y"]) == (64, 32)
    buf = buffers_for(api, scn, echo)
    g = scn.grid
    idx = subset_indices(scn, 2048)
    rng = np.random.default_rng(17)
    vals = (rng.normal(size=idx.size) + 1j * rng.normal(size=idx.size)).astype(np.complex64)
    gbar = torch.zeros(g.n_pix, dtype=torch.complex64, device="cuda")
    gbar[torch.as_tensor(idx, device="cuda")] = torch.as_tensor(vals, device="cuda")
    gbar = gbar.reshape(g.n[2], g.n[1], g.n[0])
    gtx = torch.zeros((scn.n_ping, 3), dtype=torch.float64, device="cuda")
    grx = torch.zeros((scn.n_ping, scn.n_elem, 3), dtype=torch.float64, device="cuda")
    gc = torch.zeros(1, dtype=torch.float64, device="cuda")
    api.sas_bp_adjoint(plan, [buf], [gbar], [gtx], [grx], [gc])
    torch.cuda.synchronize()
    assert plan.status() == 0
    gpu = np.concatenate([(gtx.cpu().numpy() + grx.cpu().numpy().sum(axis=1)).ravel(), gc.cpu().numpy()])
    pts = oracle.pixel_points(g.origin, g.spacing, g.n, idx)
    args = (echo.cpu().numpy(), scn.tx, scn.rx, scn.c, scn.fc, scn.fs, scn.t0, pts, vals.astype(np.complex128))
    otx, orx, oc = oracle.vjp(*args)
    btx, brx, bc = oracle.vjp_segment_bound(*args, delta=SEG_DELTA)
    ref = np.concatenate([(otx + orx.sum(axis=1)).ravel(), [oc]])
    bnd = np.concatenate([(btx + brx.sum(axis=1)).ravel(), [bc]])
    assert gpu.size == 769
    ex_p = np.linalg.norm(np.maximum(np.abs(gpu[:-1] - ref[:-1]) - bnd[:-1], 0.0)) / np.linalg.norm(ref[:-1])
    ex_c = max(abs(gpu[-1] - ref[-1]) - bnd[-1], 0.0) / abs(ref[-1])
    print(f"[c5 full gradient] rel {_rel(gpu[:-1], ref[:-1]):.2e} (c {abs(gpu[-1] - ref[-1]) / abs(ref[-1]):.2e}); "
          f"beyond segment bound: positions {ex_p:.2e}, c {ex_c:.2e}", flush=True)
    assert np.linalg.norm(ref[:-1]) > 0
    assert ex_p <= GRAD_REL and ex_c <= GRAD_REL


def test_adjoint_is_deterministic(api):
    scn, echo, plan, buf, gbar, gtx, grx, gc = _grad_case(api, "c2", n_ping=30, n_elem=4, nx=70, ny=40,
                                                        n_sample=4096, n_scat=10, n_speckle=30)
    gtx2 = torch.zeros((scn.n_ping, 3), dtype=torch.float64, device="cuda")
    grx2 = torch.zeros((scn.n_ping, scn.n_elem, 3), dtype=torch.float64, device="cuda")
    gc2 = torch.zeros(1, dtype=torch.float64, device="cuda")
    for _ in range(2):
        api.sas_bp_adjoint(plan, [buf], [gbar], [gtx2], [grx2], [gc2])
        torch.cuda.synchronize()
        assert np.array_equal(gtx2.cpu().numpy(), gtx)
        assert np.array_equal(grx2.cpu().numpy(), grx)
        assert float(gc2.cpu()[0]) == gc


def test_sharpness_and_cotangent(api):
    scn = make_config("c5", n_ping=16, n_elem=4, nx=96, ny=64, n_scat=12)
    echo = synthesize_echo(scn, dtype=torch.complex64)
    plan = api.sas_bp_plan([desc_for(api, scn)])
    buf = buffers_for(api, scn, echo)
    api.sas_bp_image(plan, [buf])
    S = torch.zeros(1, dtype=torch.float64, device="cuda")
    G = torch.empty_like(buf.image)
    api.sas_bp_sharpness(plan, buf.image, S, G)
    torch.cuda.synchronize()
    img = buf.image.cpu().numpy()
    assert float(S.cpu()[0]) == pytest.approx(oracle.sharpness(img), rel=1e-12)
    gref = oracle.sharpness_cotangent(img)
    assert _rel(G.cpu().numpy(), gref) <= 1e-6
    # identities: one bright pixel -> 1, uniform magnitude over N pixels -> 1/N
    one = torch.zeros(1000, dtype=torch.complex64, device="cuda")
    one[123] = 3 - 2j
    api.sas_bp_sharpness(plan, one, S)
    torch.cuda.synchronize()
    assert float(S.cpu()[0]) == pytest.approx(1.0, rel=1e-12)
    uni = torch.polar(torch.full((777,), 2.0, device="cuda"), torch.linspace(0, 6, 777, device="cuda"))
    api.sas_bp_sharpness(plan, uni.to(torch.complex64), S)
    torch.cuda.synchronize()
    assert float(S.cpu()[0]) == pytest.approx(1.0 / 777, rel=1e-6)


def test_autograd_function(api):
    from paper_2101_05888_amd.autograd import tdbp_image
    scn = make_config("c5", n_ping=16, n_elem=4, nx=64, ny=48, n_scat=12)
    echo = synthesize_echo(scn, dtype=torch.complex64).cuda()
    plan = api.sas_bp_plan([desc_for(api, scn)])
    tx = torch.as_tensor(scn.tx, device="cuda").requires_grad_(True)
    rx = torch.as_tensor(scn.rx, device="cuda").requires_grad_(True)
    c = torch.tensor([scn.c], dtype=torch.float64, device="cuda").requires_grad_(True)
    img = tdbp_image(plan, echo, tx, rx, c)
    loss = (torch.view_as_real(img) ** 2).sum()     # cotangent exactly 2 I
    loss.backward()
    # same gradient through the C ABI directly
    gbar = (2.0 * img.detach()).to(torch.complex64)
    buf = buffers_for(api, scn, echo)
    gtx = torch.zeros_like(tx)
    grx = torch.zeros_like(rx)
    gc = torch.zeros_like(c)
    api.sas_bp_adjoint(plan, [buf], [gbar], [gtx], [grx], [gc])
    torch.cuda.synchronize()
    assert torch.equal(tx.grad, gtx)
    assert torch.equal(rx.grad, grx)
    assert torch.equal(c.grad, gc)
