"""Shared test plumbing: scenario -> C-ABI descriptors/buffers, oracle calls."""
from __future__ import annotations

import os

import numpy as np
import torch

import oracle
from synth import Scenario, synthesize_echo, quantize_echo, dequantize_echo

# FP32 path bounds against the FP64 oracle (relative L2 over the compared
# pixels; phase over pixels within 30 dB of the reference peak).
FP32_REL_L2 = 1e-4
FP32_PHASE_MRAD = 10.0
# 16-bit echo storage, error against the oracle on the original FP32 echo.
# Derivation: per-component relative rounding ~u/sqrt(3) of the ping's peak
# with u = 2^-11 (FP16) or 2^-8 (BF16) gives about 2.8e-4 and 2.3e-3 relative
# L2 for these scenes; the bounds leave a factor of ~2-3.
F16_REL_L2, F16_PHASE_MRAD = 1e-3, 30.0
BF16_REL_L2, BF16_PHASE_MRAD = 5e-3, 100.0


def workers() -> int:
    """Workers of the oracle's pool (started by the test session before any GPU call)."""
    from oracle import pool
    return pool.default_workers()


def desc_for(api, scn: Scenario, echo_dtype: str = "c64", c_min: float = 0.0, interp: str = "linear",
             motion=False, refraction=None, track=None):
    g = scn.grid
    return api.swath_desc(scn.n_ping, scn.n_elem, scn.n_sample, g.n, g.origin, g.spacing,
                          scn.fc, scn.fs, scn.t0, scn.gate_half_angle, echo_dtype, c_min, interp, motion,
                          refraction, track)


def buffers_for(api, scn: Scenario, echo: torch.Tensor, device="cuda", echo_scale=None,
                tx=None, rx=None, c=None, rx_vel=None, rx_track=None):
    g = scn.grid
    dev = torch.device(device)
    tx = scn.tx if tx is None else tx
    rx = scn.rx if rx is None else rx
    return api.SwathBuffers(
        echo=echo.to(dev).contiguous(),
        tx=torch.as_tensor(np.ascontiguousarray(tx), dtype=torch.float64, device=dev),
        rx=torch.as_tensor(np.ascontiguousarray(rx), dtype=torch.float64, device=dev),
        c=torch.tensor([scn.c if c is None else c], dtype=torch.float64, device=dev),
        image=torch.zeros((g.n[2], g.n[1], g.n[0]), dtype=torch.complex64, device=dev),
        echo_scale=None if echo_scale is None else echo_scale.to(dev).contiguous(),
        rx_vel=None if rx_vel is None else torch.as_tensor(np.ascontiguousarray(rx_vel), dtype=torch.float64,
                                                           device=dev),
        rx_track=None if rx_track is None else torch.as_tensor(np.ascontiguousarray(rx_track), dtype=torch.float64,
                                                               device=dev),
    )


def gpu_image(api, scn: Scenario, echo: torch.Tensor, echo_dtype="c64", echo_scale=None, interp="linear",
              rx_vel=None, refraction=None, rx_track=None, **plan_kw):
    motion = "table" if rx_track is not None else rx_vel is not None
    track = None if rx_track is None else (rx_track[0].shape[1], rx_track[1])
    plan = api.sas_bp_plan([desc_for(api, scn, echo_dtype, interp=interp, motion=motion, refraction=refraction,
                                     track=track)], **plan_kw)
    buf = buffers_for(api, scn, echo, echo_scale=echo_scale, rx_vel=rx_vel,
                      rx_track=None if rx_track is None else rx_track[0])
    api.sas_bp_image(plan, [buf])
    torch.cuda.synchronize()
    assert plan.status() == 0
    return buf.image.cpu().numpy(), plan, buf


def oracle_image(scn: Scenario, echo_np: np.ndarray, index=None, interp="linear", rx_vel=None, refraction=None,
                 chunk=4096, rx_track=None):
    g = scn.grid
    pts = oracle.pixel_points(g.origin, g.spacing, g.n, index)
    return oracle.backproject(echo_np, scn.tx, scn.rx, scn.c, scn.fc, scn.fs, scn.t0, pts,
                              scn.gate_half_angle, workers=workers(), chunk=chunk,
                              interp="sinc" if interp == "sinc8" else interp, rx_vel=rx_vel, refraction=refraction,
                              rx_track=rx_track)


def volume_subset(scn: Scenario, count: int, seabed_z: float) -> np.ndarray:
    """Seeded voxel subset (flat indices, sorted, unique) of a volume: half
    drawn uniformly, a quarter from the seven voxel planes around the seabed
    and a quarter from the outer tenth of the footprint on either horizontal
    axis (large horizontal offsets from the array)."""
    g = scn.grid
    nx, ny, nz = (int(v) for v in g.n)
    rng = scn.streams()["subset"]
    uni = rng.choice(nx * ny * nz, count // 2, replace=False)
    q = count // 4
    kz = int(round((seabed_z - g.origin[2]) / g.spacing[2]))
    zs = rng.integers(max(0, kz - 3), min(nz, kz + 4), q)
    sea = (zs * ny + rng.integers(0, ny, q)) * nx + rng.integers(0, nx, q)
    bx, by = max(1, nx // 10), max(1, ny // 10)
    ex = rng.integers(0, 2 * bx, q)
    ex = np.where(ex < bx, ex, nx - 2 * bx + ex)
    ey = rng.integers(0, 2 * by, q)
    ey = np.where(ey < by, ey, ny - 2 * by + ey)
    on_x = rng.random(q) < 0.5
    ix = np.where(on_x, ex, rng.integers(0, nx, q))
    iy = np.where(on_x, rng.integers(0, ny, q), ey)
    edge = (rng.integers(0, nz, q) * ny + iy) * nx + ix
    return np.unique(np.concatenate([uni, sea, edge]).astype(np.int64))


def report(name, img, ref):
    r = oracle.rel_l2(img, ref)
    ph = oracle.phase_error_mrad(img, ref)
    print(f"[{name}] rel_l2={r:.3e} max_phase={ph:.3f} mrad", flush=True)
    return r, ph
