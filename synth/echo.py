"""Echo synthesis from the point-scatterer forward model (Eq. 1, Sec. II-A).

Each receiver's time series is the sum over scatterers of a range-compressed,
basebanded return

    e[i, e, k] = sum_s  g_ie(x_s) * a_s * h(k - u_s) * exp(-j 2 pi f_c tau_s)

with tau_s = (|x_s - T_i| + |x_s - R_ie|) / c the two-way travel time and
u_s = (tau_s - t0) * f_s its position in samples. The pulse shape
h(d) = sinc(d * B / f_s) * taper(d) is the compressed pulse of bandwidth B,
truncated to |d| < H samples by a flat-top (Tukey) taper that equals 1 for
|d| <= H/2, so the two samples nearest the true delay carry the exact sinc.
With ``rx_vel`` (per-ping velocity [P, 3]) the receivers move during
reception, R_ie(t) = R_ie + v_i t (t after transmit; the transmitter is
stationary while it transmits), and tau_s solves
c tau = |x_s - T_i| + |x_s - R_ie - v_i tau|, found by fixed-point iteration
(contraction |v| / c). The gate stays that of the ping-time positions.
With ``rx_track = (table [P, N, 3], h)`` the receivers are displaced by the
table, R_ie(t) = R_ie + Delta_i(t), sampled every h seconds from transmit and
joined by straight lines (also beyond both ends); tau_s again by fixed-point
iteration.
With ``refraction = (c_sed, z_int)`` the seafloor z = z_int separates water
(sound speed c, above) from sediment (c_sed, below): a leg from an apex X
in the water to a scatterer below the interface crosses it at the point of
least travel time, found here by golden-section search along the vertical
plane through both (the travel time is convex there); legs to scatterers at
or above the interface are straight.
There is no spherical spreading: time-varying gain is taken as already applied
(Eq. 10, Sec. II-E). The gate g is the +-theta transmit AND receive cone about
the broadside plane, the same one the imager applies; g = 1 when no gate.

Arithmetic runs in float64 on any torch device; the result is cast to the
requested complex dtype. On a GPU the scatter-add uses atomics, so repeated
syntheses agree only to rounding; every comparison in this repository feeds the
same materialised cube to both sides.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from .scenario import Scenario


def _taper(d: torch.Tensor, half: int) -> torch.Tensor:
    a = d.abs()
    flat = half / 2.0
    w = 0.5 * (1.0 + torch.cos(math.pi * (a - flat) / flat))
    w = torch.where(a <= flat, torch.ones_like(w), w)
    return torch.where(a < half, w, torch.zeros_like(w))


def _leg_time(X: torch.Tensor, p: torch.Tensor, c: float, refraction: tuple) -> torch.Tensor:
    """One-way travel time from X (water) to p across the flat interface
    z = z_int (golden-section search over the crossing point's horizontal
    distance r from X along the vertical plane through X and p)."""
    c_sed, z_int = float(refraction[0]), float(refraction[1])
    X, p = torch.broadcast_tensors(X, p)
    D = torch.linalg.norm(p[..., :2] - X[..., :2], dim=-1)
    h1 = z_int - X[..., 2]
    h2 = p[..., 2] - z_int
    below = h2 > 0
    h2c = torch.clamp(h2, min=0.0)
    t_of = lambda r: torch.sqrt(r * r + h1 * h1) / c + torch.sqrt((D - r) ** 2 + h2c * h2c) / c_sed
    lo, hi = torch.zeros_like(D), D.clone()
    g = (math.sqrt(5.0) - 1.0) / 2.0
    a = hi - g * (hi - lo)
    b = lo + g * (hi - lo)
    ta, tb = t_of(a), t_of(b)
    for _ in range(90):
        left = ta < tb
        hi = torch.where(left, b, hi)
        lo = torch.where(left, lo, a)
        b_new = torch.where(left, a, lo + g * (hi - lo))
        a_new = torch.where(left, hi - g * (hi - lo), b)
        tb_new = torch.where(left, ta, t_of(b_new))
        ta_new = torch.where(left, t_of(a_new), tb)
        a, b, ta, tb = a_new, b_new, ta_new, tb_new
    t_ref = t_of(0.5 * (lo + hi))
    straight = torch.linalg.norm(p - X, dim=-1) / c
    return torch.where(below, t_ref, straight)


def _track_at(table: torch.Tensor, h: float, t: torch.Tensor) -> torch.Tensor:
    """Displacement of each ping's table [p, N, 3] at times t [p, ...] (sample
    j at j h, straight lines between samples and beyond both ends)."""
    n = table.shape[1]
    u = t / h
    j = torch.clamp(torch.floor(u), 0, n - 2).to(torch.int64)
    f = (u - j.to(u.dtype))[..., None]
    flat = j.reshape(j.shape[0], -1)                                           # [p, M]
    a = torch.gather(table, 1, flat[..., None].expand(-1, -1, 3))
    b = torch.gather(table, 1, (flat + 1)[..., None].expand(-1, -1, 3))
    a = a.reshape(*j.shape, 3)
    b = b.reshape(*j.shape, 3)
    return a + f * (b - a)


def pulse(d, bandwidth: float, fs: float, half: int):
    """Compressed pulse h(d) at offset d samples from the true delay (numpy or torch)."""
    if isinstance(d, np.ndarray):
        return pulse(torch.from_numpy(d), bandwidth, fs, half).numpy()
    return torch.sinc(d * (bandwidth / fs)) * _taper(d, half)


def synthesize_echo(scn: Scenario, device="cpu", dtype=torch.complex128,
                    tx: np.ndarray | None = None, rx: np.ndarray | None = None,
                    max_chunk: int = 1 << 22, noise: bool = True, noise_on_device: bool = False,
                    rx_vel: np.ndarray | None = None, refraction: tuple | None = None,
                    rx_track: tuple | None = None) -> torch.Tensor:
    """Echo cube [P, E, N_s] for the scenario, optionally with its seeded noise.

    ``tx``/``rx`` default to the positions the scene was recorded with
    (``scn.synth_tx()``), which differ from the imager's navigation only in the
    autofocus workload.
    """
    tx = scn.synth_tx() if tx is None else tx
    rx = scn.synth_rx() if rx is None else rx
    P, E, Ns = tx.shape[0], rx.shape[1], scn.n_sample
    rdt = torch.float64 if dtype == torch.complex128 else torch.float32
    dev = torch.device(device)
    out = torch.zeros(P * E * Ns, 2, dtype=rdt, device=dev)
    f64 = torch.float64
    pos = torch.as_tensor(scn.scat_pos, dtype=f64, device=dev)
    amp = torch.as_tensor(scn.scat_amp, dtype=torch.complex128, device=dev)
    txd = torch.as_tensor(tx, dtype=f64, device=dev)
    rxd = torch.as_tensor(rx, dtype=f64, device=dev)
    veld = None if rx_vel is None else torch.as_tensor(rx_vel, dtype=f64, device=dev)
    trk = None if rx_track is None else torch.as_tensor(np.asarray(rx_track[0]), dtype=f64, device=dev)
    trk_h = None if rx_track is None else float(rx_track[1])
    H = int(scn.taper_half)
    taps = torch.arange(-H + 1, H + 1, device=dev, dtype=f64)
    sin_g = math.sin(scn.gate_half_angle) if scn.gate_half_angle > 0 else None
    S = pos.shape[0]
    # pings per pass bounded so that [S, E] intermediates stay modest
    pp = max(1, min(P, (1 << 24) // max(1, S * E)))
    for i0 in range(0, P, pp):
        i1 = min(P, i0 + pp)
        T = txd[i0:i1]                                  # [p,3]
        R = rxd[i0:i1]                                  # [p,E,3]
        dT = torch.linalg.norm(pos[None, :, :] - T[:, None, :], dim=-1)              # [p,S]
        dR = torch.linalg.norm(pos[None, :, None, :] - R[:, None, :, :], dim=-1)     # [p,S,E]
        tau = (dT[:, :, None] + dR) / scn.c                                           # [p,S,E]
        if refraction is not None:
            tT = _leg_time(T[:, None, :], pos[None, :, :], scn.c, refraction)           # [p,S]
            tR = _leg_time(R[:, None, :, :], pos[None, :, None, :], scn.c, refraction)  # [p,S,E]
            tau = tT[:, :, None] + tR
        if trk is not None:
            Tk = trk[i0:i1]                                                           # [p,N,3]
            rel = pos[None, :, None, :] - R[:, None, :, :]                            # [p,S,E,3]
            for _ in range(8):
                moved = rel - _track_at(Tk, trk_h, tau)
                tau = (dT[:, :, None] + torch.linalg.norm(moved, dim=-1)) / scn.c
        if veld is not None:
            V = veld[i0:i1]                                                           # [p,3]
            rel = pos[None, :, None, :] - R[:, None, :, :]                            # [p,S,E,3]
            for _ in range(8):
                moved = rel - V[:, None, None, :] * tau[..., None]
                tau = (dT[:, :, None] + torch.linalg.norm(moved, dim=-1)) / scn.c
        if sin_g is not None:
            gT = (pos[None, :, 0] - T[:, None, 0]).abs() <= sin_g * dT               # [p,S]
            gR = (pos[None, :, None, 0] - R[:, None, :, 0]).abs() <= sin_g * dR       # [p,S,E]
            keep = gT[:, :, None] & gR
        else:
            keep = torch.ones_like(tau, dtype=torch.bool)
        ip, isc, ie = torch.nonzero(keep, as_tuple=True)
        if ip.numel() == 0:
            continue
        step = max(1, max_chunk // (2 * H))
        for j0 in range(0, ip.numel(), step):
            a_p, a_s, a_e = ip[j0:j0 + step], isc[j0:j0 + step], ie[j0:j0 + step]
            t = tau[a_p, a_s, a_e]
            u = (t - scn.t0) * scn.fs
            k = torch.floor(u)[:, None] + taps[None, :]                 # [M, 2H]
            h = pulse(k - u[:, None], scn.bandwidth, scn.fs, H)
            cyc = torch.frac(scn.fc * t)
            ph = torch.polar(torch.ones_like(cyc), -2.0 * math.pi * cyc)
            val = (amp[a_s] * ph)[:, None] * h                           # complex128 [M,2H]
            ki = k.to(torch.int64)
            ok = (ki >= 0) & (ki < Ns)
            flat = ((a_p + i0) * E + a_e)[:, None] * Ns + ki
            flat = flat[ok]
            v = torch.view_as_real(val[ok]).to(rdt)
            out.index_add_(0, flat, v)
    echo = torch.view_as_complex(out.view(P, E, Ns, 2))
    if noise and scn.snr_db is not None:
        echo = add_noise(echo, scn, on_device=noise_on_device)
    return echo


def add_noise(echo: torch.Tensor, scn: Scenario, on_device: bool = False) -> torch.Tensor:
    """Add CN(0, sigma^2) noise, sigma^2 = mean |signal|^2 over the cube / 10^(SNR/10).

    By default the noise is drawn on the CPU from a torch generator seeded from
    the scenario's noise stream, one ping at a time, so it is the same whatever
    device the cube lives on. ``on_device`` draws it with a generator on the
    cube's device instead (same seed, different stream of numbers): much faster
    for cubes of many gigabytes.
    """
    p_sig = float((echo.real.double() ** 2 + echo.imag.double() ** 2).mean())
    sigma = math.sqrt(p_sig / (10.0 ** (scn.snr_db / 10.0)))
    seed = int(scn.streams()["noise"].integers(0, 2 ** 62))
    gdev = echo.device if on_device else torch.device("cpu")
    g = torch.Generator(device=gdev).manual_seed(seed)
    rdt = torch.float64 if echo.dtype == torch.complex128 else torch.float32
    s = sigma / math.sqrt(2.0)
    er = torch.view_as_real(echo)
    for i in range(echo.shape[0]):
        n = torch.randn(er.shape[1:], generator=g, dtype=torch.float32, device=gdev).to(rdt) * s
        er[i] += n.to(echo.device)
    return echo


# ----------------------------------------------------------- quantisation ---

QUANT_K = {"f16": 2.0 ** 15, "bf16": 1.0}


def quantize_echo(echo: torch.Tensor, kind: str):
    """Per-ping max-abs scaling to FP16 or BF16 storage.

    s_i = max over elements, samples and {Re, Im} of the component magnitude of
    ping i; stored = round_to_nearest_even(echo * K / s_i) with K = 2^15 (FP16,
    keeps values below 65504 and far above the subnormal range) or 1 (BF16).
    Returns (stored [P,E,N_s,2] in the 16-bit type, dequantisation scale f32[P]
    equal to s_i / K).
    """
    K = QUANT_K[kind]
    tdt = torch.float16 if kind == "f16" else torch.bfloat16
    er = torch.view_as_real(echo)
    P = er.shape[0]
    s = er.abs().reshape(P, -1).amax(dim=1).double()
    s = torch.where(s > 0, s, torch.ones_like(s))
    mult = (K / s).to(er.dtype)
    q = (er * mult[:, None, None, None]).to(tdt)
    scale = (s / K).to(torch.float32)
    return q.contiguous(), scale


def dequantize_echo(q: torch.Tensor, scale: torch.Tensor, dtype=torch.complex128) -> torch.Tensor:
    rdt = torch.float64 if dtype == torch.complex128 else torch.float32
    v = q.to(rdt) * scale.to(rdt)[:, None, None, None]
    return torch.view_as_complex(v.contiguous())
