#!/usr/bin/env python3
"""Benchmark: time-domain backprojection throughput on one MI355X.

Workload (the operational-size stripmap swath): 512 pings at 0.3 m spacing,
32 receivers at 3.75 cm pitch, 16384 complex samples per (ping, receiver)
(c = 1500 m/s, f_c = 100 kHz, B = 20 kHz, f_s = 80 kHz), a 4096 x 4096 pixel
image at 1.5 cm spacing over 20-81.4 m ground range, every receiver's
contribution gated to +-10 deg about broadside; 2000 point targets plus 1e5
weak speckle scatterers plus noise at 20 dB SNR, all seeded and synthetic.

A step is one call of ``sas_bp_image``: the captured graph runs the cull, the
cost ordering and the persistent image kernel over the whole swath, with the
echo cube, navigation and image already resident in HBM. The metric counts
useful pixel-ping-element updates (terms inside both beam cones), the count
coming from the library and checked against the oracle in the tests.

Printed: one JSON line (metric, value, roofline of the image kernel, the
FP16/BF16 echo forms with their speed-up and error, and the FP64 oracle timed
on the host cores on a bounded pixel sample).
"""
from __future__ import annotations

import argparse
import hashlib
import re
import json
import math
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3           # MI355X FP32 vector peak (256 CU x 2.4 GHz)
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "image_kernel_operational_swath_counters.txt")
METRIC = "pixel·ping·element updates/s; mixed vs FP32 at ≤1e-4 rel-L2 vs FP64 oracle"


def flops_per_update(n_elem: int) -> float:
    """Algorithmic FLOPs of one (pixel, ping, element) term of the sum, the
    cost model fixed before any tuning (an FMA counts 2, a transcendental 1):

    receiver displacement p - R (3), its squared norm (1 mul + 2 FMA: 5), the
    two legs summed (1), sample coordinate (tau - t0) f_s (1 FMA: 2), floor
    and fraction (2), carrier cycles f_c tau (1), complex lerp a + w (b - a)
    (2 sub + 2 FMA: 6), complex multiply-accumulate (4 FMA: 8), sqrt, sin and
    cos (3): 31, plus the transmitter leg (9) shared by the E elements.
    """
    return 31.0 + 9.0 / n_elem


IMAGE_KERNEL_SOURCES = ("tdbp_dev.h", "tdbp_geom.h", "tdbp_image.hip")
# Plan fields that fix the image kernel's launch (tile, chunking, LDS, grid,
# occupancy); the committed counters hold the values they were taken with.
LAUNCH_KEYS = ("tile_x", "tile_y", "tile_z", "pings_per_chunk", "window", "lds_bytes", "grid", "threads",
               "records_per_chunk", "workgroups_per_cu")


def _code_only(text: str) -> str:
    """Source text without comments and with whitespace collapsed."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_sources_digest() -> str:
    """SHA-256 over the code (comments and layout ignored) of the sources the
    image kernel is compiled from, to tell whether counters still describe it."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2101_05888_amd", "csrc")
    for fn in sorted(os.listdir(d)):
        if fn in IMAGE_KERNEL_SOURCES:
            h.update(fn.encode())
            with open(os.path.join(d, fn), encoding="utf-8") as f:
                h.update(_code_only(f.read()).encode())
    return h.hexdigest()


def launch_config_string(info: dict) -> str:
    return " ".join(f"{k}={int(info[k])}" for k in LAUNCH_KEYS)


def committed_counters(info: dict):
    """Key/value lines of the committed counter summary, or {} when the image
    kernel's code or its launch configuration (``info``, the plan's fields)
    differ from those the counters were taken with."""
    try:
        with open(TRAFFIC_SUMMARY) as f:
            kv = dict((k.strip(), v.strip()) for k, v in
                      (l.split(":", 1) for l in f.read().splitlines() if ":" in l and not l.startswith(" ")))
    except OSError:
        return {}
    if kv.get("kernel_sources_sha256") != kernel_sources_digest():
        return {}
    if kv.get("launch_config") != launch_config_string(info):
        return {}
    return kv


def issue_roofline(kernel_ms: float, info: dict):
    """Instruction-issue roofline of the image kernel: VALU wave-instructions
    per launch (committed counters) per CU clock (256 CUs at 2.4 GHz).

    The peak is the architectural FP32 VALU issue rate implied by the
    157.3 TFLOP/s vector peak: 157.3e12 / (2 flops x 64 lanes x 256 CUs x
    2.4 GHz) = 2 wave64 instructions per CU per clock, without packed math.
    Also reported against what independent FP32 FMA chains reach on this GPU
    (the issue_probe microbenchmark) at 8 waves per SIMD: 1.44 with one VGPR
    operand, 1.18 with three (1.00 with three at the 3 waves per SIMD the
    image kernel runs with)."""
    kv = committed_counters(info)
    try:
        valu = float(kv["valu_wave_instructions_per_launch"])
        trans = float(kv["trans_wave_instructions_per_launch"])
    except (KeyError, ValueError):
        return None
    rate = valu / (kernel_ms * 1e-3 * 2.4e9 * 256)
    peak = 2.0
    ceilings = {"fma_one_vgpr_operand_8_waves": 1.44, "fma_three_vgpr_operands_8_waves": 1.18,
                "fma_three_vgpr_operands_3_waves": 1.00}
    return {"valu_wave_instructions": valu, "trans_wave_instructions": trans,
            "achieved_wave_instr_per_cu_clock": rate, "peak_wave_instr_per_cu_clock": peak,
            "frac": rate / peak, "measured_fma_ceilings": ceilings,
            "frac_of_measured_ceilings": {k: rate / v for k, v in ceilings.items()}}


def measured_traffic(info: dict):
    """HBM bytes per image-kernel launch from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE scaled by the copy calibration), or None when the
    kernel or its launch configuration changed since the counters were taken."""
    try:
        return float(committed_counters(info)["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def oracle_workers() -> int:
    from oracle import pool
    return pool.get()[1]


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def time_steps(fn, steps: int, warmup: int) -> float:
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        fn()
    stop.record()
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / steps


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_leg(scn, echo_cpu: np.ndarray, images: dict, sample: int) -> dict:
    """Time the FP64 oracle on a seeded pixel sample on the host cores and
    compare every GPU form with it on the same pixels."""
    import oracle
    from oracle import pool
    from synth import subset_indices
    _, workers = pool.get()
    idx = subset_indices(scn, sample)
    g = scn.grid
    pts = oracle.pixel_points(g.origin, g.spacing, g.n, idx)
    t0 = time.perf_counter()
    ref, useful = oracle.backproject(echo_cpu, scn.tx, scn.rx, scn.c, scn.fc, scn.fs, scn.t0, pts,
                                     scn.gate_half_angle, workers=workers, return_count=True)
    dt = time.perf_counter() - t0
    acc = {}
    for name, img in images.items():
        got = img.reshape(-1)[idx]
        acc[name] = {"rel_l2": oracle.rel_l2(got, ref),
                     "max_phase_mrad": oracle.phase_error_mrad(got, ref),
                     "p99_phase_mrad": oracle.phase_error_mrad(got, ref, stat="p99")}
    return {"value": useful / dt, "unit": "updates/s", "cores": workers, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"{sample} seeded pixels of the same swath, all 512x32 (ping, element) terms "
                      f"evaluated and gated ({useful} useful updates) in {dt:.1f} s",
            "seconds": dt, "useful_updates": int(useful), "accuracy": acc}


def _buffers(api, scn, echo):
    g = scn.grid
    return api.SwathBuffers(
        echo=echo, tx=torch.as_tensor(scn.tx, device="cuda"), rx=torch.as_tensor(scn.rx, device="cuda"),
        c=torch.tensor([scn.c], dtype=torch.float64, device="cuda"),
        image=torch.empty((g.n[2], g.n[1], g.n[0]), dtype=torch.complex64, device="cuda"))


def _desc(api, scn):
    g = scn.grid
    return api.swath_desc(scn.n_ping, scn.n_elem, scn.n_sample, g.n, g.origin, g.spacing, scn.fc, scn.fs,
                          scn.t0, scn.gate_half_angle)


def reprojection_leg(api, plan, buf, useful: int, steps: int, warmup: int, forward_kernel_ms: float) -> dict:
    """Reprojection (the linear adjoint of the image in the echo) on the same
    swath and plan: the FP32 image as the image-side input, the whole echo cube
    as output. Also the adjoint identity <A x, y> = <x, A^H y> between the
    timed forward and adjoint at full size, in FP64 on the host."""
    y = buf.image.clone()
    out = torch.empty_like(buf.echo)
    api.sas_bp_set_kernel_timing(plan, True)
    for _ in range(warmup):
        api.sas_bp_reproject(plan, [buf], [y], [out])
    api.sas_bp_kernel_time(plan)
    ms = time_steps(lambda: api.sas_bp_reproject(plan, [buf], [y], [out]), steps, 0)
    k_total, k_n = api.sas_bp_kernel_time(plan)
    api.sas_bp_set_kernel_timing(plan, False)
    kms = k_total / k_n
    lhs = torch.vdot(buf.image.reshape(-1).to(torch.complex128), y.reshape(-1).to(torch.complex128)).item()
    rhs = torch.vdot(buf.echo.reshape(-1).to(torch.complex128), out.reshape(-1).to(torch.complex128)).item()
    ident = abs(lhs - rhs) / abs(lhs)
    log(f"reprojection: {ms:.3f} ms/call, kernel {kms:.3f} ms ({kms / forward_kernel_ms:.2f}x the image kernel), "
        f"adjoint identity {ident:.2e}")
    del out, y
    return {"ms_per_call": ms, "kernel_ms": kms, "useful_updates_per_s": useful / (kms * 1e-3),
            "vs_image_kernel": kms / forward_kernel_ms, "adjoint_identity_rel": ident,
            "note": "float atomics: not bitwise reproducible"}


def sinc_leg(api, scn, echo, useful: int, steps: int, warmup: int, forward_kernel_ms: float, sample: int) -> dict:
    """The windowed-sinc interpolation variant (8 taps) on the same swath:
    image kernel time, and its error against the oracle's sinc variant on a
    seeded pixel sample."""
    import oracle
    from synth import subset_indices
    d = _desc(api, scn)
    d.interp = 1
    plan = api.sas_bp_plan([d])
    buf = _buffers(api, scn, echo)
    api.sas_bp_set_kernel_timing(plan, True)
    for _ in range(warmup):
        api.sas_bp_image(plan, [buf])
    api.sas_bp_kernel_time(plan)
    ms = time_steps(lambda: api.sas_bp_image(plan, [buf]), steps, 0)
    k_total, k_n = api.sas_bp_kernel_time(plan)
    kms = k_total / k_n
    idx = subset_indices(scn, sample)
    got = buf.image.reshape(-1)[torch.as_tensor(idx, device="cuda")].cpu().numpy()
    g = scn.grid
    pts = oracle.pixel_points(g.origin, g.spacing, g.n, idx)
    ref = oracle.backproject(echo.cpu().numpy(), scn.tx, scn.rx, scn.c, scn.fc, scn.fs, scn.t0, pts,
                             scn.gate_half_angle, workers=oracle_workers(), interp="sinc")
    r, ph = oracle.rel_l2(got, ref), oracle.phase_error_mrad(got, ref)
    log(f"sinc8: {ms:.3f} ms/step, image kernel {kms:.3f} ms ({kms / forward_kernel_ms:.2f}x linear), "
        f"rel_l2 {r:.2e}, max phase {ph:.3f} mrad on {sample} pixels")
    plan.destroy()
    return {"interpolator": "Hann-windowed sinc, 8 taps", "ms_per_step": ms, "image_kernel_ms": kms,
            "useful_updates_per_s": useful / (kms * 1e-3), "vs_linear_kernel": kms / forward_kernel_ms,
            "rel_l2": r, "max_phase_mrad": ph, "sample_pixels": sample}


def motion_leg(api, scn, echo, useful: int, steps: int, warmup: int, forward_kernel_ms: float, sample: int,
               model: str = "velocity") -> dict:
    """Continuous receiver motion during reception on the same swath: the
    receivers moving at the track's 1.46 m/s (``velocity``), or displaced
    along an up-sampled position table (``table``: 2 ms samples, 1.5 m/s
    surge with millimetre sway and heave oscillations) during each ping's
    reception. Image kernel time, and its error against the oracle's exact
    delay root on a seeded pixel sample (same echo cube; the timing does not
    depend on it)."""
    import oracle
    from synth import subset_indices, receiver_velocity, receiver_track
    d = _desc(api, scn)
    buf = _buffers(api, scn, echo)
    if model == "table":
        tab, h = receiver_track(scn)
        d.motion, d.track_n, d.track_dt = 2, tab.shape[1], h
        buf.rx_track = torch.as_tensor(tab, dtype=torch.float64, device="cuda")
        kw = dict(rx_track=(tab, h))
        what = "receivers displaced along a position table (per ping and tile the line of the segment at the " \
               "centre's delay, certified within 2e-6 m; FP64 centre root, per-pixel Newton step)"
    else:
        vel = receiver_velocity(scn)
        d.motion = 1
        buf.rx_vel = torch.as_tensor(vel, dtype=torch.float64, device="cuda")
        kw = dict(rx_vel=vel)
        what = "receivers moving during reception (exact FP64 centre root, per-pixel Newton step)"
    plan = api.sas_bp_plan([d])
    api.sas_bp_set_kernel_timing(plan, True)
    for _ in range(warmup):
        api.sas_bp_image(plan, [buf])
    api.sas_bp_kernel_time(plan)
    ms = time_steps(lambda: api.sas_bp_image(plan, [buf]), steps, 0)
    k_total, k_n = api.sas_bp_kernel_time(plan)
    kms = k_total / k_n
    status = plan.status()
    idx = subset_indices(scn, sample)
    got = buf.image.reshape(-1)[torch.as_tensor(idx, device="cuda")].cpu().numpy()
    g = scn.grid
    pts = oracle.pixel_points(g.origin, g.spacing, g.n, idx)
    ref = oracle.backproject(echo.cpu().numpy(), scn.tx, scn.rx, scn.c, scn.fc, scn.fs, scn.t0, pts,
                             scn.gate_half_angle, workers=oracle_workers(), chunk=32, **kw)
    r, ph = oracle.rel_l2(got, ref), oracle.phase_error_mrad(got, ref)
    log(f"motion ({model}): {ms:.3f} ms/step, image kernel {kms:.3f} ms ({kms / forward_kernel_ms:.2f}x stop-and-hop), "
        f"rel_l2 {r:.2e}, max phase {ph:.3f} mrad on {sample} pixels, status {status}")
    plan.destroy()
    return {"model": what, "ms_per_step": ms, "image_kernel_ms": kms, "useful_updates_per_s": useful / (kms * 1e-3),
            "vs_stop_and_hop_kernel": kms / forward_kernel_ms, "rel_l2": r, "max_phase_mrad": ph,
            "sample_pixels": sample, "status": status}


def drc_leg(api, plan, image: torch.Tensor, steps: int, warmup: int) -> dict:
    """Dynamic range compression of the operational image (16.7 M pixels) for
    display at brightness 0.3: time, HBM bytes the algorithm moves (the image
    read five times: maximum, three radix-select passes and the map; the FP32
    output written once), and the largest difference from the FP64 oracle
    over the whole image."""
    import oracle
    n = image.numel()
    out = torch.empty(image.shape, dtype=torch.float32, device="cuda")
    prm = torch.zeros(3, dtype=torch.float64, device="cuda")
    ms = time_steps(lambda: api.sas_bp_drc(plan, image, 0.3, out, prm), steps, warmup)
    moved = 5 * n * 8 + n * 4
    ref, rp = oracle.drc(image.cpu().numpy().astype(np.complex128), 0.3)
    err = float(np.abs(out.cpu().numpy() - ref).max())
    log(f"drc: {ms:.3f} ms for {n} pixels, {moved / (ms * 1e-3) / 1e9:.0f} GB/s, max |out - oracle| {err:.1e}")
    return {"pixels": int(n), "ms": ms, "algorithmic_bytes": moved, "gb_per_s": moved / (ms * 1e-3) / 1e9,
            "hbm_peak_frac": moved / (ms * 1e-3) / 8e12, "max_abs_error_vs_oracle": err,
            "q": float(prm[2]), "median": float(prm[1])}


def tvg_leg(api, plan, echo: torch.Tensor, steps: int) -> dict:
    """Time-varying gain (Eq. 10) of the operational echo cube (512 x 32 x
    16384 complex samples, on a copy): time and the HBM bytes the algorithm
    moves (the cube read by three radix-select passes, then read and written
    by the gain)."""
    x = echo.clone()
    n = x.numel()
    api.sas_bp_tvg(plan, 0, x, 0.1)   # warm-up (also allocates the workspace)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        api.sas_bp_tvg(plan, 0, x, 0.1)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / steps
    moved = 5 * n * 8
    log(f"tvg: {ms:.3f} ms for {n} samples, {moved / (ms * 1e-3) / 1e9:.0f} GB/s")
    del x
    return {"samples": int(n), "ms": ms, "algorithmic_bytes": moved, "gb_per_s": moved / (ms * 1e-3) / 1e9,
            "hbm_peak_frac": moved / (ms * 1e-3) / 8e12}


def whiten_leg(api, plan, echo: torch.Tensor, steps: int) -> dict:
    """Spectral whitening (Eq. 9) of the operational echo cube on a copy:
    forward FFT, power estimate, gain, inverse FFT (16384 rows of 16384
    points; the hand-written two-pass form). Algorithmic bytes: the cube read
    and written twice (spectra in place between the passes)."""
    x = echo.clone()
    api.sas_bp_whiten(plan, 0, x, 0.1)   # warm-up (also makes the FFT plan)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        api.sas_bp_whiten(plan, 0, x, 0.1)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / steps
    moved = 4 * echo.numel() * 8
    log(f"whiten: {ms:.3f} ms for {x.numel()} samples, {moved / (ms * 1e-3) / 1e9:.0f} GB/s")
    del x
    return {"samples": int(echo.numel()), "ms": ms, "algorithmic_bytes": moved,
            "gb_per_s": moved / (ms * 1e-3) / 1e9, "hbm_peak_frac": moved / (ms * 1e-3) / 8e12}


def rangec_leg(api, plan, echo: torch.Tensor, fs: float, steps: int) -> dict:
    """Range compression and basebanding of the operational echo cube on a
    copy, with a 5 ms, 20 kHz linear-FM replica (400 taps): the fused
    overlap-save kernel (4096-point segments, 3697 outputs each, 5 per row).
    Algorithmic bytes: the cube read and written once."""
    from synth.waveform import lfm_replica
    x = echo.clone()
    q = torch.as_tensor(lfm_replica(20e3, 5e-3, fs).astype(np.complex64), device="cuda")
    api.sas_bp_range_compress(plan, 0, x, q)   # warm-up (also allocates the workspace)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        api.sas_bp_range_compress(plan, 0, x, q)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / steps
    n = x.numel()
    moved = 2 * n * 8
    log(f"range compression: {ms:.3f} ms for {n} samples, {moved / (ms * 1e-3) / 1e9:.0f} GB/s")
    del x
    return {"samples": int(n), "taps": int(q.numel()), "ms": ms, "samples_per_s": n / (ms * 1e-3),
            "algorithmic_bytes": moved, "gb_per_s": moved / (ms * 1e-3) / 1e9,
            "hbm_peak_frac": moved / (ms * 1e-3) / 8e12}


def dpc_tde_leg(api, plan, echo: torch.Tensor, steps: int) -> dict:
    """Time-delay estimation between consecutive pings of the operational cube
    for the DPC motion estimate: 16 element pairs (e + 16 of ping i, e of ping
    i + 1: the phase centres that coincide after the 0.3 m advance), 128-sample
    windows every 64 samples, lags to +-16: 511 ping pairs x 255 windows.
    Algorithmic bytes: both looks of every window read once."""
    pairs = [(e + 16, e) for e in range(16)]
    out = api.sas_bp_dpc_tde(plan, 0, echo, pairs, 128, 64, 16)   # warm-up (also allocates the pair buffer)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        api.sas_bp_dpc_tde(plan, 0, echo, pairs, 128, 64, 16, out=out)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / steps
    P1, K = out.shape[0], out.shape[1]
    macs = P1 * K * len(pairs) * 128 * 33
    moved = P1 * K * len(pairs) * (128 + 128 + 32) * 8
    sig = (out[..., 2] > 0.2).sum().item()
    log(f"dpc tde: {ms:.3f} ms for {P1 * K} windows ({sig} with rho > 0.2), "
        f"{macs * 8 / (ms * 1e-3) / 1e12:.1f} TFLOP/s of correlation, {moved / (ms * 1e-3) / 1e9:.0f} GB/s")
    return {"ping_pairs": P1, "windows": int(P1 * K), "element_pairs": len(pairs), "window": 128, "hop": 64,
            "max_lag": 16, "ms": ms, "windows_per_s": P1 * K / (ms * 1e-3),
            "correlation_tflops": macs * 8 / (ms * 1e-3) / 1e12, "algorithmic_bytes": moved,
            "gb_per_s": moved / (ms * 1e-3) / 1e9, "windows_rho_above_0.2": int(sig)}


def dpc_solve_leg(api, scn, tde: torch.Tensor, max_iter: int) -> dict:
    """The motion estimate on the operational cube's time-delay estimates:
    511 ping pairs x 255 windows (weights rho where rho > 0.5, else 0),
    footprints from the straight nominal track, surge 0.3 m per 0.2048 s
    ping interval, Huber loss; times the GPU residual pass and a bounded
    Levenberg-Marquardt solve (dense normal equations on the host). The echoes
    were synthesized stop-and-hop, so the estimate itself is not scored."""
    P, K = scn.n_ping, tde.shape[1]
    pri = scn.n_sample / scn.fs
    dt = np.full(P - 1, pri)
    vx = np.full(P, float(scn.tx[1, 0] - scn.tx[0, 0]) / pri)
    lever_rx = np.asarray(scn.rx[0] - scn.tx[0], dtype=np.float64)
    pairs = np.array([(e + 16, e) for e in range(16)], dtype=np.int32)
    t_ref = scn.t0 + (np.arange(K) * 64 + 64) / scn.fs
    est = tde.cpu().numpy().astype(np.float64)
    delay = est[..., 0]
    weight = np.where(est[..., 2] > 0.5, est[..., 2], 0.0)
    p0 = np.asarray(scn.tx[0], dtype=np.float64)
    d = api.dpc_desc(P, K, len(pairs), scn.n_elem, scn.c, 2e-6, 1e-2, 1.0, p0, (0.0, 0.0, 0.0), True, max_iter)
    nominal = np.column_stack([vx, np.zeros(P), np.zeros(P)])
    ps = api.sas_bp_dpc_footprints(d, nominal, dt, lever_rx, pairs, t_ref, 0.0, 1.0)   # seafloor at z = 0
    z_dvl = np.full(P, p0[2])
    pos, rows = api.sas_bp_dpc_residual(d, nominal, dt, lever_rx, pairs, t_ref, ps, delay)   # warm-up
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(5):
        api.sas_bp_dpc_residual(d, nominal, dt, lever_rx, pairs, t_ref, ps, delay)
    torch.cuda.synchronize()
    res_ms = (time.perf_counter() - t) / 5 * 1e3
    t = time.perf_counter()
    v, loss = api.sas_bp_dpc_solve(d, vx, dt, lever_rx, pairs, t_ref, ps, delay, weight, z_dvl, np.zeros((P, 2)))
    solve_s = time.perf_counter() - t
    log(f"dpc solve: residual pass {res_ms:.3f} ms (with transfers) for {(P - 1) * K} rows; "
        f"{max_iter}-iteration Huber solve over {2 * P} velocities {solve_s:.2f} s, loss {loss:.4e}, "
        f"{int((weight > 0).sum())} weighted windows")
    return {"rows": int((P - 1) * K), "unknowns": 2 * P, "residual_pass_ms": res_ms, "max_iter": max_iter,
            "solve_s": solve_s, "final_loss": loss, "weighted_windows": int((weight > 0).sum())}


def volume_leg(api, steps: int, warmup: int) -> dict:
    """The 3D workload at full size: 256 pings x 64 receivers (32 across x 2
    along), 8192 samples, 512 x 512 x 128 voxels at 2 cm, no gate. The seabed
    carries 5000 weak scatterers instead of 1e5 to keep synthesis short (the
    echo content does not change the work)."""
    from synth import make_config, synthesize_echo
    scn = make_config("c3", n_seabed=5000)
    echo = synthesize_echo(scn, device="cuda", dtype=torch.complex64, noise_on_device=True)
    plan = api.sas_bp_plan([_desc(api, scn)])
    buf = _buffers(api, scn, echo)
    updates = scn.nominal_updates()
    api.sas_bp_set_kernel_timing(plan, True)
    for _ in range(warmup):
        api.sas_bp_image(plan, [buf])
    api.sas_bp_kernel_time(plan)
    ms = time_steps(lambda: api.sas_bp_image(plan, [buf]), steps, 0)
    k_total, k_n = api.sas_bp_kernel_time(plan)
    kms = k_total / k_n
    info = plan.info()
    log(f"volume: {ms:.2f} ms/step, image kernel {kms:.2f} ms, {updates / (kms * 1e-3):.4e} updates/s, plan {info}")
    plan.destroy()
    # the same volume with the sediment-water interface (seabed at 5.5 m, sand at
    # 1650 m/s; the straight-path echo is reused: the timing does not depend on it)
    d = _desc(api, scn)
    d.refract, d.c_sediment, d.z_interface = 1, 1650.0, 5.5
    rplan = api.sas_bp_plan([d])
    api.sas_bp_set_kernel_timing(rplan, True)
    api.sas_bp_image(rplan, [buf])
    api.sas_bp_kernel_time(rplan)
    rms = time_steps(lambda: api.sas_bp_image(rplan, [buf]), 1, 0)
    r_total, r_n = api.sas_bp_kernel_time(rplan)
    rkms = r_total / r_n
    log(f"volume with sediment refraction: {rms:.2f} ms/step, kernel {rkms:.2f} ms "
        f"({rkms / kms:.1f}x straight paths), {updates / (rkms * 1e-3):.4e} updates/s")
    rplan.destroy()
    del echo, buf
    torch.cuda.empty_cache()
    return {"workload": "3D volume 512x512x128 voxels at 2 cm, 256 pings x 64 receivers, 8192 samples, no gate",
            "updates": int(updates), "ms_per_step": ms, "image_kernel_ms": kms,
            "updates_per_s": updates / (ms * 1e-3), "kernel_updates_per_s": updates / (kms * 1e-3),
            "tile": [info["tile_x"], info["tile_y"], info["tile_z"]], "records_per_chunk": info["records_per_chunk"],
            "workgroups_per_cu": info["workgroups_per_cu"],
            "refraction": {"c_sediment": 1650.0, "z_interface": 5.5, "ms_per_step": rms, "kernel_ms": rkms,
                           "kernel_updates_per_s": updates / (rkms * 1e-3), "vs_straight": rkms / kms}}


def autofocus_leg(api, steps: int, warmup: int) -> dict:
    """One autofocus iteration on the differentiable workload (256 pings x 16
    receivers, 1024 x 1024 pixels, no gate): image, sharpness and its
    cotangent, then the geometry adjoint."""
    from synth import make_config, synthesize_echo
    scn = make_config("c5")
    echo = synthesize_echo(scn, device="cuda", dtype=torch.complex64)
    plan = api.sas_bp_plan([_desc(api, scn)])
    buf = _buffers(api, scn, echo)
    S = torch.zeros(1, dtype=torch.float64, device="cuda")
    G = torch.empty_like(buf.image)
    gtx = torch.empty((scn.n_ping, 3), dtype=torch.float64, device="cuda")
    grx = torch.empty((scn.n_ping, scn.n_elem, 3), dtype=torch.float64, device="cuda")
    gc = torch.empty(1, dtype=torch.float64, device="cuda")
    fwd = time_steps(lambda: api.sas_bp_image(plan, [buf]), steps, warmup)
    sharp = time_steps(lambda: api.sas_bp_sharpness(plan, buf.image, S, G), steps, warmup)
    adj = time_steps(lambda: api.sas_bp_adjoint(plan, [buf], [G], [gtx], [grx], [gc]), steps, warmup)
    updates = scn.nominal_updates()
    log(f"autofocus: forward {fwd:.3f} ms, sharpness {sharp:.3f} ms, adjoint {adj:.3f} ms")
    # the whole autofocus from the nominal track: envelope then coherent ascent
    from paper_2101_05888_amd.autofocus import autofocus, default_stages, detrended_rms, line_of_sight_frame
    g = scn.grid
    tx0, rx0 = buf.tx.clone(), buf.rx.clone()
    truth = scn.true_tx - scn.tx
    centre = [g.origin[0] + 0.5 * (g.n[0] - 1) * g.spacing[0], g.origin[1] + 0.5 * (g.n[1] - 1) * g.spacing[1], 0.0]
    R = line_of_sight_frame(scn.tx, centre)
    torch.cuda.synchronize()
    t = time.perf_counter()
    res = autofocus(default_stages(plan, buf), tx0, rx0, frame=R)
    torch.cuda.synchronize()
    af_s = time.perf_counter() - t
    err = res.offsets - truth
    run = {"seconds": af_s, "evaluations": len(res.sharpness), "sharpness_start": res.sharpness[0],
           "sharpness_end": res.sharpness[-1],
           "error_mm_detrended": {"line_of_sight": float(detrended_rms((err @ R[1])[:, None])[0] * 1e3),
                                  "perpendicular": float(detrended_rms((err @ R[2])[:, None])[0] * 1e3),
                                  "y": float(detrended_rms(err[:, 1:2])[0] * 1e3),
                                  "z": float(detrended_rms(err[:, 2:3])[0] * 1e3)},
           "initial_error_mm_detrended": {"line_of_sight": float(detrended_rms((truth @ R[1])[:, None])[0] * 1e3),
                                          "y": float(detrended_rms(truth[:, 1:2])[0] * 1e3),
                                          "z": float(detrended_rms(truth[:, 2:3])[0] * 1e3)},
           "lambda_over_16_mm": 1e3 * scn.c / scn.fc / 16}
    log(f"autofocus run: {af_s:.1f} s, errors (mm) {run['error_mm_detrended']}")
    return {"workload": "256 pings x 16 receivers, 4096 samples, 1024x1024 px, no gate",
            "updates": int(updates), "forward_ms": fwd, "sharpness_ms": sharp, "adjoint_ms": adj,
            "forward_updates_per_s": updates / (fwd * 1e-3), "adjoint_updates_per_s": updates / (adj * 1e-3),
            "iteration_ms": fwd + sharp + adj, "autofocus": run}


def batched_leg(api, steps: int, warmup: int) -> dict:
    """24 swaths of uneven size in one persistent graph launch against 24
    separate plans launched one after the other on the same stream."""
    from synth import make_config, synthesize_echo
    scns = [make_config(f"c4b:{k}") for k in range(24)]
    echoes = [synthesize_echo(s, device="cuda", dtype=torch.complex64, noise_on_device=True) for s in scns]
    torch.cuda.synchronize()
    bufs = [_buffers(api, s, e) for s, e in zip(scns, echoes)]
    t = time.perf_counter()
    tuned = api.sas_bp_autotune([_desc(api, s) for s in scns], bufs, reps=2)
    tune_s = time.perf_counter() - t
    kw = {k: v for k, v in tuned.items() if k != "ms"}
    log(f"batched: autotuned {kw} in {tune_s:.1f} s")
    plan = api.sas_bp_plan([_desc(api, s) for s in scns], **kw)
    useful = sum(api.sas_bp_useful_updates(plan, bufs))
    one = time_steps(lambda: api.sas_bp_image(plan, bufs), steps, warmup)
    plans = [api.sas_bp_plan([_desc(api, s)], **kw) for s in scns]

    def separate():
        for p, b in zip(plans, bufs):
            api.sas_bp_image(p, [b])

    sep = time_steps(separate, steps, warmup)
    log(f"batched: one launch {one:.2f} ms, 24 launches {sep:.2f} ms, useful {useful:.3e}")
    nominal = sum(s.nominal_updates() for s in scns)
    for p in plans:
        p.destroy()
    plan.destroy()
    return {"workload": "24 swaths, sides U{512..4096} px, 128-512 pings, 16-32 receivers, +-10 deg gate",
            "useful_updates": int(useful), "nominal_updates": int(nominal),
            "tiling": {"tile": list(kw["tile"]), "threads": kw["threads"], "pings_per_chunk": kw["pings_per_chunk"],
                       "elems_per_chunk": kw["elems_per_chunk"]},
            "autotune_seconds": tune_s,
            "one_launch_ms": one, "separate_launches_ms": sep, "speedup": sep / one,
            "one_launch_updates_per_s": useful / (one * 1e-3)}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-sample", type=int, default=196608)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-autofocus", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-reprojection", action="store_true")
    ap.add_argument("--no-volume", action="store_true")
    ap.add_argument("--no-sinc", action="store_true")
    ap.add_argument("--no-drc", action="store_true")
    ap.add_argument("--no-tvg", action="store_true")
    ap.add_argument("--no-whiten", action="store_true")
    ap.add_argument("--no-rangec", action="store_true")
    ap.add_argument("--no-motion", action="store_true")
    ap.add_argument("--no-dpc", action="store_true")
    ap.add_argument("--profile", action="store_true", help="few steps, no CPU leg (for rocprofv3 runs)")
    ap.add_argument("--profile-leg", choices=["rangec", "tvg", "drc", "whiten", "dpc", "volume", "autofocus", "mixed", "sinc"], default=None,
                    help="with --profile, also run this one leg")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        return 2
    if args.profile:
        args.no_cpu_baseline = args.no_autofocus = args.no_batched = args.no_mixed = True
        args.no_reprojection = args.no_volume = args.no_sinc = args.no_drc = args.no_tvg = args.no_whiten = args.no_rangec = args.no_motion = args.no_dpc = True
        if args.profile_leg:
            setattr(args, "no_" + args.profile_leg, False)
    if not (args.no_cpu_baseline and args.no_sinc and args.no_motion):
        # the oracle's worker processes are forked now, before this process
        # initialises the GPU runtime (it never forks afterwards)
        from oracle import pool
        pool.start()
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no HIP device visible"}), flush=True)
        return 3

    import paper_2101_05888_amd as api
    from synth import make_config, synthesize_echo, quantize_echo

    scn = make_config("c2")
    log("synthesizing echoes")
    t = time.perf_counter()
    echo = synthesize_echo(scn, device="cuda", dtype=torch.complex64)
    torch.cuda.synchronize()
    log(f"synthesized {tuple(echo.shape)} in {time.perf_counter() - t:.1f} s")
    g = scn.grid

    def make(echo_t, kind="c64", scale=None):
        d = api.swath_desc(scn.n_ping, scn.n_elem, scn.n_sample, g.n, g.origin, g.spacing, scn.fc, scn.fs,
                           scn.t0, scn.gate_half_angle, kind)
        plan = api.sas_bp_plan([d])
        buf = api.SwathBuffers(
            echo=echo_t, tx=torch.as_tensor(scn.tx, device="cuda"), rx=torch.as_tensor(scn.rx, device="cuda"),
            c=torch.tensor([scn.c], dtype=torch.float64, device="cuda"),
            image=torch.empty((g.n[2], g.n[1], g.n[0]), dtype=torch.complex64, device="cuda"),
            echo_scale=scale)
        return plan, buf

    if args.profile:
        # calibration for the HBM byte counters: one elementwise kernel that
        # reads and writes exactly 256 MiB each (torch.neg, a kernel nothing
        # else in this program launches)
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
    plan, buf = make(echo)
    useful = api.sas_bp_useful_updates(plan, [buf])[0]
    nominal = scn.nominal_updates()
    info = plan.info()
    log(f"plan {info}; useful updates {useful} of {nominal}")
    # Timed region: the image kernel is bracketed by HIP events on the launch
    # stream (the library then enqueues the cull, ordering and image kernels
    # directly instead of replaying its graph).
    api.sas_bp_set_kernel_timing(plan, True)
    for _ in range(args.warmup):
        api.sas_bp_image(plan, [buf])
    api.sas_bp_kernel_time(plan)
    ms = time_steps(lambda: api.sas_bp_image(plan, [buf]), args.steps, 0)
    k_total, k_launches = api.sas_bp_kernel_time(plan)
    api.sas_bp_set_kernel_timing(plan, False)
    kernel_ms = k_total / k_launches
    graph_ms = time_steps(lambda: api.sas_bp_image(plan, [buf]), args.steps, 1)
    if plan.status() != 0:
        log("device reported bad navigation")
        return 4
    value = useful / (ms * 1e-3)
    log(f"fp32: {ms:.3f} ms/step ({graph_ms:.3f} ms as a graph replay), image kernel {kernel_ms:.3f} ms, "
        f"{value:.4e} useful updates/s")
    fpu = flops_per_update(scn.n_elem)
    achieved = useful * fpu / (kernel_ms * 1e-3) / 1e12
    images = {"fp32": buf.image.cpu().numpy()}

    out = {
        "metric": METRIC, "value": value, "unit": "updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "stripmap swath 4096x4096 px at 1.5 cm, 512 pings x 32 receivers, "
                               "16384 samples, +-10 deg tx/rx gate, 2000 targets + 1e5 speckle",
                   "pings": scn.n_ping, "elements": scn.n_elem, "samples": scn.n_sample,
                   "pixels": g.n_pix, "useful_updates": int(useful), "nominal_updates": int(nominal),
                   "tile": [info["tile_x"], info["tile_y"], info["tile_z"]],
                   "records_per_chunk": info["records_per_chunk"], "grid": info["grid"],
                   "workgroups_per_cu": info["workgroups_per_cu"]},
        "nominal_updates_per_s": nominal / (ms * 1e-3),
        "graph_ms_per_step": graph_ms,
        "image_kernel_ms": kernel_ms,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": measured_traffic(info),
                     "flops_per_update": fpu, "kernel": "image_kernel", "launch_ms": kernel_ms,
                     "updates_per_launch": int(useful)},
        "issue_roofline": issue_roofline(kernel_ms, info),
    }

    if not args.no_mixed:
        mixed = {}
        for kind in ("f16", "bf16"):
            q, scale = quantize_echo(echo, kind)
            p2, b2 = make(q, kind, scale.cuda())
            ms2 = time_steps(lambda: api.sas_bp_image(p2, [b2]), args.steps, args.warmup)
            mixed[kind] = {"value": useful / (ms2 * 1e-3), "ms_per_step": ms2, "speedup_vs_fp32": ms / ms2}
            images[kind] = b2.image.cpu().numpy()
            log(f"{kind}: {ms2:.3f} ms/step ({ms / ms2:.3f}x)")
            p2.destroy()
            del q, b2
        out["mixed"] = mixed

    if not args.no_drc:
        out["drc"] = drc_leg(api, plan, buf.image, max(3, args.steps // 4), 1)
    if not args.no_tvg:
        out["tvg"] = tvg_leg(api, plan, echo, 3)
    if not args.no_whiten:
        out["whiten"] = whiten_leg(api, plan, echo, 3)
    if not args.no_rangec:
        out["range_compression"] = rangec_leg(api, plan, echo, scn.fs, 3)
    if not args.no_dpc:
        out["dpc_tde"] = dpc_tde_leg(api, plan, echo, 3)
        tde = api.sas_bp_dpc_tde(plan, 0, echo, [(e + 16, e) for e in range(16)], 128, 64, 16)
        out["dpc_solve"] = dpc_solve_leg(api, scn, tde, 5)
    if not args.no_sinc:
        out["sinc8"] = sinc_leg(api, scn, echo, useful, max(3, args.steps // 4), 1, kernel_ms, 512)
    if not args.no_motion:
        out["motion"] = motion_leg(api, scn, echo, useful, max(3, args.steps // 4), 1, kernel_ms, 512)
        out["motion_table"] = motion_leg(api, scn, echo, useful, max(3, args.steps // 4), 1, kernel_ms, 512,
                                         model="table")
    if not args.no_reprojection:
        out["reprojection"] = reprojection_leg(api, plan, buf, useful, max(3, args.steps // 4), 1, kernel_ms)
    if not args.no_volume:
        out["volume"] = volume_leg(api, max(3, args.steps // 4), 1)
    if not args.no_autofocus:
        out["autofocus_step"] = autofocus_leg(api, args.steps, args.warmup)
    if not args.no_batched:
        out["batched"] = batched_leg(api, max(3, args.steps // 4), 1)

    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on the host cores")
        echo_cpu = echo.cpu().numpy()
        cb = cpu_baseline_leg(scn, echo_cpu, images, args.cpu_sample)
        acc = cb.pop("accuracy")
        out["cpu_baseline"] = cb
        out["accuracy_vs_oracle"] = acc
        for kind in out.get("mixed", {}):
            out["mixed"][kind].update(acc.get(kind, {}))
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
