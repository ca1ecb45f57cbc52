"""Python binding of the C ABI, argument marshalling only.

Every function here has the name of the C entry point it calls and does no
arithmetic of the method: it checks tensor shapes, dtypes and devices, packs
the ctypes structures and forwards device pointers and the current HIP stream.
All computation happens in the HIP library.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import math
from typing import Optional, Sequence

import numpy as np
import torch

from . import _native as N
from ._native import check

ECHO_DTYPES = {"c64": N.ECHO_C64, "f16": N.ECHO_F16X2, "bf16": N.ECHO_BF16X2}
INTERPS = {"linear": N.INTERP_LINEAR, "sinc8": N.INTERP_SINC8}
TUNE_MODES = {"default": N.TUNE_DEFAULT, "cached": N.TUNE_CACHED, "search": N.TUNE_SEARCH}


def swath_desc(n_ping: int, n_elem: int, n_sample: int, n: Sequence[int], origin: Sequence[float],
               spacing: Sequence[float], f_c: float, f_s: float, t0: float = 0.0,
               gate_half_angle: float = 0.0, echo_dtype: str = "c64", c_min: float = 0.0,
               interp: str = "linear", motion=False, refraction=None, track=None) -> N.SwathDesc:
    """Descriptor of one swath; ``interp`` is "linear" or "sinc8" (the
    Hann-windowed sinc over 8 samples); ``motion`` selects receivers moving
    during reception: True or "velocity" (``SwathBuffers.rx_vel``), or
    "table" with ``track`` = (samples per ping, seconds between samples) for
    an up-sampled position table (``SwathBuffers.rx_track``); ``refraction``
    = (c_sediment, z_interface) a sediment-water interface in the
    propagation time."""
    if interp not in INTERPS:
        raise ValueError(f"interp must be one of {sorted(INTERPS)}")
    d = N.SwathDesc()
    d.n_ping, d.n_elem, d.n_sample = int(n_ping), int(n_elem), int(n_sample)
    d.echo_dtype = ECHO_DTYPES[echo_dtype]
    for a in range(3):
        d.n[a] = int(n[a])
        d.origin[a] = float(origin[a])
        d.spacing[a] = float(spacing[a])
    d.f_c, d.f_s, d.t0 = float(f_c), float(f_s), float(t0)
    d.gate_half_angle, d.c_min = float(gate_half_angle), float(c_min)
    d.interp = INTERPS[interp]
    if motion == "table":
        if track is None:
            raise ValueError("motion='table' needs track=(samples per ping, seconds between samples)")
        d.motion, d.track_n, d.track_dt = 2, int(track[0]), float(track[1])
    elif motion in (True, 1, "velocity"):
        d.motion = 1
    elif motion in (False, 0, None, "stop_and_hop"):
        d.motion = 0
    else:
        raise ValueError(f"unknown motion model {motion!r}")
    if refraction is not None:
        d.refract, d.c_sediment, d.z_interface = 1, float(refraction[0]), float(refraction[1])
    return d


def _options(device=0, tile=(0, 0, 0), pings_per_chunk=0, use_graph=True, workspace_limit=0,
             threads=0, elems_per_chunk=0, tune_mode="default", no_cull=False, tune_cache=None) -> N.Options:
    if tune_mode not in TUNE_MODES:
        raise ValueError(f"tune_mode must be one of {sorted(TUNE_MODES)}")
    o = N.Options()
    o.tune_mode = TUNE_MODES[tune_mode]
    o.no_cull = 1 if no_cull else 0
    o.tune_cache = None if tune_cache is None else str(tune_cache).encode()
    o.device = int(device)
    o.tile_x, o.tile_y, o.tile_z = (int(v) for v in tile)
    o.pings_per_chunk = int(pings_per_chunk)
    o.elems_per_chunk = int(elems_per_chunk)
    o.threads = int(threads)
    o.use_graph = 1 if use_graph else 0
    o.workspace_limit = int(workspace_limit)
    return o


class Plan:
    """Owns a ``sas_bp_plan_t``; released by ``destroy()`` or garbage collection."""

    def __init__(self, handle: int, descs: list, device: int):
        self.handle = C.c_void_p(handle)
        self.descs = descs
        self.device = device

    def info(self) -> dict:
        arr = (C.c_int64 * 10)()
        check(N.lib().sas_bp_plan_info(self.handle, arr), "sas_bp_plan_info")
        keys = ("tile_x", "tile_y", "tile_z", "pings_per_chunk", "window", "lds_bytes", "grid", "threads",
                "records_per_chunk", "workgroups_per_cu")
        return dict(zip(keys, (int(v) for v in arr)))

    def status(self) -> int:
        return int(N.lib().sas_bp_plan_status(self.handle))

    def destroy(self) -> None:
        if self.handle is not None and self.handle.value:
            N.lib().sas_bp_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def sas_bp_plan(descs: Sequence[N.SwathDesc], device: int = 0, tile=(0, 0, 0), pings_per_chunk: int = 0,
                use_graph: bool = True, workspace_limit: int = 0, threads: int = 0,
                elems_per_chunk: int = 0, tune_mode: str = "default", no_cull: bool = False,
                tune_cache=None) -> Plan:
    """``tune_mode`` "cached" or "search" takes the tiling stored for the shape
    class (process cache, then the ``tune_cache`` file); ``no_cull`` turns the
    block cull off (every ping of every tile, every record gated per row)."""
    descs = list(descs)
    arr = (N.SwathDesc * len(descs))(*descs)
    opt = _options(device, tile, pings_per_chunk, use_graph, workspace_limit, threads, elems_per_chunk,
                   tune_mode, no_cull, tune_cache)
    out = C.c_void_p()
    check(N.lib().sas_bp_plan(arr, len(descs), C.byref(opt), C.byref(out)), "sas_bp_plan")
    return Plan(out.value, descs, device)


def sas_bp_workspace_size(descs: Sequence[N.SwathDesc], tile=(0, 0, 0), pings_per_chunk: int = 0,
                          threads: int = 0, elems_per_chunk: int = 0, tune_mode: str = "default",
                          no_cull: bool = False, tune_cache=None) -> int:
    descs = list(descs)
    arr = (N.SwathDesc * len(descs))(*descs)
    opt = _options(0, tile, pings_per_chunk, threads=threads, elems_per_chunk=elems_per_chunk,
                   tune_mode=tune_mode, no_cull=no_cull, tune_cache=tune_cache)
    out = C.c_size_t()
    check(N.lib().sas_bp_workspace_size(arr, len(descs), C.byref(opt), C.byref(out)), "sas_bp_workspace_size")
    return int(out.value)


@dataclasses.dataclass
class SwathBuffers:
    """Device tensors of one swath (see ``sas_bp_swath_io`` in the header)."""
    echo: torch.Tensor                  # complex64 [P,E,N] or float16/bfloat16 [P,E,N,2]
    tx: torch.Tensor                    # float64 [P,3]
    rx: torch.Tensor                    # float64 [P,E,3]
    c: torch.Tensor                     # float64 [1]
    image: torch.Tensor                 # complex64 [nz,ny,nx]
    echo_scale: Optional[torch.Tensor] = None   # float32 [P] for 16-bit echoes
    rx_vel: Optional[torch.Tensor] = None       # float64 [P,3], receiver velocity (continuous motion)
    rx_track: Optional[torch.Tensor] = None     # float64 [P,N,3], receiver displacement table (motion "table")


def _need(t: torch.Tensor, name: str, dtype, shape, device) -> None:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on a HIP device (got {t.device})")
    if device is not None and t.device.index != device:
        raise ValueError(f"{name} is on device {t.device.index}, plan on {device}")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _io(plan: Plan, bufs: Sequence[SwathBuffers]):
    return _io_for(plan.descs, plan.device, bufs)


def _io_for(descs, device, bufs: Sequence[SwathBuffers]):
    if len(bufs) != len(descs):
        raise ValueError(f"plan has {len(descs)} swaths, got {len(bufs)} buffers")
    arr = (N.SwathIO * len(bufs))()
    for i, (d, b) in enumerate(zip(descs, bufs)):
        P, E, Ns = d.n_ping, d.n_elem, d.n_sample
        if d.echo_dtype == N.ECHO_C64:
            _need(b.echo, f"echo[{i}]", torch.complex64, (P, E, Ns), device)
        else:
            dt = torch.float16 if d.echo_dtype == N.ECHO_F16X2 else torch.bfloat16
            _need(b.echo, f"echo[{i}]", dt, (P, E, Ns, 2), device)
            _need(b.echo_scale, f"echo_scale[{i}]", torch.float32, (P,), device)
        _need(b.tx, f"tx[{i}]", torch.float64, (P, 3), device)
        _need(b.rx, f"rx[{i}]", torch.float64, (P, E, 3), device)
        _need(b.c, f"c[{i}]", torch.float64, (1,), device)
        _need(b.image, f"image[{i}]", torch.complex64, (d.n[2], d.n[1], d.n[0]), device)
        if d.motion == 1:
            _need(b.rx_vel, f"rx_vel[{i}]", torch.float64, (P, 3), device)
        if d.motion == 2:
            _need(b.rx_track, f"rx_track[{i}]", torch.float64, (P, d.track_n, 3), device)
        arr[i].echo = b.echo.data_ptr()
        arr[i].echo_scale = b.echo_scale.data_ptr() if b.echo_scale is not None else None
        arr[i].tx_pos = b.tx.data_ptr()
        arr[i].rx_pos = b.rx.data_ptr()
        arr[i].c = b.c.data_ptr()
        arr[i].image = b.image.data_ptr()
        arr[i].rx_vel = b.rx_vel.data_ptr() if b.rx_vel is not None else None
        arr[i].rx_track = b.rx_track.data_ptr() if b.rx_track is not None else None
    return arr


def _stream(device: int, stream=None) -> C.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return C.c_void_p(stream.cuda_stream)


def sas_bp_image(plan: Plan, bufs: Sequence[SwathBuffers], stream=None) -> None:
    arr = _io(plan, bufs)
    check(N.lib().sas_bp_image(plan.handle, arr, len(bufs), _stream(plan.device, stream)), "sas_bp_image")


def sas_bp_adjoint(plan: Plan, bufs: Sequence[SwathBuffers], grad_images: Sequence[torch.Tensor],
                   grad_tx: Sequence[torch.Tensor], grad_rx: Sequence[torch.Tensor],
                   grad_c: Sequence[torch.Tensor], stream=None) -> None:
    arr = _io(plan, bufs)
    n = len(bufs)
    for i, d in enumerate(plan.descs):
        _need(grad_images[i], f"grad_image[{i}]", torch.complex64, (d.n[2], d.n[1], d.n[0]), plan.device)
        _need(grad_tx[i], f"grad_tx[{i}]", torch.float64, (d.n_ping, 3), plan.device)
        _need(grad_rx[i], f"grad_rx[{i}]", torch.float64, (d.n_ping, d.n_elem, 3), plan.device)
        _need(grad_c[i], f"grad_c[{i}]", torch.float64, (1,), plan.device)
    P = C.c_void_p
    gi = (P * n)(*[t.data_ptr() for t in grad_images])
    gt = (P * n)(*[t.data_ptr() for t in grad_tx])
    gr = (P * n)(*[t.data_ptr() for t in grad_rx])
    gc = (P * n)(*[t.data_ptr() for t in grad_c])
    check(N.lib().sas_bp_adjoint(plan.handle, arr, gi, gt, gr, gc, n, _stream(plan.device, stream)),
          "sas_bp_adjoint")


def sas_bp_reproject(plan: Plan, bufs: Sequence[SwathBuffers], images_in: Sequence[torch.Tensor],
                     echoes_out: Sequence[torch.Tensor], stream=None) -> None:
    """Linear adjoint of the image with respect to the echo: echoes_out[s]
    (complex64 [P, E, N_s], overwritten) = A^H images_in[s]."""
    arr = _io(plan, bufs)
    n = len(bufs)
    for i, d in enumerate(plan.descs):
        _need(images_in[i], f"images_in[{i}]", torch.complex64, (d.n[2], d.n[1], d.n[0]), plan.device)
        _need(echoes_out[i], f"echoes_out[{i}]", torch.complex64, (d.n_ping, d.n_elem, d.n_sample), plan.device)
    P = C.c_void_p
    yi = (P * n)(*[t.data_ptr() for t in images_in])
    eo = (P * n)(*[t.data_ptr() for t in echoes_out])
    check(N.lib().sas_bp_reproject(plan.handle, arr, yi, eo, n, _stream(plan.device, stream)), "sas_bp_reproject")


def sas_bp_whiten(plan: Plan, swath: int, echo: torch.Tensor, gamma: float, stream=None) -> None:
    """Spectral whitening of a complex64 echo cube [P, E, N_s], in place."""
    d = plan.descs[swath]
    _need(echo, "echo", torch.complex64, (d.n_ping, d.n_elem, d.n_sample), plan.device)
    check(N.lib().sas_bp_whiten(plan.handle, int(swath), echo.data_ptr(), float(gamma),
                                _stream(plan.device, stream)), "sas_bp_whiten")


def sas_bp_range_compress(plan: Plan, swath: int, echo: torch.Tensor, replica: torch.Tensor, mix: bool = True,
                          stream=None) -> None:
    """Range compression (matched filter with the complex64 replica [M]) of a
    complex64 echo cube [P, E, N_s], in place; with mix the rows are first
    brought to baseband by exp(-j 2 pi f_c t)."""
    d = plan.descs[swath]
    _need(echo, "echo", torch.complex64, (d.n_ping, d.n_elem, d.n_sample), plan.device)
    if replica.dim() != 1:
        raise ValueError("replica must be one-dimensional")
    _need(replica, "replica", torch.complex64, (replica.shape[0],), plan.device)
    check(N.lib().sas_bp_range_compress(plan.handle, int(swath), echo.data_ptr(), replica.data_ptr(),
                                        int(replica.shape[0]), 1 if mix else 0, _stream(plan.device, stream)),
          "sas_bp_range_compress")


def sas_bp_dpc_tde(plan: Plan, swath: int, echo: torch.Tensor, pairs, win: int, hop: int, max_lag: int,
                   out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Time-delay estimation between consecutive pings over element pairs
    [(e1 of ping i, e2 of ping i + 1), ...]: returns float32 [P - 1, K, 4]
    (coarse delay s, phase rad, rho, peak lag) per ping pair and window."""
    d = plan.descs[swath]
    _need(echo, "echo", torch.complex64, (d.n_ping, d.n_elem, d.n_sample), plan.device)
    pr = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
    K = (d.n_sample - int(win)) // int(hop) + 1 if d.n_sample >= int(win) and int(hop) > 0 else 0
    if out is None:
        out = torch.empty((max(d.n_ping - 1, 0), max(K, 0), 4), dtype=torch.float32, device=echo.device)
    else:
        _need(out, "out", torch.float32, (d.n_ping - 1, K, 4), plan.device)
    check(N.lib().sas_bp_dpc_tde(plan.handle, int(swath), echo.data_ptr(), pr.ctypes.data, int(pr.shape[0]),
                                 int(win), int(hop), int(max_lag), out.data_ptr(), _stream(plan.device, stream)),
          "sas_bp_dpc_tde")
    return out


def dpc_desc(n_ping: int, n_window: int, n_pairs: int, n_elem: int, c: float, sigma: float = 1e-7,
             lambda_smooth: float = 0.0, lambda_dvl: float = 0.0, p0=(0.0, 0.0, 0.0), lever_tx=(0.0, 0.0, 0.0),
             robust: bool = False, max_iter: int = 30) -> N.DpcDesc:
    """Descriptor of a motion estimate (see ``sas_bp_dpc_desc`` in the header)."""
    d = N.DpcDesc()
    d.n_ping, d.n_window, d.n_pairs, d.n_elem = int(n_ping), int(n_window), int(n_pairs), int(n_elem)
    d.robust, d.max_iter = 1 if robust else 0, int(max_iter)
    d.c, d.sigma, d.lambda_smooth, d.lambda_dvl = float(c), float(sigma), float(lambda_smooth), float(lambda_dvl)
    for a in range(3):
        d.p0[a] = float(p0[a])
        d.lever_tx[a] = float(lever_tx[a])
    return d


def _host(a, dtype, shape, name):
    a = np.ascontiguousarray(np.asarray(a, dtype=dtype))
    if a.shape != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {a.shape}")
    return a


def sas_bp_dpc_footprints(desc: N.DpcDesc, vel_nominal, dt, lever_rx, pairs, t_ref, z_floor: float,
                          look: float = 1.0) -> np.ndarray:
    """Footprints [P - 1, K, 3] of every ping pair and window (host)."""
    P, K, J, E = desc.n_ping, desc.n_window, desc.n_pairs, desc.n_elem
    v = _host(vel_nominal, np.float64, (P, 3), "vel_nominal")
    d = _host(dt, np.float64, (P - 1,), "dt")
    lr = _host(lever_rx, np.float64, (E, 3), "lever_rx")
    pr = _host(pairs, np.int32, (J, 2), "pairs")
    t = _host(t_ref, np.float64, (K,), "t_ref")
    out = np.empty((P - 1, K, 3), dtype=np.float64)
    check(N.lib().sas_bp_dpc_footprints(C.byref(desc), v.ctypes.data, d.ctypes.data, lr.ctypes.data, pr.ctypes.data,
                                        t.ctypes.data, float(z_floor), float(look), out.ctypes.data),
          "sas_bp_dpc_footprints")
    return out


def sas_bp_dpc_residual(desc: N.DpcDesc, vel, dt, lever_rx, pairs, t_ref, footprint, delay, device: int = 0,
                        stream=None):
    """Eq. 4 residuals and derivatives on the GPU: returns (positions [P, 3],
    rows [P - 1, K, 7]) as float64 device tensors."""
    P, K, J, E = desc.n_ping, desc.n_window, desc.n_pairs, desc.n_elem
    dev = torch.device("cuda", device)
    f64 = dict(dtype=torch.float64, device=dev)
    ins = [torch.as_tensor(np.ascontiguousarray(x), **f64) for x in
           (_host(vel, np.float64, (P, 3), "vel"), _host(dt, np.float64, (P - 1,), "dt"),
            _host(lever_rx, np.float64, (E, 3), "lever_rx"), _host(t_ref, np.float64, (K,), "t_ref"),
            _host(footprint, np.float64, (P - 1, K, 3), "footprint"), _host(delay, np.float64, (P - 1, K), "delay"))]
    pr = torch.as_tensor(_host(pairs, np.int32, (J, 2), "pairs"), device=dev)
    pos = torch.empty((P, 3), **f64)
    rows = torch.empty((P - 1, K, 7), **f64)
    check(N.lib().sas_bp_dpc_residual(C.byref(desc), ins[0].data_ptr(), ins[1].data_ptr(), ins[2].data_ptr(),
                                      pr.data_ptr(), ins[3].data_ptr(), ins[4].data_ptr(), ins[5].data_ptr(),
                                      pos.data_ptr(), rows.data_ptr(), _stream(device, stream)),
          "sas_bp_dpc_residual")
    return pos, rows


def sas_bp_dpc_fine_delay(tde: torch.Tensor, rows: torch.Tensor, f_c: float, out: Optional[torch.Tensor] = None,
                          stream=None) -> torch.Tensor:
    """Fine delays (Sec. II-D): the TDE phase (float32 [..., 4] from
    sas_bp_dpc_tde) unwrapped around the delay that a first solution predicts,
    -rows[..., 0] with rows (float64 [..., 7]) from sas_bp_dpc_residual at a
    zero measured delay. Returns a float64 device tensor of the leading shape."""
    if tde.dtype != torch.float32 or tde.shape[-1] != 4 or not tde.is_contiguous() or not tde.is_cuda:
        raise ValueError("tde must be a contiguous float32 CUDA tensor [..., 4]")
    if rows.dtype != torch.float64 or rows.shape[-1] != 7 or not rows.is_contiguous() or rows.device != tde.device:
        raise ValueError("rows must be a contiguous float64 tensor [..., 7] on the device of tde")
    if tuple(rows.shape[:-1]) != tuple(tde.shape[:-1]):
        raise ValueError(f"rows {tuple(rows.shape)} and tde {tuple(tde.shape)} must share their leading shape")
    if out is None:
        out = torch.empty(tde.shape[:-1], dtype=torch.float64, device=tde.device)
    elif out.dtype != torch.float64 or tuple(out.shape) != tuple(tde.shape[:-1]) or not out.is_contiguous() \
            or out.device != tde.device:
        raise ValueError("out must be a contiguous float64 tensor of the leading shape of tde, on its device")
    check(N.lib().sas_bp_dpc_fine_delay(tde.data_ptr(), rows.data_ptr(), int(out.numel()), float(f_c), out.data_ptr(),
                                        _stream(tde.device.index, stream)), "sas_bp_dpc_fine_delay")
    return out


def sas_bp_dpc_solve(desc: N.DpcDesc, vx, dt, lever_rx, pairs, t_ref, footprint, delay, weight, z_dvl, vyz0,
                     device: int = 0):
    """Levenberg-Marquardt motion estimate: returns (vyz [P, 2], final loss)."""
    P, K, J, E = desc.n_ping, desc.n_window, desc.n_pairs, desc.n_elem
    a = [_host(vx, np.float64, (P,), "vx"), _host(dt, np.float64, (P - 1,), "dt"),
         _host(lever_rx, np.float64, (E, 3), "lever_rx"), _host(pairs, np.int32, (J, 2), "pairs"),
         _host(t_ref, np.float64, (K,), "t_ref"), _host(footprint, np.float64, (P - 1, K, 3), "footprint"),
         _host(delay, np.float64, (P - 1, K), "delay"), _host(weight, np.float64, (P - 1, K), "weight"),
         _host(z_dvl, np.float64, (P,), "z_dvl")]
    v = _host(vyz0, np.float64, (P, 2), "vyz0").copy()
    loss = C.c_double(0.0)
    check(N.lib().sas_bp_dpc_solve(C.byref(desc), *[x.ctypes.data for x in a], v.ctypes.data, C.byref(loss),
                                   int(device)), "sas_bp_dpc_solve")
    return v, loss.value


def sas_bp_tvg(plan: Plan, swath: int, echo: torch.Tensor, alpha: float,
               gain_out: Optional[torch.Tensor] = None, stream=None) -> None:
    """Time-varying gain of a complex64 echo cube [P, E, N_s], in place;
    gain_out (float32 [N_s], optional) receives the power gain G(t)."""
    d = plan.descs[swath]
    _need(echo, "echo", torch.complex64, (d.n_ping, d.n_elem, d.n_sample), plan.device)
    if gain_out is not None:
        _need(gain_out, "gain_out", torch.float32, (d.n_sample,), plan.device)
    check(N.lib().sas_bp_tvg(plan.handle, int(swath), echo.data_ptr(), float(alpha),
                             gain_out.data_ptr() if gain_out is not None else None, _stream(plan.device, stream)),
          "sas_bp_tvg")


def sas_bp_envelope(plan: Plan, swath: int, echo: torch.Tensor, out: Optional[torch.Tensor] = None,
                    stream=None) -> torch.Tensor:
    """Echo envelope (|e|, 0) of swath `swath`'s cube in its storage format
    (complex64 [P, E, N_s], or float16/bfloat16 [P, E, N_s, 2]); out may be
    echo itself (in place) or a new tensor of the same kind."""
    d = plan.descs[swath]
    P, E, Ns = d.n_ping, d.n_elem, d.n_sample
    if d.echo_dtype == N.ECHO_C64:
        dt, shape = torch.complex64, (P, E, Ns)
    else:
        dt, shape = (torch.float16 if d.echo_dtype == N.ECHO_F16X2 else torch.bfloat16), (P, E, Ns, 2)
    _need(echo, "echo", dt, shape, plan.device)
    if out is None:
        out = torch.empty_like(echo)
    else:
        _need(out, "out", dt, shape, plan.device)
    check(N.lib().sas_bp_envelope(plan.handle, int(swath), echo.data_ptr(), out.data_ptr(),
                                  _stream(plan.device, stream)), "sas_bp_envelope")
    return out


def sas_bp_drc(plan: Plan, image: torch.Tensor, brightness: float, out: torch.Tensor,
               params: Optional[torch.Tensor] = None, stream=None) -> None:
    """Dynamic range compression for display: out (float32, image's shape) from
    a complex64 image; params (float64 [3], optional) gets max |I|, the
    normalised median and q."""
    if image.dtype != torch.complex64 or not image.is_contiguous() or image.device.type != "cuda":
        raise ValueError("image must be a contiguous complex64 device tensor")
    _need(out, "out", torch.float32, tuple(image.shape), plan.device)
    if params is not None:
        _need(params, "params", torch.float64, (3,), plan.device)
    check(N.lib().sas_bp_drc(plan.handle, image.data_ptr(), image.numel(), float(brightness), out.data_ptr(),
                             params.data_ptr() if params is not None else None, _stream(plan.device, stream)),
          "sas_bp_drc")


def sas_bp_useful_updates(plan: Plan, bufs: Sequence[SwathBuffers], stream=None) -> list:
    arr = _io(plan, bufs)
    out = (C.c_int64 * len(bufs))()
    check(N.lib().sas_bp_useful_updates(plan.handle, arr, len(bufs), _stream(plan.device, stream), out),
          "sas_bp_useful_updates")
    return [int(v) for v in out]


def sas_bp_sharpness(plan: Plan, image: torch.Tensor, out_S: torch.Tensor,
                     grad_image: Optional[torch.Tensor] = None, stream=None) -> None:
    if image.dtype != torch.complex64 or not image.is_contiguous() or image.device.type != "cuda":
        raise ValueError("image must be a contiguous complex64 device tensor")
    _need(out_S, "out_S", torch.float64, (1,), plan.device)
    if grad_image is not None:
        _need(grad_image, "grad_image", torch.complex64, tuple(image.shape), plan.device)
    check(N.lib().sas_bp_sharpness(plan.handle, image.data_ptr(), image.numel(), out_S.data_ptr(),
                                 grad_image.data_ptr() if grad_image is not None else None,
                                 _stream(plan.device, stream)), "sas_bp_sharpness")


def sas_bp_sharpness_static(image: torch.Tensor, out_S: torch.Tensor, grad_image: Optional[torch.Tensor] = None,
                            stream=None) -> None:
    """``sas_bp_sharpness`` without a plan and without any allocation: the
    partial sums use the library's fixed per-device array (calls that overlap
    on one device race). Runs on the image's device."""
    if image.dtype != torch.complex64 or not image.is_contiguous() or image.device.type != "cuda":
        raise ValueError("image must be a contiguous complex64 device tensor")
    dev = image.device.index
    _need(out_S, "out_S", torch.float64, (1,), dev)
    if grad_image is not None:
        _need(grad_image, "grad_image", torch.complex64, tuple(image.shape), dev)
    with torch.cuda.device(dev):
        check(N.lib().sas_bp_sharpness_static(image.data_ptr(), image.numel(), out_S.data_ptr(),
                                              grad_image.data_ptr() if grad_image is not None else None,
                                              _stream(dev, stream)), "sas_bp_sharpness_static")


def sas_bp_autotune(descs: Sequence[N.SwathDesc], bufs: Sequence[SwathBuffers], reps: int = 3, device: int = 0,
                    stream=None, tune_mode: str = "default", tune_cache=None, no_cull: bool = False) -> dict:
    """Fastest tiling for these swaths, timed on their buffers (images are
    overwritten). Returns ``sas_bp_plan`` keyword arguments (tile, threads,
    pings_per_chunk, elems_per_chunk) plus ``ms``, the mean image time (0 when
    the choice came from the process cache or the ``tune_cache`` file;
    ``tune_mode`` "search" always times)."""
    descs = list(descs)
    arr = (N.SwathDesc * len(descs))(*descs)
    io = _io_for(descs, device, bufs)
    base = _options(device, tune_mode=tune_mode, no_cull=no_cull, tune_cache=tune_cache)
    best = N.Options()
    ms = C.c_double()
    check(N.lib().sas_bp_autotune(arr, len(descs), io, C.byref(base), int(reps), _stream(device, stream),
                                  C.byref(best), C.byref(ms)), "sas_bp_autotune")
    return {"tile": (best.tile_x, best.tile_y, best.tile_z), "threads": best.threads,
            "pings_per_chunk": best.pings_per_chunk, "elems_per_chunk": best.elems_per_chunk,
            "ms": float(ms.value)}


def sas_bp_gate_class(apex, box_lo, box_hi, half_angle: float) -> tuple:
    """(record class, may_hit) of the block cull for one cone apex and one box
    of pixel centres (host only): class 0 outside, 1 inside, 2 decided per row."""
    D3 = C.c_double * 3
    a, lo, hi = (D3(*(float(v) for v in x)) for x in (apex, box_lo, box_hi))
    cls, hit = C.c_int32(), C.c_int32()
    check(N.lib().sas_bp_gate_class(a, lo, hi, float(half_angle), C.byref(cls), C.byref(hit)), "sas_bp_gate_class")
    return int(cls.value), int(hit.value)


def sas_bp_set_kernel_timing(plan: Plan, enable: bool) -> None:
    check(N.lib().sas_bp_set_kernel_timing(plan.handle, 1 if enable else 0), "sas_bp_set_kernel_timing")


def sas_bp_kernel_time(plan: Plan) -> tuple:
    """(total milliseconds, launches) of the main kernel since the last read."""
    ms = C.c_double()
    n = C.c_int64()
    check(N.lib().sas_bp_kernel_time(plan.handle, C.byref(ms), C.byref(n)), "sas_bp_kernel_time")
    return float(ms.value), int(n.value)


def sas_bp_abi_version() -> int:
    return int(N.lib().sas_bp_abi_version())
