"""Sharpness autofocus over per-ping platform positions.

The image of a swath is a function of the navigation; its sharpness
S = sum|I|^4 / (sum|I|^2)^2 peaks when the positions are right. The paper
estimates motion from the data because navigation alone is not accurate to a
fraction of a wavelength (Sec. II-D); this module does it by gradient ascent
on S, with the image, S, its cotangent and the geometry adjoint all computed
by the HIP library (``sas_bp_image``, ``sas_bp_sharpness``,
``sas_bp_adjoint``). Only the optimiser runs on the host.

The unknowns are per-ping offsets of a rigid array: the same offset moves the
transmitter and every receiver of a ping. They are represented on a uniform
cubic B-spline over the ping index and refined coarse to fine (knot spacings
``levels``), because motion errors are smooth over pings and coarse knots
widen the capture range. A first stage maximises the sharpness of the
envelope image (echo magnitudes, no carrier), which varies on the scale of
the range resolution and so has no wrapped maxima within centimetres of
error; later stages maximise the coherent image's sharpness, with Adam or
L-BFGS on the spline coefficients, in a frame aligned with the line of sight.

Sharpness cannot see a constant offset or a linear trend of the track (they
move or tilt the whole image), so those components are unobservable;
``detrended_rms`` removes them before comparing with a known truth. Offsets
perpendicular to the line of sight change ranges only through the variation
of the look angle across the swath, so they are weakly determined.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, Optional, Sequence

import numpy as np
import torch

from .api import SwathBuffers, sas_bp_adjoint, sas_bp_image, sas_bp_sharpness


def bspline_basis(n: int, spacing: float) -> np.ndarray:
    """Uniform cubic B-spline basis [n, m] over samples 0..n-1 with knots every
    ``spacing`` samples (m = ceil((n - 1) / spacing) + 3 coefficients)."""
    m = int(np.ceil((n - 1) / spacing)) + 3
    t = np.arange(n, dtype=np.float64) / spacing
    B = np.zeros((n, m))
    for j in range(m):
        ax = np.abs(t - (j - 1))                 # cubic B-spline centred on knot j - 1
        v = np.where(ax < 1.0, (4.0 - 6.0 * ax ** 2 + 3.0 * ax ** 3) / 6.0,
                     np.where(ax < 2.0, (2.0 - ax) ** 3 / 6.0, 0.0))
        B[:, j] = v
    return B


def detrended_rms(err: np.ndarray) -> np.ndarray:
    """Per-column RMS of ``err`` [n, k] after removing a least-squares constant
    and linear trend over the row index."""
    n = err.shape[0]
    A = np.stack([np.ones(n), np.arange(n, dtype=np.float64)], axis=1)
    coef, *_ = np.linalg.lstsq(A, err, rcond=None)
    r = err - A @ coef
    return np.sqrt((r ** 2).mean(axis=0))


@dataclasses.dataclass
class Stage:
    """One stage of the ascent: the plan and buffers to image with, and the
    knot spacings (coarse to fine), iterations per spacing and Adam step (m)."""
    plan: object
    buf: SwathBuffers
    levels: Sequence[float] = (16, 8)
    iters: int = 60
    lr: float = 1e-4
    method: str = "adam"          # "adam", or "lbfgs" (quasi-Newton with backtracking)


def envelope_stage(plan, buf: SwathBuffers, **kw) -> Stage:
    """A stage on the envelope image: echo magnitudes imaged without the
    carrier (f_c = 0). Its sharpness varies on the scale of the range
    resolution instead of the wavelength, so it has no wrapped maxima within
    centimetres of motion error and brings the track close enough for the
    coherent stages. Allocates its own plan and buffers."""
    from .api import sas_bp_envelope, sas_bp_plan, swath_desc
    d = plan.descs[0]
    dt = {0: "c64", 1: "f16", 2: "bf16"}[d.echo_dtype]
    env = swath_desc(d.n_ping, d.n_elem, d.n_sample, tuple(d.n), tuple(d.origin), tuple(d.spacing), 0.0, d.f_s,
                     d.t0, d.gate_half_angle, dt, d.c_min)
    p2 = sas_bp_plan([env], device=plan.device)
    mag = sas_bp_envelope(p2, 0, buf.echo)
    b2 = SwathBuffers(echo=mag, tx=buf.tx.clone(), rx=buf.rx.clone(), c=buf.c, image=torch.empty_like(buf.image),
                      echo_scale=buf.echo_scale)
    return Stage(plan=p2, buf=b2, **kw)


def default_stages(plan, buf: SwathBuffers) -> list:
    """Envelope ascent (Adam, knots every 32, 16, 8, 4 pings) followed by
    coherent L-BFGS at knots every 8 and then 4 pings."""
    return [envelope_stage(plan, buf, levels=(32, 16, 8, 4), iters=60, lr=5e-4),
            Stage(plan, buf, levels=(8,), iters=100, lr=1e-4, method="lbfgs"),
            Stage(plan, buf, levels=(4,), iters=100, lr=1e-4, method="lbfgs")]


@dataclasses.dataclass
class AutofocusResult:
    offsets: np.ndarray            # [P, 3] estimated platform offsets (metres)
    sharpness: list                # S after every iteration
    levels: list                   # (knot spacing, iterations) per level
    error_rms: Optional[list] = None   # detrended RMS error per axis after each level (with truth)


def _lbfgs_ascent(value_grad, x: np.ndarray, iters: int, step0: float, memory: int = 10,
                  max_step: float = None) -> np.ndarray:
    """Maximise f with limited-memory BFGS (two-loop recursion) and a
    backtracking line search that halves the step until f increases by at
    least a small fraction of the predicted gain. ``iters`` bounds the gradient
    evaluations; the first step moves the largest coordinate by ``step0`` and
    no step moves any coordinate by more than ``max_step`` (default 20 step0)."""
    cap = 20.0 * step0 if max_step is None else max_step
    f, g = value_grad(x)
    S_list, Y_list = [], []
    for _ in range(iters):
        # two-loop recursion on -f: direction d = H g (ascent)
        q = g.copy()
        alpha = []
        for s_, y_ in reversed(list(zip(S_list, Y_list))):
            rho = 1.0 / np.dot(y_, s_)
            a = rho * np.dot(s_, q)
            alpha.append((rho, a))
            q -= a * y_
        if S_list:
            gamma = np.dot(S_list[-1], Y_list[-1]) / np.dot(Y_list[-1], Y_list[-1])
        else:
            gamma = step0 / max(np.abs(g).max(), 1e-300)
        d = gamma * q
        for (rho, a), (s_, y_) in zip(reversed(alpha), zip(S_list, Y_list)):
            b = rho * np.dot(y_, d)
            d += s_ * (a - b)
        gain = np.dot(g, d)
        if not gain > 0:                      # not an ascent direction: restart
            S_list, Y_list = [], []
            d = (step0 / max(np.abs(g).max(), 1e-300)) * g
            gain = np.dot(g, d)
        big = np.abs(d).max()
        if big > cap:                         # trust-region style cap on the step
            d *= cap / big
            gain = np.dot(g, d)
        t = 1.0
        accepted = False
        for _ in range(8):
            f_new, _ = value_grad(x + t * d, grad=False)
            if f_new >= f + 1e-4 * t * gain:
                accepted = True
                break
            t *= 0.5
        if not accepted:
            S_list, Y_list = [], []
            continue
        x_new = x + t * d
        f_new, g_new = value_grad(x_new)
        s_, y_ = x_new - x, g - g_new          # curvature pair of -f
        if np.dot(s_, y_) > 1e-12 * np.dot(s_, s_) * max(np.dot(y_, y_), 1e-300) ** 0.5:
            S_list.append(s_)
            Y_list.append(y_)
            if len(S_list) > memory:
                S_list.pop(0)
                Y_list.pop(0)
        x, f, g = x_new, f_new, g_new
    return x


def line_of_sight_frame(tx: np.ndarray, centre: Sequence[float], perp_scale: float = 1.0) -> np.ndarray:
    """Rows: along-track x, the mean line of sight from the track to ``centre``
    projected on the y-z plane, and the y-z direction perpendicular to it. A
    range change depends on an offset mostly through its line-of-sight part,
    so the two parts have very different sensitivities; optimising in this
    frame keeps the optimiser's steps well scaled; ``perp_scale`` multiplies
    the third row, so that one unit of that coefficient moves the track by
    ``perp_scale`` metres (a preconditioner for its weaker sensitivity)."""
    los = np.asarray(centre, dtype=np.float64) - np.asarray(tx, dtype=np.float64).mean(axis=0)
    los[0] = 0.0
    los /= np.linalg.norm(los)
    return np.array([[1.0, 0.0, 0.0], los, [0.0, -los[2] * perp_scale, los[1] * perp_scale]])


def autofocus(stages: Sequence[Stage], tx_nominal: torch.Tensor, rx_nominal: torch.Tensor,
              axes: Sequence[int] = (1, 2), truth: Optional[np.ndarray] = None,
              callback: Optional[Callable[[int, float], None]] = None,
              frame: Optional[np.ndarray] = None) -> AutofocusResult:
    """Maximise sharpness over per-ping offsets of one swath, stage by stage.

    Each stage images with its own plan and buffers (its tx/rx tensors are
    overwritten with the current estimate); ``tx_nominal`` [P, 3] and
    ``rx_nominal`` [P, E, 3] are the navigation to correct (float64, device).
    The estimate carries over from stage to stage and from each knot spacing
    to the next. ``axes`` are the components optimised, in ``frame`` (rows are
    the directions; default the x, y, z axes). ``truth`` [P, 3], if given, is
    the true offset, used only to report the detrended y-z error after each
    level.
    """
    R = np.eye(3) if frame is None else np.asarray(frame, dtype=np.float64)
    P = tx_nominal.shape[0]
    dev = tx_nominal.device
    axes = list(axes)
    offsets = np.zeros((P, 3))
    history, done, errs = [], [], []
    S_dev = torch.zeros(1, dtype=torch.float64, device=dev)
    gc = torch.empty(1, dtype=torch.float64, device=dev)
    gtx = torch.empty_like(tx_nominal)
    grx = torch.empty_like(rx_nominal)

    def evaluate(st: Stage, G, off: np.ndarray, grad: bool):
        o = torch.as_tensor(off, dtype=torch.float64, device=dev)
        st.buf.tx.copy_(tx_nominal + o)
        st.buf.rx.copy_(rx_nominal + o[:, None, :])
        sas_bp_image(st.plan, [st.buf])
        sas_bp_sharpness(st.plan, st.buf.image, S_dev, G if grad else None)
        if not grad:
            return float(S_dev.item()), None
        sas_bp_adjoint(st.plan, [st.buf], [G], [gtx], [grx], [gc])
        g = (gtx + grx.sum(dim=1)).cpu().numpy()        # d S / d offset of ping i
        return float(S_dev.item()), g

    step = 0
    for st in stages:
        G = torch.empty_like(st.buf.image)
        for spacing in st.levels:
            B = bspline_basis(P, spacing)
            # start from the current estimate, projected on this level's basis
            # (coefficients are in the frame's coordinates)
            w = np.zeros((B.shape[1], 3))
            if np.any(offsets):
                w[:, axes] = np.linalg.lstsq(B, (offsets @ np.linalg.inv(R))[:, axes], rcond=None)[0]
            free = [a for a in range(3) if a in axes]

            def value_grad(wf, grad=True):
                nonlocal step
                ww = np.zeros((B.shape[1], 3))
                ww[:, free] = wf.reshape(B.shape[1], len(free))
                S, g = evaluate(st, G, (B @ ww) @ R, grad)
                history.append(S)
                if callback:
                    callback(step, S)
                step += 1
                if not grad:
                    return S, None
                gw = B.T @ (g @ R.T)                       # chain rule to the coefficients
                return S, gw[:, free].ravel()

            wf = w[:, free].ravel()
            if st.method == "lbfgs":
                wf = _lbfgs_ascent(value_grad, wf, st.iters, st.lr)
            else:
                m = np.zeros_like(wf)
                v = np.zeros_like(wf)
                b1, b2, eps = 0.9, 0.999, 1e-30
                for it in range(st.iters):
                    _, gw = value_grad(wf)
                    m = b1 * m + (1 - b1) * gw
                    v = b2 * v + (1 - b2) * gw * gw
                    mh = m / (1 - b1 ** (it + 1))
                    vh = v / (1 - b2 ** (it + 1))
                    wf = wf + st.lr * mh / (np.sqrt(vh) + eps)   # ascent on S
            w[:, free] = wf.reshape(B.shape[1], len(free))
            offsets = (B @ w) @ R
            done.append((spacing, st.iters))
            if truth is not None:
                errs.append(detrended_rms(offsets[:, 1:] - truth[:, 1:]).tolist())
    if stages:
        S, _ = evaluate(stages[-1], None, offsets, False)
        history.append(S)
    return AutofocusResult(offsets=offsets, sharpness=history, levels=done,
                           error_rms=errs if truth is not None else None)
