"""Acquisition geometry, scenes and seeds for the synthetic TDBP workloads.

Conventions (Sec. II-B, NED frame): x is along-track, y is ground range to
starboard, z points down. The origin lies on the seafloor below the first ping,
so a platform at altitude h sits at z = -h. A pixel centre is
``origin + index * spacing`` on every axis, evaluated in FP64 as one product
followed by one sum. Positions are stop-and-hop by default: the transmitter
and every receiver are fixed for the duration of a ping. Continuous receiver
motion during reception (the x_RX(t) of Eq. 1) is available to the echo
synthesis: ``synthesize_echo(..., rx_vel=receiver_velocity(scn))``.

The five workloads follow the configurations the build is measured on:

* ``c1``  2D stripmap, 64 pings x 8 receivers, 256x256 px (parity case).
* ``c2``  2D stripmap at operational swath size, 512 pings x 32 receivers,
          4096x4096 px, +-10 deg transmit/receive gate, point targets plus
          speckle (throughput case).
* ``c3``  3D, downward looking, 256 pings x 64 receivers (32 across x 2 along),
          512x512x128 voxels, buried targets below a seabed of weak scatterers.
* ``c4b:k`` swath k of the batched workload (uneven sizes).
* ``c5``  autofocus: 256 pings x 16 receivers, 1024x1024 px, smooth
          sway/heave errors that the imager does not know.

Every field that the paper leaves open is an explicit attribute here, so a
scenario is fully described by ``make_config(name, **overrides)``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

CONFIG_IDS = ("c1", "c2", "c3", "c4b", "c5")

# Root seeds of the five workloads; swath k of the batched workload uses
# 1004000 + k.
ROOT_SEEDS = {"c1": 1001, "c2": 1002, "c3": 1003, "c4": 1004, "c5": 1005}

# Independent random streams spawned from a workload's root seed.
STREAMS = ("nav", "positions", "amplitudes", "noise", "subset", "injected")


def _streams(root: int) -> dict:
    ss = np.random.SeedSequence(root)
    children = ss.spawn(len(STREAMS))
    return {name: np.random.Generator(np.random.PCG64(ch)) for name, ch in zip(STREAMS, children)}


@dataclasses.dataclass
class Grid:
    """Regular pixel/voxel grid: n = (nx, ny, nz), origin and spacing in metres."""
    n: tuple
    origin: tuple
    spacing: tuple

    @property
    def dims(self) -> int:
        return 3 if self.n[2] > 1 else 2

    @property
    def n_pix(self) -> int:
        return int(self.n[0]) * int(self.n[1]) * int(self.n[2])

    def axis(self, a: int) -> np.ndarray:
        i = np.arange(int(self.n[a]), dtype=np.float64)
        return self.origin[a] + i * self.spacing[a]

    def points(self, flat_index: Optional[np.ndarray] = None) -> np.ndarray:
        """Pixel centres, [N,3] float64, in image order (x fastest, then y, then z)."""
        nx, ny, nz = (int(v) for v in self.n)
        if flat_index is None:
            flat_index = np.arange(nx * ny * nz, dtype=np.int64)
        flat_index = np.asarray(flat_index, dtype=np.int64)
        ix = flat_index % nx
        iy = (flat_index // nx) % ny
        iz = flat_index // (nx * ny)
        out = np.empty((flat_index.size, 3), dtype=np.float64)
        out[:, 0] = self.origin[0] + ix.astype(np.float64) * self.spacing[0]
        out[:, 1] = self.origin[1] + iy.astype(np.float64) * self.spacing[1]
        out[:, 2] = self.origin[2] + iz.astype(np.float64) * self.spacing[2]
        return out


@dataclasses.dataclass
class Scenario:
    name: str
    c: float                 # sound speed, m/s
    fc: float                # carrier, Hz
    fs: float                # complex sample rate, Hz
    bandwidth: float         # chirp bandwidth B, Hz
    t0: float                # time of sample 0 relative to transmit, s
    n_sample: int
    tx: np.ndarray           # [P,3] float64, navigation known to the imager
    rx: np.ndarray           # [P,E,3] float64
    grid: Grid
    gate_half_angle: float   # rad, 0 = no gate
    scat_pos: np.ndarray     # [S,3] float64
    scat_amp: np.ndarray     # [S] complex128
    snr_db: Optional[float]  # None = noiseless
    taper_half: int          # synthesis: sinc truncated to |k-u| < taper_half samples
    seed: int
    true_tx: Optional[np.ndarray] = None   # positions the echoes were synthesized with,
    true_rx: Optional[np.ndarray] = None   # when they differ from the imager's (autofocus)
    notes: str = ""

    @property
    def n_ping(self) -> int:
        return int(self.tx.shape[0])

    @property
    def n_elem(self) -> int:
        return int(self.rx.shape[1])

    @property
    def wavelength(self) -> float:
        return self.c / self.fc

    def synth_tx(self) -> np.ndarray:
        return self.tx if self.true_tx is None else self.true_tx

    def synth_rx(self) -> np.ndarray:
        return self.rx if self.true_rx is None else self.true_rx

    def nominal_updates(self) -> int:
        return self.grid.n_pix * self.n_ping * self.n_elem

    def streams(self) -> dict:
        return _streams(self.seed)


# ---------------------------------------------------------------- geometry ---

def _random_walk(rng, n, sigma, start):
    steps = rng.normal(0.0, sigma, size=n)
    steps[0] = 0.0
    return start + np.cumsum(steps)


def linear_array_rx(tx: np.ndarray, n_elem: int, pitch: float) -> np.ndarray:
    """Receivers on a line along x, centred on the transmitter (array centre)."""
    off = (np.arange(n_elem, dtype=np.float64) - (n_elem - 1) / 2.0) * pitch
    rx = np.repeat(tx[:, None, :], n_elem, axis=1).copy()
    rx[:, :, 0] += off[None, :]
    return rx


def planar_array_rx(tx: np.ndarray, n_along: int, n_across: int, pitch: float) -> np.ndarray:
    """Receivers on an n_along (x) by n_across (y) grid centred on the transmitter.

    Element e = a * n_across + b sits at x offset (a - (n_along-1)/2) * pitch and
    y offset (b - (n_across-1)/2) * pitch.
    """
    a = (np.arange(n_along, dtype=np.float64) - (n_along - 1) / 2.0) * pitch
    b = (np.arange(n_across, dtype=np.float64) - (n_across - 1) / 2.0) * pitch
    ox = np.repeat(a, n_across)
    oy = np.tile(b, n_along)
    rx = np.repeat(tx[:, None, :], n_along * n_across, axis=1).copy()
    rx[:, :, 0] += ox[None, :]
    rx[:, :, 1] += oy[None, :]
    return rx


def _cn(rng, n, sigma=1.0):
    """Circular complex Gaussian CN(0, sigma^2)."""
    s = sigma / math.sqrt(2.0)
    return rng.normal(0.0, s, size=n) + 1j * rng.normal(0.0, s, size=n)


def _smooth_error(rng, n, rms, sigma_pings):
    """White N(0,1) smoothed by a Gaussian of sigma_pings, rescaled to the given RMS."""
    w = rng.normal(0.0, 1.0, size=n)
    half = int(math.ceil(4 * sigma_pings))
    k = np.arange(-half, half + 1, dtype=np.float64)
    g = np.exp(-0.5 * (k / sigma_pings) ** 2)
    g /= g.sum()
    sm = np.convolve(np.pad(w, half, mode="reflect"), g, mode="valid")
    sm -= sm.mean()
    return sm * (rms / math.sqrt(np.mean(sm ** 2)))


def _stripmap(name, seed, *, n_ping, ping_dx, n_elem, pitch, altitude, sway_sigma,
              nx, ny, px, y0, n_sample, gate_deg, n_scat, n_speckle, speckle_sigma,
              snr_db, taper_half, c=1500.0, fc=100e3, fs=80e3, bandwidth=20e3,
              straight=False, notes=""):
    st = _streams(seed)
    xs = np.arange(n_ping, dtype=np.float64) * ping_dx
    if straight or sway_sigma == 0.0:
        ys = np.zeros(n_ping)
        zs = np.full(n_ping, -altitude)
    else:
        ys = _random_walk(st["nav"], n_ping, sway_sigma, 0.0)
        zs = _random_walk(st["nav"], n_ping, sway_sigma, -altitude)
    tx = np.stack([xs, ys, zs], axis=1)
    rx = linear_array_rx(tx, n_elem, pitch)
    xmid = 0.5 * (xs[0] + xs[-1])
    grid = Grid(n=(nx, ny, 1),
                origin=(xmid - 0.5 * (nx - 1) * px, y0, 0.0),
                spacing=(px, px, px))
    x_lo, x_hi = grid.origin[0], grid.origin[0] + (nx - 1) * px
    y_lo, y_hi = grid.origin[1], grid.origin[1] + (ny - 1) * px
    pos = st["positions"]
    spos = np.stack([pos.uniform(x_lo, x_hi, n_scat), pos.uniform(y_lo, y_hi, n_scat),
                     np.zeros(n_scat)], axis=1)
    samp = _cn(st["amplitudes"], n_scat)
    if n_speckle:
        kpos = np.stack([pos.uniform(x_lo, x_hi, n_speckle), pos.uniform(y_lo, y_hi, n_speckle),
                         np.zeros(n_speckle)], axis=1)
        spos = np.concatenate([spos, kpos])
        samp = np.concatenate([samp, _cn(st["amplitudes"], n_speckle, speckle_sigma)])
    return Scenario(name=name, c=c, fc=fc, fs=fs, bandwidth=bandwidth, t0=0.0,
                    n_sample=n_sample, tx=tx, rx=rx, grid=grid,
                    gate_half_angle=math.radians(gate_deg), scat_pos=spos, scat_amp=samp,
                    snr_db=snr_db, taper_half=taper_half, seed=seed, notes=notes)


def _c1(**kw):
    p = dict(n_ping=64, ping_dx=0.15, n_elem=8, pitch=0.0375, altitude=10.0, sway_sigma=5e-3,
             nx=256, ny=256, px=0.015, y0=20.0, n_sample=4096, gate_deg=0.0,
             n_scat=16, n_speckle=0, speckle_sigma=0.0, snr_db=20.0, taper_half=64)
    p.update(kw)
    return _stripmap("c1", ROOT_SEEDS["c1"] if "seed" not in p else p.pop("seed"), **p)


def _c2(**kw):
    p = dict(n_ping=512, ping_dx=0.3, n_elem=32, pitch=0.0375, altitude=10.0, sway_sigma=5e-3,
             nx=4096, ny=4096, px=0.015, y0=20.0, n_sample=16384, gate_deg=10.0,
             n_scat=2000, n_speckle=100000, speckle_sigma=0.05, snr_db=20.0, taper_half=16)
    p.update(kw)
    return _stripmap("c2", ROOT_SEEDS["c2"] if "seed" not in p else p.pop("seed"), **p)


def _c3(**kw):
    p = dict(n_ping=256, ping_dx=0.1, n_along=2, n_across=32, pitch=0.0375, sway_sigma=5e-3,
             nx=512, ny=512, nz=128, vx=0.02, z0=5.0, n_sample=8192, seabed_z=5.5,
             n_surface=400, n_buried=100, bury_max=1.0, n_seabed=100000, seabed_sigma=0.05,
             snr_db=20.0, taper_half=16)
    p.update(kw)
    seed = p.pop("seed", ROOT_SEEDS["c3"])
    st = _streams(seed)
    n_ping = p["n_ping"]
    xs = np.arange(n_ping, dtype=np.float64) * p["ping_dx"]
    ys = _random_walk(st["nav"], n_ping, p["sway_sigma"], 0.0)
    zs = _random_walk(st["nav"], n_ping, p["sway_sigma"], 0.0)
    tx = np.stack([xs, ys, zs], axis=1)
    rx = planar_array_rx(tx, p["n_along"], p["n_across"], p["pitch"])
    nx, ny, nz, v = p["nx"], p["ny"], p["nz"], p["vx"]
    xmid = 0.5 * (xs[0] + xs[-1])
    grid = Grid(n=(nx, ny, nz), origin=(xmid - 0.5 * (nx - 1) * v, -0.5 * (ny - 1) * v, p["z0"]),
                spacing=(v, v, v))
    x_lo, x_hi = grid.origin[0], grid.origin[0] + (nx - 1) * v
    y_lo, y_hi = grid.origin[1], grid.origin[1] + (ny - 1) * v
    pos = st["positions"]
    n_t = p["n_surface"] + p["n_buried"]
    tz = np.full(n_t, p["seabed_z"])
    tz[p["n_surface"]:] += pos.uniform(0.0, p["bury_max"], p["n_buried"])
    tpos = np.stack([pos.uniform(x_lo, x_hi, n_t), pos.uniform(y_lo, y_hi, n_t), tz], axis=1)
    tamp = _cn(st["amplitudes"], n_t)
    if p["n_seabed"]:
        bpos = np.stack([pos.uniform(x_lo, x_hi, p["n_seabed"]), pos.uniform(y_lo, y_hi, p["n_seabed"]),
                         np.full(p["n_seabed"], p["seabed_z"])], axis=1)
        tpos = np.concatenate([tpos, bpos])
        tamp = np.concatenate([tamp, _cn(st["amplitudes"], p["n_seabed"], p["seabed_sigma"])])
    return Scenario(name="c3", c=1500.0, fc=100e3, fs=80e3, bandwidth=20e3, t0=0.0,
                    n_sample=p["n_sample"], tx=tx, rx=rx, grid=grid, gate_half_angle=0.0,
                    scat_pos=tpos, scat_amp=tamp, snr_db=p["snr_db"], taper_half=p["taper_half"],
                    seed=seed)


def _pow2_cover(dist_m, c=1500.0, fs=80e3):
    need = int(math.ceil(2.0 * dist_m / c * fs)) + 2
    n = 1
    while n < need:
        n *= 2
    return n


def c4b_swath(k: int, **kw):
    """Swath k of the batched workload: uneven size, ping and receiver counts."""
    seed = 1004000 + k
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    nx = int(rng.integers(512, 4097))
    ny = int(rng.integers(512, 4097))
    n_ping = int(rng.integers(128, 513))
    n_elem = int(rng.integers(16, 33))
    p = dict(n_ping=n_ping, ping_dx=0.3, n_elem=n_elem, pitch=0.0375, altitude=10.0,
             sway_sigma=5e-3, nx=nx, ny=ny, px=0.015, y0=20.0, n_sample=0, gate_deg=10.0,
             n_scat=200, n_speckle=0, speckle_sigma=0.0, snr_db=20.0, taper_half=16)
    p.update(kw)
    if not p["n_sample"]:
        y_far = p["y0"] + (p["ny"] - 1) * p["px"]
        gate = math.radians(p["gate_deg"]) if p["gate_deg"] else math.radians(89.0)
        half_x = math.tan(gate) * math.hypot(y_far, p["altitude"] + 0.1)
        p["n_sample"] = _pow2_cover(math.sqrt(y_far ** 2 + (p["altitude"] + 0.1) ** 2 + half_x ** 2) + 1.0)
    return _stripmap(f"c4b:{k}", seed, **p)


def _c5(**kw):
    p = dict(n_ping=256, ping_dx=0.15, n_elem=16, pitch=0.0375, altitude=10.0, sway_sigma=0.0,
             nx=1024, ny=1024, px=0.015, y0=20.0, n_sample=4096, gate_deg=0.0,
             n_scat=256, n_speckle=0, speckle_sigma=0.0, snr_db=20.0, taper_half=64,
             err_rms=0.01, err_sigma_pings=8.0)
    p.update(kw)
    err_rms = p.pop("err_rms")
    err_sig = p.pop("err_sigma_pings")
    seed = p.pop("seed", ROOT_SEEDS["c5"])
    scn = _stripmap("c5", seed, straight=True, **p)
    st = scn.streams()
    inj = st["injected"]
    n = scn.n_ping
    err = np.zeros((n, 3))
    if err_rms > 0:
        err[:, 1] = _smooth_error(inj, n, err_rms, err_sig)
        err[:, 2] = _smooth_error(inj, n, err_rms, err_sig)
    scn.true_tx = scn.tx + err
    scn.true_rx = scn.rx + err[:, None, :]
    scn.notes = "imager navigation is the straight nominal track; echoes use true_tx/true_rx"
    return scn


@dataclasses.dataclass
class DpcTrack:
    """A swath for the DPC motion estimate: the scenario (``tx``/``rx`` the
    straight nominal track, ``true_tx``/``true_rx`` the track the echoes are
    synthesized on), the true per-ping velocities [P, 3] (surge, sway, heave;
    the receivers also move with them during reception), the ping intervals
    dt [P - 1] and the platform position of the first ping."""
    scn: Scenario
    vel: np.ndarray
    dt: np.ndarray
    p0: np.ndarray


def dpc_track(n_ping: int = 16, n_sample: int = 2048, pri: float = 0.2, sway_amp: float = 0.02,
              heave_amp: float = 0.012, seed: int = 1006, n_speckle: int = 40000) -> DpcTrack:
    """Stripmap geometry of the operational workload (32 receivers at
    3.75 cm, transmitter at the array centre, 0.3 m advance per ping, so
    element e + 16 of ping i and element e of ping i + 1 share a phase centre;
    10 m altitude) over a fully developed speckle seafloor covering every
    beam, on a track whose sway and heave velocities are smooth sinusoids of
    seeded phase (amplitudes in m/s) plus a seeded constant: the platform
    drifts a few centimetres over the swath. Positions integrate the
    velocities over the ping intervals."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    ph = rng.uniform(0.0, 2.0 * math.pi, 2)
    bias = rng.uniform(-0.2, 0.2, 2)
    i = np.arange(n_ping, dtype=np.float64)
    vx = 0.3 / pri
    vel = np.column_stack([np.full(n_ping, vx),
                           sway_amp * (np.sin(2.0 * math.pi * 0.8 * i / n_ping + ph[0]) + bias[0]),
                           heave_amp * (np.cos(2.0 * math.pi * 0.6 * i / n_ping + ph[1]) + bias[1])])
    dt = np.full(n_ping - 1, float(pri))
    p0 = np.array([0.0, 0.0, -10.0])
    true_tx = p0[None, :] + np.concatenate([np.zeros((1, 3)), np.cumsum(vel[:-1] * dt[:, None], axis=0)])
    slant = 1500.0 * n_sample / 80e3 / 2.0
    half_x = math.tan(math.radians(10.0)) * slant + 0.6
    x_lo, x_hi = -half_x, true_tx[-1, 0] + half_x
    ground = math.sqrt(max(slant ** 2 - 9.0 ** 2, 1.0)) + 0.5
    px = 0.015
    nx, ny = int(math.ceil((x_hi - x_lo) / px)) + 1, int(math.ceil(ground / px)) + 1
    scn = _stripmap("dpc", seed, n_ping=n_ping, ping_dx=0.3, n_elem=32, pitch=0.0375, altitude=10.0,
                    sway_sigma=0.0, nx=nx, ny=ny, px=px, y0=0.0, n_sample=n_sample, gate_deg=10.0,
                    n_scat=0, n_speckle=n_speckle, speckle_sigma=1.0, snr_db=20.0, taper_half=16, straight=True)
    scn.grid = Grid(n=(nx, ny, 1), origin=(x_lo, 0.0, 0.0), spacing=(px, px, px))
    pos = scn.streams()["positions"]
    scn.scat_pos = np.stack([pos.uniform(x_lo, x_hi, n_speckle), pos.uniform(0.0, ground, n_speckle),
                             np.zeros(n_speckle)], axis=1)
    scn.true_tx = true_tx
    scn.true_rx = linear_array_rx(true_tx, 32, 0.0375)
    scn.notes = "DPC track: echoes on true_tx/true_rx with the receivers moving at vel during reception"
    return DpcTrack(scn=scn, vel=vel, dt=dt, p0=p0)


def make_config(name: str, **overrides) -> Scenario:
    """Build a workload by name: 'c1', 'c2', 'c3', 'c4a' (= c1), 'c4b:k', 'c5'.

    Keyword overrides shrink or alter a workload (e.g. ``n_ping=16, nx=96``)
    while keeping its geometry recipe; they are how the tests get small,
    ragged variants of each workload.
    """
    if name in ("c1", "c4a"):
        return _c1(**overrides)
    if name == "c2":
        return _c2(**overrides)
    if name == "c3":
        return _c3(**overrides)
    if name.startswith("c4b"):
        k = int(name.split(":")[1]) if ":" in name else 0
        return c4b_swath(k, **overrides)
    if name == "c5":
        return _c5(**overrides)
    raise ValueError(f"unknown workload {name!r}")


def receiver_velocity(scn: Scenario, pri: float | None = None) -> np.ndarray:
    """Per-ping platform velocity [P, 3] (m/s) for continuous-motion tests:
    central differences of the navigated transmitter track over the ping
    repetition interval (default one record, N_s / f_s), one-sided at the ends.
    The receivers share it (a rigid array)."""
    pri = scn.n_sample / scn.fs if pri is None else pri
    t = np.asarray(scn.tx, dtype=np.float64)
    if t.shape[0] < 2:
        return np.zeros_like(t)
    return np.gradient(t, axis=0) / pri


def receiver_track(scn: Scenario, n_samp: int | None = None, h: float = 2e-3, seed: int = 5):
    """An up-sampled position table per ping for continuous-motion tests:
    the receivers' displacement from their ping-time positions at t = j h
    after transmit (j = 0..n_samp - 1): a 1.5 m/s surge plus sinusoidal sway
    and heave of a few millimetres at 5 to 15 rad/s with seeded phases
    (accelerations up to about 0.9 m/s^2), zero at transmit. n_samp defaults
    to a table that covers the record plus 10 ms. Returns (table [P, n, 3], h)."""
    if n_samp is None:
        n_samp = int(math.ceil((scn.t0 + scn.n_sample / scn.fs + 0.01) / h)) + 1
    rng = np.random.default_rng(seed)
    t = np.arange(n_samp) * h
    P = scn.n_ping
    tab = np.zeros((P, n_samp, 3))
    amp = np.array([0.003, 0.004, 0.002])
    for i in range(P):
        w = rng.uniform(5.0, 15.0, 3)
        ph = rng.uniform(0, 2 * np.pi, 3)
        tab[i] = amp * (np.sin(w * t[:, None] + ph) - np.sin(ph))
        tab[i, :, 0] += 1.5 * t
    return tab, h


def subset_indices(scn: Scenario, count: int) -> np.ndarray:
    """Seeded pixel subset (flat image indices, sorted) drawn without replacement."""
    rng = scn.streams()["subset"]
    n = scn.grid.n_pix
    count = min(count, n)
    return np.sort(rng.choice(n, size=count, replace=False)).astype(np.int64)
