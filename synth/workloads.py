"""Seeded phantoms, angle schedules, flows and noise directions.

Five workloads are defined, all synthetic stand-ins for the paper's test data
(moving rigid objects under limited, shifted angle sets, Sec. 5.1, Tests 1-2):

* ``cfg_disk32``      32x32x8, one disk translating +1 px/frame, 10 angles.
* ``cfg_ellipse128``  128x128x16, 3 ellipses with integer velocities, 30 angles.
* ``cfg_blur_ragged`` 40 rotating-ellipse sequences of uneven sizes, 9x9 blur.
* ``cfg_autograd256`` 256x256x16 phantom + texture, smooth flow, loss weights.
* ``cfg_large1024``   1024x1024x64, 12 moving/rotating ellipses, 90 angles.

Noise is returned as an unscaled standard-normal direction ``g``; the data are
``b = clean + level * ||clean|| * g / ||g||`` (``noisy``), where ``clean`` is
the forward operator applied to ``u_true`` by whichever side consumes it.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

# Golden angle for a 180-degree angular range: pi*(sqrt(5)-1)/2 rad ~ 111.246 deg.
GOLDEN_ANGLE_180 = math.pi * (math.sqrt(5.0) - 1.0) / 2.0


def bins_for(n: int) -> int:
    """Odd count of unit detector bins that covers the image diagonal: 2*floor(N/sqrt2)+1."""
    return 2 * int(math.floor(n / math.sqrt(2.0))) + 1


def angles_shifted(n_t: int, n_theta: int, shift_per_frame: float) -> np.ndarray:
    """theta[t, k] = k*pi/n_theta + t*shift_per_frame (radians), shape [n_t, n_theta]."""
    k = np.arange(n_theta, dtype=np.float64)
    t = np.arange(n_t, dtype=np.float64)[:, None]
    return k[None, :] * (math.pi / n_theta) + t * shift_per_frame


@dataclass
class Sequence:
    u_true: np.ndarray                   # [n_t, ny, nx] float64
    angles: Optional[np.ndarray] = None  # [n_t, n_theta] radians (Radon only)
    n_bins: Optional[int] = None         # detector bins (Radon only)
    noise_g: Optional[np.ndarray] = None  # standard-normal direction, data-shaped
    velocity: Optional[np.ndarray] = None  # [n_obj, 2] true px/frame (info only)

    @property
    def n_t(self) -> int:
        return int(self.u_true.shape[0])

    @property
    def ny(self) -> int:
        return int(self.u_true.shape[1])

    @property
    def nx(self) -> int:
        return int(self.u_true.shape[2])


@dataclass
class Workload:
    name: str
    op: str                      # "radon" or "blur"
    seqs: List[Sequence]
    noise_level: float
    params: dict = field(default_factory=dict)   # solver settings of the workload

    @property
    def n_pixels(self) -> int:
        return int(sum(s.u_true.size for s in self.seqs))


def angle_schedule(kind: str, n_t: int, n_views: int) -> np.ndarray:
    """Projection angles [n_t, n_views] in radians for the paper's three schedules (Sec. 5,
    Tests 1 and 2), n_views evenly spaced angles per frame over the frame's interval:
      "fixed":   [0, 180) every frame;
      "equal":   [180 (t-1) / n_t, 180 t / n_t), one of n_t equal sub-intervals per frame;
      "shifted": [z (t-1) / n_t, z (t-1) / n_t + 180) with z = 180 / n_views.
    """
    t = np.arange(n_t)[:, None]
    k = np.arange(n_views)[None, :]
    if kind == "fixed":
        deg = np.broadcast_to(180.0 * k / n_views, (n_t, n_views))
    elif kind == "equal":
        deg = 180.0 * t / n_t + (180.0 / n_t) * k / n_views
    elif kind == "shifted":
        deg = (180.0 / n_views) * t / n_t + 180.0 * k / n_views
    else:
        raise ValueError(kind)
    return np.radians(np.array(deg, dtype=np.float64))


def noisy(clean: np.ndarray, g: np.ndarray, level: float) -> np.ndarray:
    """b = clean + level*||clean||*g/||g||  (Gaussian noise at a relative level)."""
    clean = np.asarray(clean, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64).reshape(clean.shape)
    return clean + level * np.linalg.norm(clean) * g / np.linalg.norm(g)


# --------------------------------------------------------------------------- phantoms

def _pixel_grid(ny: int, nx: int):
    y, x = np.mgrid[0:ny, 0:nx]
    return x.astype(np.float64), y.astype(np.float64)


def paint_ellipses(ny: int, nx: int, ells: List[dict], t: float) -> np.ndarray:
    """Painter's-order union of filled ellipses at frame time t (later ones overwrite).

    Each ellipse dict holds cx, cy (pixel-index coordinates at t=0), a, b (semi-axes,
    px), phi (rad), val, vx, vy (px/frame) and om (rad/frame).  A pixel belongs to an
    ellipse when its centre satisfies the implicit inequality.
    """
    img = np.zeros((ny, nx))
    for e in ells:
        cx = e["cx"] + e.get("vx", 0.0) * t
        cy = e["cy"] + e.get("vy", 0.0) * t
        ph = e["phi"] + e.get("om", 0.0) * t
        c, s = math.cos(ph), math.sin(ph)
        R = max(e["a"], e["b"]) + 1.0
        x0, x1 = max(0, int(math.floor(cx - R))), min(nx, int(math.ceil(cx + R)) + 1)
        y0, y1 = max(0, int(math.floor(cy - R))), min(ny, int(math.ceil(cy + R)) + 1)
        if x0 >= x1 or y0 >= y1:
            continue
        y, x = np.mgrid[y0:y1, x0:x1]
        dx, dy = x - cx, y - cy
        xr = c * dx + s * dy
        yr = -s * dx + c * dy
        inside = (xr / e["a"]) ** 2 + (yr / e["b"]) ** 2 <= 1.0
        img[y0:y1, x0:x1][inside] = e["val"]
    return img


def _place_centres(rng, n, R, vx, vy, n_t, margin=1.0, tries=10000):
    """Centre so that a radius-R disk stays >= margin px inside for every frame."""
    lo_x = R + margin - min(0.0, vx * (n_t - 1))
    hi_x = n - 1 - R - margin - max(0.0, vx * (n_t - 1))
    lo_y = R + margin - min(0.0, vy * (n_t - 1))
    hi_y = n - 1 - R - margin - max(0.0, vy * (n_t - 1))
    if hi_x < lo_x or hi_y < lo_y:
        return None
    return rng.uniform(lo_x, hi_x), rng.uniform(lo_y, hi_y)


def _random_ellipses(rng, n, n_t, count, ax_lo, ax_hi, vel_mode, rot_deg=None):
    ells = []
    while len(ells) < count:
        a = rng.uniform(ax_lo, ax_hi)
        b = rng.uniform(ax_lo, ax_hi)
        phi = rng.uniform(0.0, math.pi)
        val = rng.uniform(0.3, 1.0)
        if vel_mode == "int":
            vx, vy = (float(v) for v in rng.integers(-2, 3, size=2))
        elif vel_mode == "real":
            vx, vy = (float(v) for v in rng.uniform(-2.0, 2.0, size=2))
        else:
            vx = vy = 0.0
        if rot_deg is None:
            om = 0.0
        elif isinstance(rot_deg, tuple) and rot_deg[0] == "pm":
            om = math.radians(rng.uniform(rot_deg[1], rot_deg[2])) * (1.0 if rng.random() < 0.5 else -1.0)
        else:
            om = math.radians(rng.uniform(-rot_deg, rot_deg))
        c = _place_centres(rng, n, max(a, b), vx, vy, n_t)
        if c is None:
            continue
        ells.append(dict(cx=c[0], cy=c[1], a=a, b=b, phi=phi, val=val, vx=vx, vy=vy, om=om))
    return ells


def _sequence_from(ells, n, n_t):
    return np.stack([paint_ellipses(n, n, ells, float(t)) for t in range(n_t)])


# --------------------------------------------------------------------------- flows

def random_field(shape, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).standard_normal(shape)


def smooth_flow(n_pairs: int, n: int, seed: int, sigma: float = 16.0, vmax: float = 3.0) -> np.ndarray:
    """Smooth random flow [n_pairs, 2, n, n]: N(0,1) per component, Gaussian-smoothed
    (reflect borders), rescaled so that max |v| = vmax."""
    from scipy.ndimage import gaussian_filter

    g = np.random.default_rng(seed).standard_normal((n_pairs, 2, n, n))
    out = np.empty_like(g)
    for p in range(n_pairs):
        for c in range(2):
            out[p, c] = gaussian_filter(g[p, c], sigma=sigma, mode="reflect")
    return out * (vmax / np.abs(out).max())


def smooth_flow_coarse(n_pairs: int, n: int, seed: int, coarse: int = 16, vmax: float = 3.0) -> np.ndarray:
    """Smooth random flow [n_pairs, 2, n, n]: N(0,1) on a coarse grid, bilinearly upsampled,
    rescaled so that max |v| = vmax (cheap at large n)."""
    from scipy.ndimage import zoom

    g = np.random.default_rng(seed).standard_normal((n_pairs, 2, coarse, coarse))
    out = np.empty((n_pairs, 2, n, n))
    for p in range(n_pairs):
        for c in range(2):
            out[p, c] = zoom(g[p, c], n / coarse, order=1, mode="nearest")[:n, :n]
    return out * (vmax / np.abs(out).max())


def nudge_off_kinks(v: np.ndarray, gap: float = 1e-3) -> np.ndarray:
    """Move every component's fractional part at least ``gap`` away from 0 and 1.

    Sample positions are pixel index + v, so this keeps them off the integer grid
    (the kinks of bilinear interpolation and the clamp edges 0 and N-1)."""
    v = np.array(v, dtype=np.float64, copy=True)
    fr = v - np.floor(v)
    v = np.where(fr < gap, np.floor(v) + gap, v)
    v = np.where(fr > 1.0 - gap, np.floor(v) + 1.0 - gap, v)
    return v


# --------------------------------------------------------------------------- workloads

def cfg_disk32() -> Workload:
    """32x32 x 8 frames; disk r=6 (value 1 on 0) translating +1 px/frame in x;
    10 angles over [0,pi) offset 1 deg/frame, 45 bins; noise 1%; 20 alternations."""
    n, n_t = 32, 8
    x, y = _pixel_grid(n, n)
    u = np.stack([(((x - (12.0 + t)) ** 2 + (y - 16.0) ** 2) <= 36.0).astype(np.float64)
                  for t in range(n_t)])
    ang = angles_shifted(n_t, 10, math.radians(1.0))
    nb = bins_for(n)
    g = np.random.default_rng(1).standard_normal((n_t, 10, nb))
    seq = Sequence(u_true=u, angles=ang, n_bins=nb, noise_g=g, velocity=np.array([[1.0, 0.0]]))
    return Workload("disk32x32x8", "radon", [seq], 0.01,
                    dict(alpha=0.1, k_max=20, tau=1, ell=10, n_sweeps=200, eps=1e-3, eta=1.01,
                         delta_r=1, op_dtype="f64"))


def cfg_krylov210() -> Workload:
    """20x20 x 3 frames; disk of radius sqrt(20) (value 1 on 0) translating +1 px/frame in x;
    8 angles over [0,pi) offset 5 deg/frame, 29 bins; noise 2% (seed 3).  Solved with the
    paper's iteration budget (Sec. 5): ell = 10 start vectors and 201 MM iterations, so the
    last projected problem has 210 columns, flow every 20 iterations."""
    n, n_t = 20, 3
    x, y = _pixel_grid(n, n)
    u = np.stack([(((x - (6.0 + t)) ** 2 + (y - 10.0) ** 2) <= 20.0).astype(np.float64) for t in range(n_t)])
    ang = angles_shifted(n_t, 8, math.radians(5.0))
    nb = bins_for(n)
    g = np.random.default_rng(3).standard_normal((n_t, 8, nb))
    seq = Sequence(u_true=u, angles=ang, n_bins=nb, noise_g=g, velocity=np.array([[1.0, 0.0]]))
    return Workload("krylov210x20x20x3", "radon", [seq], 0.02,
                    dict(alpha=0.2, k_max=201, tau=20, ell=10, n_sweeps=20, eps=1e-3, eta=1.01,
                         delta_r=1, op_dtype="f64"))


def cfg_ellipse128(seed: int = 2) -> Workload:
    """128x128 x 16; 3 ellipses (semi-axes 8-30 px, values U[0.3,1]) translating with
    integer velocities in [-2,2]; 30 angles/frame rotated 6 deg/frame; 181 bins; 2% noise."""
    n, n_t = 128, 16
    rng = np.random.default_rng(seed)
    ells = _random_ellipses(rng, n, n_t, 3, 8.0, 30.0, "int")
    u = _sequence_from(ells, n, n_t)
    ang = angles_shifted(n_t, 30, math.radians(6.0))
    nb = bins_for(n)
    g = rng.standard_normal((n_t, 30, nb))
    vel = np.array([[e["vx"], e["vy"]] for e in ells])
    seq = Sequence(u_true=u, angles=ang, n_bins=nb, noise_g=g, velocity=vel)
    return Workload("ellipse128x128x16", "radon", [seq], 0.02,
                    dict(alpha=0.1, k_max=30, tau=10, ell=10, n_sweeps=200, eps=1e-3, eta=1.01,
                         delta_r=1, op_dtype="f32"))


def cfg_blur_ragged(n_seq: int = 40, seed: int = 3, n_lo: int = 64, n_hi: int = 256,
                    t_lo: int = 8, t_hi: int = 32) -> Workload:
    """40 sequences of uneven sizes (64^2..256^2, 8..32 frames), 3 rotating ellipses
    each (2-5 deg/frame, random sign), 9x9 Gaussian blur sigma=2, 1% noise."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(n_lo, n_hi + 1, size=n_seq)
    frames = rng.integers(t_lo, t_hi + 1, size=n_seq)
    seqs = []
    for i in range(n_seq):
        r = np.random.default_rng(seed * 1000 + i)
        n, n_t = int(sizes[i]), int(frames[i])
        ells = _random_ellipses(r, n, n_t, 3, 0.06 * n, 0.25 * n, "none", rot_deg=("pm", 2.0, 5.0))
        u = _sequence_from(ells, n, n_t)
        g = r.standard_normal(u.shape)
        seqs.append(Sequence(u_true=u, noise_g=g))
    return Workload("blur_ragged40", "blur", seqs, 0.01,
                    dict(alpha=0.1, k_max=30, tau=10, ell=10, n_sweeps=100, eps=1e-3, eta=1.01,
                         delta_r=1, op_dtype="f32", ksize=9, sigma=2.0))


def cfg_autograd256(n: int = 256, n_t: int = 16) -> Workload:
    """256x256 x 16 phantom plus a smooth texture; smooth flow (|v| <= 3, nudged off the
    bilinear kinks); Radon with 30 angles rotated 6 deg/frame and 363 bins."""
    from scipy.ndimage import gaussian_filter

    rng = np.random.default_rng(2)
    s = n / 128.0
    ells = _random_ellipses(rng, n, n_t, 3, 8.0 * s, 30.0 * s, "int")
    u = _sequence_from(ells, n, n_t)
    tex = gaussian_filter(np.random.default_rng(4).normal(0.0, 0.05, (n, n)), sigma=4.0, mode="reflect")
    u = u + tex[None]
    v = nudge_off_kinks(smooth_flow(n_t - 1, n, seed=4, sigma=16.0 * n / 256.0, vmax=3.0))
    ang = angles_shifted(n_t, 30, math.radians(6.0))
    seq = Sequence(u_true=u, angles=ang, n_bins=bins_for(n))
    wl = Workload("autograd256x256x16", "radon", [seq], 0.0, dict(op_dtype="f32"))
    wl.params["flow"] = v
    wl.params["loss_seed"] = 5
    return wl


def cfg_large1024(n: int = 1024, n_t: int = 64, n_theta: int = 90, n_ell: int = 12, seed: int = 6) -> Workload:
    """1024x1024 x 64; 12 ellipses (semi-axes 30-200 px) with real velocities in [-2,2]
    and rotations in [-3,3] deg/frame; 90 angles/frame shifted by the golden angle per
    frame; 1449 bins; 2% noise."""
    rng = np.random.default_rng(seed)
    sc = n / 1024.0
    ells = _random_ellipses(rng, n, n_t, n_ell, 30.0 * sc, 200.0 * sc, "real", rot_deg=3.0)
    u = _sequence_from(ells, n, n_t)
    ang = angles_shifted(n_t, n_theta, GOLDEN_ANGLE_180)
    nb = bins_for(n)
    g = rng.standard_normal((n_t, n_theta, nb))
    vel = np.array([[e["vx"], e["vy"]] for e in ells])
    seq = Sequence(u_true=u, angles=ang, n_bins=nb, noise_g=g, velocity=vel)
    return Workload("large1024x1024x64", "radon", [seq], 0.02,
                    dict(alpha=0.1, k_max=50, tau=10, ell=10, n_sweeps=100, eps=1e-3, eta=1.01,
                         delta_r=1, op_dtype="f32"))
