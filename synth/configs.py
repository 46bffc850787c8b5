"""Seeded problem generators (inputs only; no arithmetic of the method).

Geometry conventions used by every consumer:

* Arrays are indexed ``[z, y, x]`` with ``x`` fastest (C order).  Voxel
  ``(ix, iy, iz)`` sits at position ``(ix, iy, iz) * dx``.
* The absorbing layer (PML) lies *inside* the stated grid, ``P`` cells deep at
  both ends of every axis, so the grid sizes are the FFT sizes.
* Transducers are point-like (Sec. 4.1) and snapped to the nearest voxel
  ``floor(pos + 1/2)``; duplicate voxels are rejected.
* The bowl is a hemisphere of golden-section points (Sec. 4.1: 2048 points on
  a half-sphere) centred in x/y with its rim plane at ``z_b = P + 2`` and the
  cup extending towards +z.  Even-numbered points emit, odd-numbered points
  receive (half of the transducers emit, half receive, Sec. 4.1).
* The region of interest Gamma is the half-ball ``|x - x_b| <= R_G,
  z >= z_b + 2`` inside the bowl (a full ball for the tiny case); its boundary
  layer dGamma is the set of Gamma voxels closer than ``L_b`` cells to Gamma's
  surface (Sec. 4.2 studies layers of 1/2/4/8 voxels and keeps 8).
* Sound speed: water 1500 m/s outside Gamma; inside a fat-like 1470 m/s
  background plus seeded Gaussian inclusions, within the paper's palette of
  1470-1650 m/s (Fig. Setup) and the bounds 1350-1800 m/s (Sec. 4.1).
* Time step: dt = cfl * dx / c_max with cfl = 0.3 and c_max = 1800 m/s
  (Sec. 4.1), which gives 83.3 ns at 0.5 mm.
* Source pulse: a Hann-windowed three-cycle toneburst at f0 = 1 MHz scaled by
  0.5 mm / dx, a smooth "click" in the sense of Sec. 4.1.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Optional, Tuple

import numpy as np

C_WATER = 1500.0
C_FAT = 1470.0
C_MIN = 1350.0
C_MAX = 1800.0
RHO0 = 1000.0
CFL = 0.3
PML_ALPHA = 2.0

CONFIG_NAMES = ("tiny", "c128", "batch", "serve96", "serve160", "serve224", "full")


@dataclasses.dataclass
class Problem:
    """One synthetic measurement problem.  All arrays are numpy (host)."""

    name: str
    shape: Tuple[int, int, int]          # (nz, ny, nx)
    dx: float                            # m
    dt: float                            # s
    nt: int                              # time steps
    c_ref: float                         # m/s, k-space reference speed
    c_min: float
    c_max: float
    rho0: float
    pml: Tuple[int, int, int]            # PML cells per axis, (px, py, pz)
    pml_alpha: float
    precision: int                       # 4 or 8 (compute type of the GPU path)
    src_ijk: np.ndarray                  # int32 [n_src, 3] (ix, iy, iz)
    rec_ijk: np.ndarray                  # int32 [n_rec, 3]
    gamma: np.ndarray                    # uint8 [nz, ny, nx], 1 inside Gamma
    boundary: np.ndarray                 # uint8 [nz, ny, nx], 1 on dGamma
    c_true: np.ndarray                   # float64 [nz, ny, nx]
    c_eval: np.ndarray                   # float64 [nz, ny, nx] (inclusions removed)
    pulse: np.ndarray                    # float64 [nt]
    enc_seed: int                        # seed of the Rademacher encoding weights
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def n_cells(self) -> int:
        nz, ny, nx = self.shape
        return nz * ny * nx

    @property
    def n_src(self) -> int:
        return int(self.src_ijk.shape[0])

    @property
    def n_rec(self) -> int:
        return int(self.rec_ijk.shape[0])

    def src_signals(self) -> np.ndarray:
        """Per-source signals [nt, n_src]: every source emits the same pulse."""
        return np.repeat(self.pulse[:, None], self.n_src, axis=1).copy()


# --------------------------------------------------------------------------
# elementary generators
# --------------------------------------------------------------------------

def time_step(dx: float, cfl: float = CFL, c_max: float = C_MAX) -> float:
    """dt = cfl * dx / c_max (Sec. 4.1)."""
    return cfl * dx / c_max


def toneburst(nt: int, dt: float, f0: float, cycles: int = 3) -> np.ndarray:
    """Hann-windowed toneburst sampled at t_n = n dt, zero after its end."""
    t = np.arange(nt, dtype=np.float64) * dt
    tb = cycles / f0
    s = np.sin(2.0 * np.pi * f0 * t) * 0.5 * (1.0 - np.cos(2.0 * np.pi * t / tb))
    s[t > tb] = 0.0
    return s


def golden_section_cap(n: int, center, radius: float, cap_deg: float = 90.0,
                       axis_sign: float = 1.0) -> np.ndarray:
    """n points spread over a spherical cap by the golden-section spiral.

    Returns float positions [n, 3] in voxel units (x, y, z).  The cap is the
    set of polar angles <= cap_deg measured from the +z (axis_sign=+1) or -z
    axis.
    """
    i = np.arange(n, dtype=np.float64)
    u_min = math.cos(math.radians(cap_deg))
    u = 1.0 - (i + 0.5) / n * (1.0 - u_min)          # cos(polar angle)
    phi = i * math.pi * (3.0 - math.sqrt(5.0))
    s = np.sqrt(np.maximum(0.0, 1.0 - u * u))
    cx, cy, cz = center
    return np.stack([cx + radius * s * np.cos(phi),
                     cy + radius * s * np.sin(phi),
                     cz + axis_sign * radius * u], axis=1)


def snap_to_voxels(pos: np.ndarray) -> np.ndarray:
    ijk = np.floor(pos + 0.5).astype(np.int32)
    keys = {tuple(v) for v in ijk.tolist()}
    if len(keys) != ijk.shape[0]:
        raise ValueError("two transducers snap to the same voxel")
    return ijk


def ball_masks(shape, center, radius: float, layer: int):
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    r = np.sqrt((x - center[0]) ** 2 + (y - center[1]) ** 2 + (z - center[2]) ** 2)
    gamma = r <= radius
    boundary = gamma & (r > radius - layer)
    return gamma.astype(np.uint8), boundary.astype(np.uint8)


def half_ball_masks(shape, center, radius: float, z_floor: int, layer: int):
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    r = np.sqrt((x - center[0]) ** 2 + (y - center[1]) ** 2 + (z - center[2]) ** 2)
    gamma = (r <= radius) & (z >= z_floor)
    boundary = gamma & ((r > radius - layer) | (z < z_floor + layer))
    return gamma.astype(np.uint8), boundary.astype(np.uint8)


def gaussian_inclusions(shape, gamma: np.ndarray, center, radius: float, z_floor: int,
                        dx: float, n_blobs: int, rng: np.random.Generator,
                        sigma_mm=(2.0, 6.0), amp_range=(-40.0, 90.0),
                        peak_range=None, clip=(1430.0, 1560.0),
                        background=C_FAT, outside=C_WATER):
    """Breast-like phantom: background + seeded Gaussian blobs inside Gamma.

    Blob centres are uniform in Gamma shrunk by the blob's sigma.  Either an
    amplitude range or a peak-speed range (peak = background + amplitude) is
    given.  Returns (c_true, c_eval) where c_eval has the blobs removed.
    """
    nz, ny, nx = shape
    c_eval = np.full(shape, outside, dtype=np.float64)
    c_eval[gamma.astype(bool)] = background
    field = np.zeros(shape, dtype=np.float64)
    zz = np.arange(nz, dtype=np.float64)[:, None, None]
    yy = np.arange(ny, dtype=np.float64)[None, :, None]
    xx = np.arange(nx, dtype=np.float64)[None, None, :]
    for _ in range(n_blobs):
        sig = rng.uniform(*sigma_mm) * 1e-3 / dx        # cells
        if peak_range is not None:
            amp = rng.uniform(*peak_range) - background
        else:
            amp = rng.uniform(*amp_range)
        r_in = max(radius - sig, 1.0)
        while True:
            p = rng.uniform(-r_in, r_in, size=3)
            q = np.array([center[0] + p[0], center[1] + p[1], center[2] + abs(p[2])])
            if np.linalg.norm(p) <= r_in and q[2] >= z_floor + sig:
                break
        # separable evaluation of exp(-|x-q|^2 / (2 sig^2))
        gx = np.exp(-((xx - q[0]) ** 2) / (2 * sig * sig))
        gy = np.exp(-((yy - q[1]) ** 2) / (2 * sig * sig))
        gz = np.exp(-((zz - q[2]) ** 2) / (2 * sig * sig))
        field += amp * (gz * gy * gx)
    c_true = c_eval.copy()
    inside = gamma.astype(bool)
    c_true[inside] = np.clip(background + field[inside], clip[0], clip[1])
    return c_true, c_eval


# --------------------------------------------------------------------------
# problem builders
# --------------------------------------------------------------------------

def _bowl_problem(name, shape, dx, nt, pml, n_elements, n_fire, phantom_seed,
                  enc_seed, layer, n_blobs, precision, amp_range=(-40.0, 90.0),
                  peak_range=None, clip=(1430.0, 1560.0), subset_seed=None):
    nz, ny, nx = shape
    z_b = pml + 2
    cx, cy = (nx - 1) / 2.0, (ny - 1) / 2.0
    r_b = math.floor(min(cx - pml - 2, cy - pml - 2, (nz - 1 - pml - 2) - z_b))
    r_g = math.floor(0.75 * r_b)
    pos = golden_section_cap(n_elements, (cx, cy, z_b), r_b, 90.0, +1.0)
    ijk = snap_to_voxels(pos)
    emitters = ijk[0::2]
    receivers = ijk[1::2]
    rng_sub = np.random.default_rng(enc_seed if subset_seed is None else subset_seed)
    sel = np.sort(rng_sub.choice(emitters.shape[0], size=n_fire, replace=False))
    src = np.ascontiguousarray(emitters[sel])
    gamma, boundary = half_ball_masks(shape, (cx, cy, z_b), r_g, z_b + 2, layer)
    rng = np.random.default_rng(phantom_seed)
    c_true, c_eval = gaussian_inclusions(shape, gamma, (cx, cy, z_b), r_g, z_b + 2, dx,
                                         n_blobs, rng, amp_range=amp_range,
                                         peak_range=peak_range, clip=clip)
    dt = time_step(dx)
    f0 = 1.0e6 * (0.5e-3 / dx)
    return Problem(
        name=name, shape=shape, dx=dx, dt=dt, nt=nt, c_ref=C_MAX, c_min=C_MIN,
        c_max=C_MAX, rho0=RHO0, pml=(pml, pml, pml), pml_alpha=PML_ALPHA,
        precision=precision, src_ijk=src, rec_ijk=np.ascontiguousarray(receivers),
        gamma=gamma, boundary=boundary, c_true=c_true, c_eval=c_eval,
        pulse=toneburst(nt, dt, f0), enc_seed=enc_seed,
        meta=dict(r_bowl=r_b, r_gamma=r_g, z_b=z_b, emitter_index=sel,
                  n_emitters=int(emitters.shape[0]), all_emitters=emitters),
    )


def _tiny(precision=8, nt=160):
    shape = (64, 64, 64)
    dx = 0.5e-3
    pml = 10
    ctr = (32.0, 32.0, 32.0)
    src = np.array([[32, 32, 16]], dtype=np.int32)        # -z pole, radius 16
    rec = snap_to_voxels(golden_section_cap(32, ctr, 16.0, 60.0, +1.0))
    gamma, boundary = ball_masks(shape, ctr, 12.0, 4)
    c_eval = np.full(shape, C_WATER)
    c_true = c_eval.copy()
    z, y, x = np.meshgrid(np.arange(64), np.arange(64), np.arange(64), indexing="ij")
    c_true[(x - 32) ** 2 + (y - 32) ** 2 + (z - 32) ** 2 <= 8 ** 2] = 1560.0
    dt = time_step(dx)
    return Problem(
        name="tiny", shape=shape, dx=dx, dt=dt, nt=nt, c_ref=C_MAX, c_min=C_MIN,
        c_max=C_MAX, rho0=RHO0, pml=(pml, pml, pml), pml_alpha=PML_ALPHA,
        precision=precision, src_ijk=src, rec_ijk=rec, gamma=gamma, boundary=boundary,
        c_true=c_true, c_eval=c_eval, pulse=toneburst(nt, dt, 1.0e6), enc_seed=1,
        meta=dict(r_gamma=12, layer=4),
    )


def make_config(name: str, index: int = 0, nt: Optional[int] = None,
                precision: Optional[int] = None) -> Problem:
    """Build one of the named workloads.

    tiny     : 64^3, 0.5 mm, PML 10, 160 steps, FP64, one source, 32 receivers
    c128     : 128^3, 0.5 mm, PML 10, 600 steps, FP32, 512-element bowl,
               8 encoded emitters, 20 blobs (phantom seed 2, encoding seed 1002)
    batch    : c128 with phantom seed 300+index and encoding seed 1300+index
    serve96  : 96^3 @ 1.0 mm, 300 steps;  serve160: 160^3 @ 0.75 mm, 600 steps;
    serve224 : 224x224x112 @ 0.5 mm, 1200 steps (PML 10, 8 encoded emitters)
    full     : 448x448x224, 0.5 mm, PML 20, 2200 steps, 2048-element bowl,
               32 encoded emitters, 60 inclusions (seed 5, encoding seed 1005)
    """
    if name == "tiny":
        p = _tiny(precision=precision or 8, nt=nt or 160)
    elif name == "c128":
        p = _bowl_problem("c128", (128, 128, 128), 0.5e-3, nt or 600, 10, 512, 8, 2, 1002,
                          8, 20, precision or 4)
    elif name == "batch":
        p = _bowl_problem(f"batch{index}", (128, 128, 128), 0.5e-3, nt or 600, 10, 512, 8,
                          300 + index, 1300 + index, 8, 20, precision or 4)
    elif name == "serve96":
        p = _bowl_problem("serve96", (96, 96, 96), 1.0e-3, nt or 300, 10, 512, 8,
                          40 + index, 4000 + index, 8, 20, precision or 4)
    elif name == "serve160":
        p = _bowl_problem("serve160", (160, 160, 160), 0.75e-3, nt or 600, 10, 512, 8,
                          41 + index, 4100 + index, 8, 20, precision or 4)
    elif name == "serve224":
        p = _bowl_problem("serve224", (112, 224, 224), 0.5e-3, nt or 1200, 10, 1024, 8,
                          42 + index, 4200 + index, 8, 20, precision or 4)
    elif name == "full":
        p = _bowl_problem("full", (224, 448, 448), 0.5e-3, nt or 2200, 20, 2048, 32, 5, 1005,
                          8, 60, precision or 4, peak_range=(1430.0, 1600.0),
                          clip=(1430.0, 1600.0))
    else:
        raise ValueError(f"unknown config {name!r}; known: {CONFIG_NAMES}")
    return p


def make_small(shape=(24, 28, 32), pml=3, nt=48, dx=0.5e-3, n_src=2, n_rec=12,
               layer=2, seed=7, precision=8, periodic=False, c_ref=C_MAX,
               homogeneous=False, f0=None, r_transducer=None, r_gamma=None) -> Problem:
    """A small problem for pins and parity: ball-shaped Gamma in the centre,
    sources and receivers on a sphere around it, seeded blobs inside Gamma.

    ``periodic=True`` removes the absorbing layer (PML size 0).  The sphere
    radii default to the largest that fit; they can be given (in cells).
    """
    nz, ny, nx = shape
    p = 0 if periodic else pml
    ctr = ((nx - 1) / 2.0, (ny - 1) / 2.0, (nz - 1) / 2.0)
    r_t = min(nx, ny, nz) / 2.0 - p - 1.5 if r_transducer is None else float(r_transducer)
    r_g = max(2.0, r_t - 3.0) if r_gamma is None else float(r_gamma)
    pos = golden_section_cap(2 * max(n_src, n_rec), ctr, r_t, 180.0, +1.0)
    ijk = snap_to_voxels(pos)
    src = np.ascontiguousarray(ijk[0::2][:n_src])
    rec = np.ascontiguousarray(ijk[1::2][:n_rec])
    gamma, boundary = ball_masks(shape, ctr, r_g, layer)
    rng = np.random.default_rng(seed)
    if homogeneous:
        c_true = np.full(shape, C_WATER)
        c_eval = c_true.copy()
    else:
        c_true, c_eval = gaussian_inclusions(shape, gamma, ctr, r_g, -10**6, dx, 3, rng,
                                             sigma_mm=(0.5, 1.0), amp_range=(-30.0, 60.0),
                                             clip=(1430.0, 1560.0))
    dt = time_step(dx)
    if f0 is None:
        f0 = 1.0e6 * (0.5e-3 / dx)
    return Problem(
        name=f"small{nx}x{ny}x{nz}", shape=tuple(shape), dx=dx, dt=dt, nt=nt, c_ref=c_ref,
        c_min=C_MIN, c_max=C_MAX, rho0=RHO0, pml=(p, p, p), pml_alpha=PML_ALPHA,
        precision=precision, src_ijk=src, rec_ijk=rec, gamma=gamma, boundary=boundary,
        c_true=c_true, c_eval=c_eval, pulse=toneburst(nt, dt, f0), enc_seed=seed + 1000,
        meta=dict(r_gamma=r_g, r_transducer=r_t),
    )


def random_traces(nt: int, n_rec: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """Seeded Gaussian traces [nt, n_rec], used as synthetic observed data."""
    rng = np.random.default_rng(seed)
    return scale * rng.standard_normal((nt, n_rec))
