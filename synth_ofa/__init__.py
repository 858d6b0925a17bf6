"""Seeded synthetic focus-array workloads.

The paper (Liu et al., "Fast generation of arbitrary optical focus array",
arXiv:2206.12661) evaluates its method on a 1000x1000 phase-only SLM pupil
(Table 1) with a 9x9 grid of foci and a 66-focus random pattern (Sec. 2,
Fig. 2), and on experimental patterns whose data are not published.  None of
those inputs exist as files, so every workload here is generated from a seed
with the shapes, coordinate ranges and intensity distributions of the paper's
kind of problem.

This module is input plumbing only.  It draws pupil amplitudes, sampling
coordinates, focus positions, target intensities and initial phases; it holds
none of the method's arithmetic (no propagation, no weighting, no projection).
Both the FP64 oracle and the GPU library consume exactly the arrays it returns.

Conventions (shared by every consumer):
  * the pupil is ``ny x nx`` samples, row-major, rows along y / v, columns
    along x / u;
  * pupil coordinates are in pixels, centred: ``u_i = i - (nx - 1) / 2``;
  * focal coordinates are in focal units ``lambda f / (N_axis du)``, so the
    kernel phase is ``2 pi s u x`` with ``s_x = 1 / nx`` and ``s_y = 1 / ny``;
  * the initial phase is drawn in float64 on [0, 2 pi) and rounded to float32;
    both sides use the float32 values;
  * every config k draws from ``numpy.random.default_rng([12661, k])`` in the
    order: focus positions, jitter, target intensities, initial phase.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

SEED_BASE = 12661


@dataclass
class Hologram:
    """One phase-retrieval problem: pupil, sampling, foci and start phase."""

    name: str
    ny: int
    nx: int
    amplitude: np.ndarray      # float32 [ny, nx], >= 0, zero outside the aperture
    u: np.ndarray              # float64 [nx], pupil x coordinates (pixels)
    v: np.ndarray              # float64 [ny], pupil y coordinates (pixels)
    s_x: float                 # kernel phase scale along x
    s_y: float                 # kernel phase scale along y
    fx: np.ndarray             # float64 [N], focus x (focal units)
    fy: np.ndarray             # float64 [N], focus y (focal units)
    target: np.ndarray         # float64 [N], target intensities
    phi0: np.ndarray           # float32 [ny, nx], initial phase
    n_iter: int = 20
    meta: dict = field(default_factory=dict)
    fz: Optional[np.ndarray] = None   # float64 [N], axial positions (None: focal plane)

    @property
    def n_foci(self) -> int:
        return int(self.fx.shape[0])


def centred(n: int) -> np.ndarray:
    """Centred pixel coordinates ``i - (n - 1) / 2`` as float64."""
    return np.arange(n, dtype=np.float64) - (n - 1) / 2.0


def disc(ny: int, nx: int, radius: float) -> np.ndarray:
    """Closed disc ``r^2 <= R^2`` on the centred pixel grid (bool [ny, nx])."""
    y = centred(ny)[:, None]
    x = centred(nx)[None, :]
    return (x * x + y * y) <= radius * radius


def gaussian_amplitude(ny: int, nx: int, w: float) -> np.ndarray:
    """Amplitude of a Gaussian beam whose intensity falls to 1/e^2 at radius w."""
    y = centred(ny)[:, None]
    x = centred(nx)[None, :]
    return np.exp(-(x * x + y * y) / (w * w))


def initial_phase(rng: np.random.Generator, ny: int, nx: int) -> np.ndarray:
    """Uniform [0, 2 pi) in float64, rounded to float32."""
    return rng.uniform(0.0, 2.0 * np.pi, size=(ny, nx)).astype(np.float32)


def grid_foci(k_rows: int, k_cols: int, pitch: float):
    """Square grid of foci centred at 0; focus n = i * k_cols + j sits at
    (x_j, y_i) with x_j = pitch (j - (k_cols - 1) / 2)."""
    xs = pitch * (np.arange(k_cols, dtype=np.float64) - (k_cols - 1) / 2.0)
    ys = pitch * (np.arange(k_rows, dtype=np.float64) - (k_rows - 1) / 2.0)
    fy, fx = np.meshgrid(ys, xs, indexing="ij")
    return fx.reshape(-1).copy(), fy.reshape(-1).copy()


def dart_throw(rng: np.random.Generator, n: int, half_width: float,
               min_spacing: float, max_tries: int = 10_000_000) -> np.ndarray:
    """Sequential dart throwing: uniform candidates in [-h, h]^2, kept when no
    kept point lies closer than ``min_spacing`` (Euclidean)."""
    pts = np.empty((n, 2), dtype=np.float64)
    k = 0
    tries = 0
    ms2 = min_spacing * min_spacing
    while k < n:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("dart throwing did not converge")
        p = rng.uniform(-half_width, half_width, size=2)
        if k:
            d = pts[:k] - p
            if np.min(np.einsum("ij,ij->i", d, d)) < ms2:
                continue
        pts[k] = p
        k += 1
    return pts


def _assemble(name, ny, nx, amp, fx, fy, target, phi0, n_iter, **meta) -> Hologram:
    return Hologram(
        name=name, ny=ny, nx=nx,
        amplitude=np.ascontiguousarray(amp, dtype=np.float32),
        u=centred(nx), v=centred(ny), s_x=1.0 / nx, s_y=1.0 / ny,
        fx=np.ascontiguousarray(fx, dtype=np.float64),
        fy=np.ascontiguousarray(fy, dtype=np.float64),
        target=np.ascontiguousarray(target, dtype=np.float64),
        phi0=np.ascontiguousarray(phi0, dtype=np.float32),
        n_iter=n_iter, meta=dict(meta))


def config1() -> Hologram:
    """64x64 pupil, closed disc R = 32 px, unit amplitude; 4x4 grid of foci at
    pitch 5.5 focal units centred on 0; equal targets; 20 iterations."""
    rng = np.random.default_rng([SEED_BASE, 1])
    ny = nx = 64
    amp = disc(ny, nx, 32.0).astype(np.float32)
    fx, fy = grid_foci(4, 4, 5.5)
    target = np.ones(fx.shape[0])
    phi0 = initial_phase(rng, ny, nx)
    return _assemble("plain-64x64-disc-4x4grid", ny, nx, amp, fx, fy, target, phi0, 20)


def config2() -> Hologram:
    """512x512 pupil, disc R = 256 px, Gaussian amplitude (1/e^2 radius 200 px);
    10x10 grid at pitch 7.3 plus uniform jitter in [-0.5, 0.5] per axis per
    focus; equal targets; 50 iterations."""
    rng = np.random.default_rng([SEED_BASE, 2])
    ny = nx = 512
    amp = np.where(disc(ny, nx, 256.0), gaussian_amplitude(ny, nx, 200.0), 0.0)
    fx, fy = grid_foci(10, 10, 7.3)
    jitter = rng.uniform(-0.5, 0.5, size=(fx.shape[0], 2))
    fx = fx + jitter[:, 0]
    fy = fy + jitter[:, 1]
    target = np.ones(fx.shape[0])
    phi0 = initial_phase(rng, ny, nx)
    return _assemble("plain-512x512-gauss-10x10jitter", ny, nx, amp, fx, fy, target, phi0, 50)


def config3() -> Hologram:
    """1152 x 1920 pupil, full rectangle, unit amplitude; 1000 foci by dart
    throwing in a 200x200 focal-unit ROI with minimum spacing 2; targets
    uniform in [0.5, 1]; 100 iterations."""
    rng = np.random.default_rng([SEED_BASE, 3])
    ny, nx = 1152, 1920
    amp = np.ones((ny, nx), dtype=np.float32)
    pts = dart_throw(rng, 1000, 100.0, 2.0)
    target = rng.uniform(0.5, 1.0, size=1000)
    phi0 = initial_phase(rng, ny, nx)
    return _assemble("gsw-1152x1920-1000foci", ny, nx, amp, pts[:, 0], pts[:, 1],
                     target, phi0, 100)


def config4(count: int = 64) -> List[Hologram]:
    """Batch of independent holograms: square pupils with side log-uniform in
    [256, 1024] and inscribed closed-disc apertures; foci counts log-uniform in
    [16, 2000] at uniform positions within +-0.4 side focal units (exact
    duplicates redrawn); targets uniform in [0.2, 1]; 50 iterations each.
    Per hologram the draw order is side, focus count, positions, targets, phase."""
    rng = np.random.default_rng([SEED_BASE, 4])
    out = []
    for h in range(count):
        side = int(round(float(np.exp(rng.uniform(np.log(256.0), np.log(1024.0))))))
        n = int(round(float(np.exp(rng.uniform(np.log(16.0), np.log(2000.0))))))
        lim = 0.4 * side
        pts = rng.uniform(-lim, lim, size=(n, 2))
        while True:
            _, first = np.unique(pts, axis=0, return_index=True)
            if first.shape[0] == n:
                break
            dup = np.setdiff1d(np.arange(n), first)
            pts[dup] = rng.uniform(-lim, lim, size=(dup.shape[0], 2))
        target = rng.uniform(0.2, 1.0, size=n)
        amp = disc(side, side, side / 2.0).astype(np.float32)
        phi0 = initial_phase(rng, side, side)
        out.append(_assemble(f"batch-{h:02d}-{side}px-{n}foci", side, side, amp,
                             pts[:, 0], pts[:, 1], target, phi0, 50, index=h))
    return out


def config5_targets(k: int = 50) -> np.ndarray:
    """Target pattern T_ij = 1 + 0.5 sin(2 pi i / 17) cos(2 pi j / 23) on a k x k
    grid, focus n = i * k + j, normalised to sum 1."""
    i = np.arange(k, dtype=np.float64)[:, None]
    j = np.arange(k, dtype=np.float64)[None, :]
    t = 1.0 + 0.5 * np.sin(2.0 * np.pi * i / 17.0) * np.cos(2.0 * np.pi * j / 23.0)
    t = t.reshape(-1)
    return t / t.sum()


def config5() -> Hologram:
    """1152 x 1920 pupil, full rectangle, unit amplitude; 50x50 grid at pitch
    3.7 (x_j = 3.7 (j - 24.5)); targets from ``config5_targets``; phase
    optimised by gradient descent (Adam, lr 0.05, 200 steps)."""
    rng = np.random.default_rng([SEED_BASE, 5])
    ny, nx = 1152, 1920
    amp = np.ones((ny, nx), dtype=np.float32)
    fx, fy = grid_foci(50, 50, 3.7)
    target = config5_targets(50)
    phi0 = initial_phase(rng, ny, nx)
    return _assemble("adam-1152x1920-50x50grid", ny, nx, amp, fx, fy, target, phi0, 200,
                     lr=0.05, betas=(0.9, 0.999), eps=1e-8, eta_weight=0.1)


def config5_gradcheck() -> Hologram:
    """Gradient-check sub-case: the 64x64 disc pupil of ``config1`` with a 4x4
    grid at pitch 3.7 and the top-left 4x4 block of the config-5 pattern."""
    rng = np.random.default_rng([SEED_BASE, 55])
    ny = nx = 64
    amp = disc(ny, nx, 32.0).astype(np.float32)
    fx, fy = grid_foci(4, 4, 3.7)
    i = np.arange(4, dtype=np.float64)[:, None]
    j = np.arange(4, dtype=np.float64)[None, :]
    t = (1.0 + 0.5 * np.sin(2.0 * np.pi * i / 17.0) * np.cos(2.0 * np.pi * j / 23.0)).reshape(-1)
    phi0 = initial_phase(rng, ny, nx)
    return _assemble("gradcheck-64x64-4x4grid", ny, nx, amp, fx, fy, t / t.sum(), phi0, 1)


# Foci-count sweep (Sec. 2, Fig. 2(e)): uniform k x k arrays on the
# 1000 x 1000 SLM area of Table 1 at the 20-camera-pixel minimum gap, which is
# 4.39 focal units in the units of Table 1 (at most 227 x 227 foci).
SWEEP_PITCH = 4.39


def sweep_case(k: int, n_iter: int = 100) -> Hologram:
    """1000 x 1000 unit-amplitude pupil (the full SLM area); k x k grid at
    pitch 4.39 focal units; equal targets."""
    rng = np.random.default_rng([SEED_BASE, 6, k])
    ny = nx = 1000
    amp = np.ones((ny, nx), dtype=np.float32)
    fx, fy = grid_foci(k, k, SWEEP_PITCH)
    phi0 = initial_phase(rng, ny, nx)
    return _assemble(f"sweep-{k}x{k}", ny, nx, amp, fx, fy, np.ones(fx.shape[0]), phi0, n_iter)


def double_heart(pitch: float = 0.8, n_iter: int = 100) -> Hologram:
    """A continuous pattern (Sec. 2, Fig. 3(k)-(m) stand-in): two heart
    shapes filled with samples at a pitch below the diffraction limit (0.8
    focal units), with a smooth nonuniform target ramp across the pattern, on
    the 1000 x 1000 pupil.  Heart outline: x = 16 sin^3 t,
    y = 13 cos t - 5 cos 2t - 2 cos 3t - cos 4t, scaled to 60 focal units
    wide, the two centred at x = -40 and x = +40."""
    rng = np.random.default_rng([SEED_BASE, 7])
    ny = nx = 1000
    amp = np.ones((ny, nx), dtype=np.float32)
    t = np.linspace(0.0, 2.0 * np.pi, 2001)
    hx = 16.0 * np.sin(t) ** 3
    hy = 13.0 * np.cos(t) - 5.0 * np.cos(2 * t) - 2.0 * np.cos(3 * t) - np.cos(4 * t)
    sc = 60.0 / 32.0
    hx, hy = hx * sc, hy * sc

    def inside(px, py):   # even-odd rule against the closed outline
        c = np.zeros(px.shape, dtype=bool)
        x0, y0 = hx[:-1], hy[:-1]
        x1, y1 = hx[1:], hy[1:]
        for a, b, cc, d in zip(x0, y0, x1, y1):
            cond = (b > py) != (d > py)
            xi = a + (py - b) * (cc - a) / np.where(d != b, d - b, 1.0)
            c ^= cond & (px < xi)
        return c

    g = np.arange(-40.0, 40.0 + 1e-9, pitch)
    gx, gy = np.meshgrid(g, g)
    keep = inside(gx.ravel(), gy.ravel())
    px, py = gx.ravel()[keep], gy.ravel()[keep]
    fx = np.concatenate([px - 40.0, px + 40.0])
    fy = np.concatenate([py, py])
    target = 0.5 + 0.5 * (fx - fx.min()) / (fx.max() - fx.min())
    phi0 = initial_phase(rng, ny, nx)
    return _assemble("double-heart", ny, nx, amp, fx, fy, target, phi0, n_iter)


def volume_case(seed: int, ny: int, nx: int, n_per_plane: int, planes=(-30.0, 0.0, 30.0), *,
                radius: Optional[float] = None, roi: Optional[float] = None,
                grid: Optional[tuple] = None, n_iter: int = 20) -> Hologram:
    """3-D foci (Sec. 3 outlook: the axial position of a focus set by a
    defocus phase of the pupil): ``n_per_plane`` random foci (or a k x l grid,
    shifted by half a pitch from plane to plane) on each axial plane z of
    ``planes``; targets uniform in [0.3, 1]."""
    rng = np.random.default_rng([SEED_BASE, 2000 + seed])
    lim = roi if roi is not None else 0.3 * min(ny, nx)
    fxs, fys, fzs = [], [], []
    for q, z in enumerate(planes):
        if grid is not None:
            gx, gy = grid_foci(grid[0], grid[1], 3.1)
            gx, gy = gx + 1.55 * q, gy + 1.55 * q
        else:
            pts = rng.uniform(-lim, lim, size=(n_per_plane, 2))
            gx, gy = pts[:, 0], pts[:, 1]
        fxs.append(gx)
        fys.append(gy)
        fzs.append(np.full(gx.shape[0], float(z)))
    fx, fy, fz = np.concatenate(fxs), np.concatenate(fys), np.concatenate(fzs)
    target = rng.uniform(0.3, 1.0, size=fx.shape[0])
    amp = np.ones((ny, nx)) if radius is None else disc(ny, nx, radius).astype(np.float64)
    phi0 = initial_phase(rng, ny, nx)
    h = _assemble(f"volume-{seed}-{ny}x{nx}-{fx.shape[0]}", ny, nx, amp, fx, fy, target, phi0,
                  n_iter)
    h.fz = np.ascontiguousarray(fz)
    return h


def config(k: int):
    return {1: config1, 2: config2, 3: config3, 4: config4, 5: config5}[k]()


def random_case(seed: int, ny: int, nx: int, n_foci: int, *, radius: Optional[float] = None,
                roi: Optional[float] = None, grid: Optional[tuple] = None,
                amplitude: str = "uniform", n_iter: int = 5,
                u: Optional[np.ndarray] = None, v: Optional[np.ndarray] = None) -> Hologram:
    """Small seeded case for parity tests.  ``radius`` gives a closed-disc
    aperture (default: full rectangle); ``grid=(k, l)`` places k x l grid foci
    at pitch 3.1 (``n_foci`` ignored), otherwise foci are uniform in
    +-``roi`` (default 0.3 * min(ny, nx)) focal units; ``amplitude`` is
    ``uniform`` or ``random`` (uniform in [0.2, 1] inside the aperture)."""
    rng = np.random.default_rng([SEED_BASE, 1000 + seed])
    if grid is not None:
        fx, fy = grid_foci(grid[0], grid[1], 3.1)
    else:
        lim = roi if roi is not None else 0.3 * min(ny, nx)
        pts = rng.uniform(-lim, lim, size=(n_foci, 2))
        fx, fy = pts[:, 0].copy(), pts[:, 1].copy()
    target = rng.uniform(0.3, 1.0, size=fx.shape[0])
    ap = np.ones((ny, nx), dtype=bool) if radius is None else disc(ny, nx, radius)
    if amplitude == "random":
        amp = np.where(ap, rng.uniform(0.2, 1.0, size=(ny, nx)), 0.0)
    else:
        amp = ap.astype(np.float64)
    phi0 = initial_phase(rng, ny, nx)
    h = _assemble(f"random-{seed}-{ny}x{nx}-{fx.shape[0]}", ny, nx, amp, fx, fy, target,
                  phi0, n_iter)
    if u is not None:
        h.u = np.ascontiguousarray(u, dtype=np.float64)
    if v is not None:
        h.v = np.ascontiguousarray(v, dtype=np.float64)
    return h


__all__ = [
    "Hologram", "centred", "disc", "gaussian_amplitude", "initial_phase", "grid_foci",
    "dart_throw", "config1", "config2", "config3", "config4", "config5",
    "config5_targets", "config5_gradcheck", "config", "random_case", "SEED_BASE",
]
