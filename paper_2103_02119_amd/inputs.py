"""Seeded synthetic inputs for the rectangular-lattice LBM workloads.

This module holds only field recipes and random numbers: initial density and
velocity fields of the flows used in the paper's validation (Sec. 5) and of
the benchmark workloads, plus seeded noise.  It contains none of the method's
arithmetic (no equilibria, moments or collision), so both the HIP library's
tests and the CPU oracle can draw their inputs from it.

Coordinates: node (i, j) sits at x = i, y = j * a (lattice units, dx = 1,
dy = a); fields are float64 arrays of shape (ny, nx).
"""
from __future__ import annotations

import numpy as np

DEFAULT_SEED = 2103


def rng(seed: int = DEFAULT_SEED) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def coords(nx: int, ny: int, a: float):
    x = np.arange(nx, dtype=np.float64)[None, :] * np.ones((ny, 1))
    y = np.arange(ny, dtype=np.float64)[:, None] * a * np.ones((1, nx))
    return x, y


def taylor_green(nx: int, ny: int, a: float, u0: float, cs2: float, rho0: float = 1.0,
                 Lx: float | None = None, Ly: float | None = None):
    """Decaying Taylor-Green vortex on a doubly periodic box of size Lx x Ly
    (defaults: Lx = nx, Ly = ny * a).  Velocity
    ux = -u0 cos(kx x) sin(ky y), uy = u0 (kx/ky) sin(kx x) cos(ky y) and the
    incompressible pressure turned into density with p = rho cs2."""
    Lx = float(nx) if Lx is None else Lx
    Ly = float(ny) * a if Ly is None else Ly
    kx, ky = 2 * np.pi / Lx, 2 * np.pi / Ly
    x, y = coords(nx, ny, a)
    ux = -u0 * np.cos(kx * x) * np.sin(ky * y)
    uy = u0 * (kx / ky) * np.sin(kx * x) * np.cos(ky * y)
    p = -(rho0 * u0 * u0 / 4.0) * (np.cos(2 * kx * x) + (kx / ky) ** 2 * np.cos(2 * ky * y))
    rho = rho0 + p / cs2
    return rho, ux, uy


def shear_wave(nx: int, ny: int, a: float, u0: float, direction: str, rho0: float = 1.0):
    """Transverse shear wave: direction 'x' gives ux = u0 sin(ky y) (varies
    across y); direction 'y' gives uy = u0 sin(kx x) (varies across x)."""
    x, y = coords(nx, ny, a)
    rho = np.full((ny, nx), rho0)
    ux = np.zeros((ny, nx))
    uy = np.zeros((ny, nx))
    if direction == "x":
        ux = u0 * np.sin(2 * np.pi * y / (ny * a))
    else:
        uy = u0 * np.sin(2 * np.pi * x / nx)
    return rho, ux, uy


def shear_layer(nx: int, ny: int, a: float, u0: float = 0.04, kappa: float = 80.0,
                delta: float = 0.05, rho0: float = 1.0):
    """Doubly periodic shear layer on a square physical box (side nx):
    ux = u0 tanh(kappa (y' - 1/4)) for y' <= 1/2, u0 tanh(kappa (3/4 - y'))
    above; uy = delta u0 sin(2 pi (x' + 1/4)); x' = x/nx, y' = y/(ny a)."""
    x, y = coords(nx, ny, a)
    xp = x / nx
    yp = y / (ny * a)
    ux = np.where(yp <= 0.5, u0 * np.tanh(kappa * (yp - 0.25)), u0 * np.tanh(kappa * (0.75 - yp)))
    uy = delta * u0 * np.sin(2 * np.pi * (xp + 0.25))
    rho = np.full((ny, nx), rho0)
    return rho, ux, uy


def random_fields(seed: int, nx: int, ny: int, rho0: float = 1.0, rho_amp: float = 0.01,
                  u_amp: float = 0.02):
    """rho = rho0 (1 + rho_amp xi), u = u_amp xi', xi ~ U(-1, 1)."""
    g = rng(seed)
    rho = rho0 * (1.0 + rho_amp * g.uniform(-1, 1, (ny, nx)))
    ux = u_amp * g.uniform(-1, 1, (ny, nx))
    uy = u_amp * g.uniform(-1, 1, (ny, nx))
    return rho, ux, uy


def relative_noise(seed: int, nx: int, ny: int, amp: float = 1e-3):
    """Multiplicative population noise 1 + amp xi, xi ~ U(-1, 1), shape (9, ny, nx)."""
    g = rng(seed + 7919)
    return 1.0 + amp * g.uniform(-1, 1, (9, ny, nx))


def cavity_rest(nx: int, ny: int, rho0: float = 1.0):
    """Fluid at rest (the cavity's cold start)."""
    return np.full((ny, nx), rho0), np.zeros((ny, nx)), np.zeros((ny, nx))


def batch_sweep(n: int = 512, seed: int = DEFAULT_SEED, kinds=("cavity", "channel"),
                nx_range=(64, 512), re_range=(100.0, 5000.0), ratios=(0.25, 0.5, 1.0),
                speed: float = 0.05):
    """Seeded parameters of n independent cases: kind drawn from `kinds`,
    nx ~ U{nx_range}, r from `ratios`, ny = round(nx r) (at least 3),
    Re ~ U(re_range), velocity scale `speed` (lid speed or centreline
    velocity).  Plain parameters only; turning them into relaxation rates and
    forces is the caller's business."""
    g = rng(seed)
    out = []
    for _ in range(n):
        kind = kinds[int(g.integers(len(kinds)))]
        nx = int(g.integers(nx_range[0], nx_range[1] + 1))
        r = float(ratios[int(g.integers(len(ratios)))])
        ny = max(3, int(round(nx * r)))
        re = float(g.uniform(*re_range))
        out.append(dict(kind=kind, nx=nx, ny=ny, r=r, Re=re, U=speed))
    return out


def rect_obstacles(nx: int, ny: int, seed: int, nbox: int = 4, wmax: int = 5, hmax: int = 5,
                   wrap: bool = True):
    """Seeded obstacle mask (ny, nx) of uint8 (1 = solid): nbox axis-aligned
    rectangles of 1..wmax x 1..hmax nodes at uniform positions; with wrap they
    may straddle the periodic seams, otherwise they are clipped."""
    g = rng(seed)
    m = np.zeros((ny, nx), np.uint8)
    for _ in range(nbox):
        w, h = int(g.integers(1, wmax + 1)), int(g.integers(1, hmax + 1))
        x0, y0 = int(g.integers(0, nx)), int(g.integers(0, ny))
        for j in range(y0, y0 + h):
            for i in range(x0, x0 + w):
                if wrap:
                    m[j % ny, i % nx] = 1
                elif j < ny and i < nx:
                    m[j, i] = 1
    return m


def cavity_obstacles(nx: int, ny: int, seed: int, nmax: int = 3, margin: int = 4,
                     lid_gap: int = 12):
    """Seeded obstacles for a lid-driven cavity: 1..nmax axis-aligned boxes
    of nx/32..nx/4 by ny/16..ny/3 nodes, kept `margin` nodes from the walls
    and `lid_gap` rows below the lid.  Returns a (ny, nx) uint8 mask."""
    g = rng(seed)
    m = np.zeros((ny, nx), np.uint8)
    for _ in range(int(g.integers(1, nmax + 1))):
        w = int(g.integers(max(2, nx // 32), max(3, nx // 4) + 1))
        h = int(g.integers(max(2, ny // 16), max(3, ny // 3) + 1))
        x0 = int(g.integers(margin, max(margin + 1, nx - margin - w)))
        y0 = int(g.integers(margin, max(margin + 1, ny - lid_gap - h)))
        m[y0:y0 + h, x0:x0 + w] = 1
    return m


def warmstart_cases(n: int, seed: int = DEFAULT_SEED, re_range=(100.0, 5000.0),
                    ratios=(0.25, 0.5, 1.0)):
    """Seeded (Re, r, obstacle seed) parameters of n cavity cases."""
    g = rng(seed)
    return [dict(Re=float(g.uniform(*re_range)), r=float(ratios[int(g.integers(len(ratios)))]),
                 mask_seed=int(g.integers(1 << 30))) for _ in range(n)]
