"""Problem set-up helpers: physical parameters -> the library's cases.

The relaxation rates follow the paper's choice (Sec. 2.3): omega_4 = omega_5
= 1/tau with nu = cs2 (tau - 1/2) (Eq. 32), every other rate 1.  The default
cs2 is min(1/3, 0.64 a^2), the rule of the paper's channel runs (Table 1) at
a = 1, 0.5 and 0.25; its cavity runs (Table 3) use cavity_cs2.  cs2 must
stay below min(1, a^2) for positive rest weights.
"""
from __future__ import annotations

from . import lbm as L


def default_cs2(a: float) -> float:
    return min(1.0 / 3.0, 0.64 * a * a)


def cavity_cs2(a: float) -> float:
    """Squared sound speed of the paper's cavity runs (Table 3): 1/3 on the
    square lattice, 0.04 at a = 0.5 and a = 0.25 (min(0.04, 0.64 a^2) below 1)."""
    return 1.0 / 3.0 if a >= 1.0 else min(0.04, 0.64 * a * a)


def paper_rates(nu: float, cs2: float):
    tau = nu / cs2 + 0.5
    return [1.0, 1.0, 1.0, 1.0, 1.0 / tau, 1.0 / tau, 1.0, 1.0, 1.0]


def cavity_case(nx: int, ny: int, a: float, Re: float, U: float, cs2: float | None = None):
    """Lid-driven cavity: walls on three sides, the top (y-max) face moving at
    (U, 0); Re = U nx / nu (the width in lattice units)."""
    cs2 = default_cs2(a) if cs2 is None else cs2
    nu = U * nx / Re
    return L.make_case(nx, ny, a, paper_rates(nu, cs2),
                       bc_types=(L.LBM_BC_WALL, L.LBM_BC_WALL, L.LBM_BC_WALL, L.LBM_BC_MOVING_WALL),
                       u_wall=((0, 0), (0, 0), (0, 0), (U, 0)), cs2=cs2)


def channel_case(nx: int, ny: int, a: float, Re: float, U: float, cs2: float | None = None,
                 rho0: float = 1.0):
    """Body-force-driven channel, periodic in x, walls in y (Sec. 5.1):
    height H = ny a, Re = U H / nu with U the centreline velocity of the
    Poiseuille profile, so Fx = 8 rho0 nu U / H^2."""
    cs2 = default_cs2(a) if cs2 is None else cs2
    H = ny * a
    nu = U * H / Re
    Fx = 8.0 * rho0 * nu * U / (H * H)
    return L.make_case(nx, ny, a, paper_rates(nu, cs2),
                       bc_types=(L.LBM_BC_PERIODIC, L.LBM_BC_PERIODIC, L.LBM_BC_WALL, L.LBM_BC_WALL),
                       cs2=cs2, force=(Fx, 0.0), rho0=rho0)


def sweep_cases(params):
    """lbm_case list for parameter dicts of inputs.batch_sweep."""
    make = {"cavity": cavity_case, "channel": channel_case}
    return [make[p["kind"]](p["nx"], p["ny"], p["r"], p["Re"], p["U"]) for p in params]
