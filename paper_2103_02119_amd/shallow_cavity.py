"""Shear flow in a shallow lid-driven cavity, H/L = 0.25 at Re = U L / nu =
100 (Sec. 5.5): the same flow on the square lattice (a = 1, 400 x 100
nodes) and on the rectangular one (a = 0.2, 100 x 125 nodes, finer across
the lid-normal gradient), RC collision, FP64.

Both lattices run at the same Mach number U / cs (cs2 = 1/3 on the square
lattice; on the rectangular one cs2 must stay below a^2 and takes
0.64 a^2), so the physical time that one step covers is about the same and
both need about as many steps; the saving is the node count (3.2x) and the
memory.  `compare` reports steps and wall time to a per-step residual, the
bytes of population storage, and the centreline profiles of the two
solutions (u on the vertical, v on the horizontal centreline) against each
other.  `scale` multiplies both grids, so that the comparison can also be
made where the GPU is bandwidth-bound rather than launch-bound.
"""
from __future__ import annotations

import time

import numpy as np

from . import lbm as L
from . import workloads as Wk

SQUARE = (400, 100, 1.0)
RECT = (100, 125, 0.2)
SETTLE_STEPS = 50  # steps before the smoothing step that removes the impulsive start's staggered mode


def run_case(nx, ny, a, re=100.0, mach=0.05 * np.sqrt(3.0), tol=1e-8, check_every=1000,
             max_steps=5_000_000, precision=L.LBM_FP64):
    """Runs one cavity from rest to a per-step residual <= tol; returns the
    run's record and its final (rho, ux, uy)."""
    import torch

    cs2 = Wk.default_cs2(a)
    U = mach * np.sqrt(cs2)
    nu = U * nx / re  # L = nx grid spacings of unit length
    tau = nu / cs2 + 0.5
    rates = [1.0, 1.0, 1.0, 1.0, 1.0 / tau, 1.0 / tau, 1.0, 1.0, 1.0]
    lat = L.Lattice(nx, ny, a, rates, bc_types=(1, 1, 1, 2), u_wall=((0, 0), (0, 0), (0, 0), (U, 0)),
                    cs2=cs2, collision=L.LBM_RC, precision=precision)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.step(SETTLE_STEPS)
    lat.smooth_step()
    steps, R = SETTLE_STEPS + 1, float("inf")
    while steps < max_steps:
        lat.step(check_every)
        steps += check_every
        R = lat.residual()
        if R <= tol:
            break
    wall = time.perf_counter() - t0
    fields = lat.moments()
    lat.close()
    rec = dict(nx=nx, ny=ny, a=a, nodes=nx * ny, cs2=cs2, U=U, nu=nu, tau=tau,
               steps=steps if R <= tol else None, seconds=round(wall, 3), residual=R,
               population_bytes=L.lbm_required_bytes(nx, ny, precision))
    return rec, fields


def centrelines(nx, ny, ux, uy, U):
    """u / U on the vertical centreline against y / H, v / U on the
    horizontal centreline against x / L (the two middle columns / rows are
    averaged when the count is even)."""
    def mid(v, axis, n):
        k = n // 2
        return np.take(v, k, axis) if n % 2 else 0.5 * (np.take(v, k - 1, axis) + np.take(v, k, axis))
    y = (np.arange(ny) + 0.5) / ny
    x = (np.arange(nx) + 0.5) / nx
    return (y, mid(ux, 1, nx) / U), (x, mid(uy, 0, ny) / U)


def compare(scale=1, re=100.0, tol=1e-8, check_every=1000, log=None):
    out = {}
    profiles = {}
    for name, (nx, ny, a) in (("square", SQUARE), ("rectangular", RECT)):
        rec, (rho, ux, uy) = run_case(nx * scale, ny * scale, a, re=re, tol=tol,
                                      check_every=check_every)
        out[name] = rec
        profiles[name] = centrelines(nx * scale, ny * scale, ux, uy, rec["U"])
        if log:
            log(f"shallow cavity {name}: {rec}")
    (ys, us), (xs, vs) = profiles["square"]
    (yr, ur), (xr, vr) = profiles["rectangular"]
    # the rectangular solution interpolated to the square lattice's points
    out["max_abs_diff_u_vertical"] = float(np.abs(np.interp(ys, yr, ur) - us).max())
    out["max_abs_diff_v_horizontal"] = float(np.abs(np.interp(xs, xr, vr) - vs).max())
    sq, rc = out["square"], out["rectangular"]
    out["node_ratio"] = sq["nodes"] / rc["nodes"]
    out["memory_ratio"] = sq["population_bytes"] / rc["population_bytes"]
    if sq["steps"] and rc["steps"]:
        out["step_ratio"] = sq["steps"] / rc["steps"]
        out["node_update_ratio"] = sq["steps"] * sq["nodes"] / (rc["steps"] * rc["nodes"])
    out["wall_ratio"] = sq["seconds"] / rc["seconds"]
    out["scale"] = scale
    out["re"] = re
    out["tol"] = tol
    return out


if __name__ == "__main__":
    import argparse
    import json

    ap = argparse.ArgumentParser(description="shallow cavity: square vs rectangular lattice")
    ap.add_argument("--scale", type=int, nargs="+", default=[1, 4])
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    log = lambda s: print(s, flush=True)  # noqa: E731
    res = [compare(scale=s, tol=args.tol, log=log) for s in args.scale]
    text = json.dumps(res)
    print(text, flush=True)
    if args.out:
        with open(args.out, "w") as fh:
            fh.write(text)
