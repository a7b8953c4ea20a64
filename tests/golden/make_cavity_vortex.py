"""Writes tests/golden/cavity_vortex_oracle.json: the FP64 oracle's lid-driven
cavity at the paper's own set-ups (Table 3, a = 0.5) after a fixed number of
steps from rest, for the primary-vortex pins (the paper's primary-vortex
table, Sec. 5.4) and the GPU parity test of the same runs.

  Re 100:  100 x 200 nodes, U = 0.04, cs2 = 0.18, tau = 0.736
  Re 1000: 150 x 300 nodes, U = 0.02, cs2 = 0.04, tau = 0.5745
           (Table 3 prints nu = 0.0003 for this row; tau and cs2 give 0.00298)

Both collisions (RC, RNR), the paper's rates (omega_4 = omega_5 = 1/tau, all
others 1), half-way bounce-back walls with the lid on the top face.  Stored
per run: the step count, the per-step residual of the last step, the
primary-vortex centre (tests/cavity_vortex.py) and the velocity on the two
middle columns and the two middle rows, as exact decimal strings of the
doubles.  Calls only the oracle (which starts from the rest state).  Run
from the repository root:

    python tests/golden/make_cavity_vortex.py

It takes about 25 minutes on 8 cores.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import oracle as O  # noqa: E402
from cavity_vortex import primary_vortex  # noqa: E402

OUT = os.path.join(HERE, "cavity_vortex_oracle.json")

CASES = {
    "re100": dict(nx=100, ny=200, a=0.5, U=0.04, cs2=0.18, tau=0.736, steps=40_000),
    "re1000": dict(nx=150, ny=300, a=0.5, U=0.02, cs2=0.04, tau=0.5745, steps=250_000),
}


def params(c, coll):
    return O.make_params(c["nx"], c["ny"], c["a"], c["cs2"], O.paper_rates(c["tau"]),
                         collision=coll, bc=(1, 1, 1, 2),
                         u_wall=((0, 0), (0, 0), (0, 0), (c["U"], 0)))


def run(c, coll):
    p = params(c, coll)
    f = O.run(p, O.init(p), c["steps"] - 1)
    _, ux0, uy0 = O.moments(p, f)
    f = O.run(p, f, 1)
    _, ux, uy = O.moments(p, f)
    R = float(np.sqrt(((ux - ux0) ** 2 + (uy - uy0) ** 2).sum() / (ux ** 2 + uy ** 2).sum()))
    xc, yc, psi = primary_vortex(ux, uy, c["a"])
    nx, ny = c["nx"], c["ny"]
    return dict(steps=c["steps"], residual=R, centre=[xc, yc], psi_min=psi,
                ux_cols=[[repr(float(v)) for v in ux[:, i]] for i in (nx // 2 - 1, nx // 2)],
                uy_rows=[[repr(float(v)) for v in uy[j, :]] for j in (ny // 2 - 1, ny // 2)])


def main():
    out = dict(cases={k: {q: v for q, v in c.items()} for k, c in CASES.items()}, runs={})
    for name, c in CASES.items():
        for coll, cname in ((O.RC, "RC"), (O.RNR, "RNR")):
            t0 = time.perf_counter()
            out["runs"][f"{name}_{cname}"] = r = run(c, coll)
            print(f"{name} {cname}: centre ({r['centre'][0]:.4f}, {r['centre'][1]:.4f}), "
                  f"R {r['residual']:.2e}, {time.perf_counter() - t0:.0f} s", flush=True)
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
