"""FP32 deviation storage at the converged state of the 512 x 1024, a = 0.5,
Re 1000 lid-driven cavity (lid 0.05, cs2 0.16), against the FP64 run.

The FP64 path is pinned to the oracle per step (1e-12) and over thousands of
steps; the oracle itself cannot run the ~600 000 steps this cavity needs to
reach a per-step residual of 1e-8 (about 3e11 node updates), so the FP64 GPU
run stands in for it here.  At the step where the FP64 run reaches 1e-8,
both FP32-storage modes must be within the 1e-5 velocity bar (max |du| /
max |u|).  Run on past that point, rounding noise keeps exciting the
cavity's weakly damped (1, 1) acoustic mode and the difference grows to a
few 1e-5 by 1 000 000 steps; that drift is recorded and held below the
floor measured for it (1e-4 with FP32 arithmetic, 5e-5 with FP64
arithmetic)."""
import numpy as np
import pytest

from paper_2103_02119_amd import inputs as I
from paper_2103_02119_amd import lbm as L

pytestmark = pytest.mark.gpu

NX, NY, A, CS2, U, RE = 512, 1024, 0.5, 0.16, 0.05, 1000.0
LONG = 1_000_000


def cavity(prec):
    nu = U * NX / RE
    tau = nu / CS2 + 0.5
    lat = L.Lattice(NX, NY, A, [1, 1, 1, 1, 1 / tau, 1 / tau, 1, 1, 1], bc_types=(1, 1, 1, 2),
                    u_wall=((0, 0), (0, 0), (0, 0), (U, 0)), cs2=CS2, precision=prec)
    lat.set_fields(*I.cavity_rest(NX, NY))
    return lat


def diff(lat, ux64, uy64):
    _, ux, uy = lat.moments()
    return float(np.hypot(ux - ux64, uy - uy64).max() / np.hypot(ux64, uy64).max())


def test_fp32_storage_error_at_the_converged_cavity(record_property):
    print("case: fp64 cavity 512x1024 to R <= 1e-8", flush=True)
    ref = cavity(L.LBM_FP64)
    steps, R = 0, 1.0
    while R > 1e-8 and steps < LONG:
        ref.step(10_000)
        steps += 10_000
        R = ref.residual()
    assert R <= 1e-8, R
    _, ux64, uy64 = ref.moments()
    record_property("steps_to_1e-8_fp64", steps)
    errs, drift = {}, {}
    lats = {}
    for prec, name in ((L.LBM_FP32_DEV, "fp32"), (L.LBM_FP32_DEV_F64, "fp32_f64arith")):
        print(f"case: {name} cavity 512x1024, {steps} steps", flush=True)
        lats[name] = lat = cavity(prec)
        lat.step(steps)
        errs[name] = diff(lat, ux64, uy64)
        record_property(f"steady_error_{name}", errs[name])
    print("steps", steps, "errors at the converged state", errs, flush=True)
    ref.step(LONG - steps)
    _, ux64, uy64 = ref.moments()
    ref.close()
    for name, lat in lats.items():
        lat.step(LONG - steps)
        drift[name] = diff(lat, ux64, uy64)
        record_property(f"error_after_{LONG}_steps_{name}", drift[name])
        lat.close()
    print("errors after", LONG, "steps", drift, flush=True)
    assert errs["fp32"] < 1e-5 and errs["fp32_f64arith"] < 1e-5, errs
    assert drift["fp32"] < 1e-4 and drift["fp32_f64arith"] < 5e-5, drift
