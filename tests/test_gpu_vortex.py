"""The paper's lid-driven cavities (Table 3, a = 0.5; Re 100 on 100 x 200
nodes for 40 000 steps, Re 1000 on 150 x 300 nodes for 250 000 steps) on the
GPU in FP64 against the oracle's stored runs of the same length
(tests/golden/cavity_vortex_oracle.json): the velocity on the two middle
columns and rows, and the primary-vortex centre against the paper's
primary-vortex table (Sec. 5.4)."""
import numpy as np
import pytest

from cavity_vortex import primary_vortex
from paper_2103_02119_amd import lbm as L
from test_oracle_vortex import TOL_CENTRE, golden, printed_centres

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


@pytest.mark.parametrize("run", ["re100_RC", "re100_RNR", "re1000_RC", "re1000_RNR"])
def test_gpu_cavity_matches_the_oracle_run_and_the_paper(run, record_property):
    g = golden()
    name, cname = run.split("_")
    c = g["cases"][name]
    ref = g["runs"][run]
    print(f"case: {run} {c['nx']}x{c['ny']} {c['steps']} steps", flush=True)
    tau = c["tau"]
    lat = L.Lattice(c["nx"], c["ny"], c["a"], [1, 1, 1, 1, 1 / tau, 1 / tau, 1, 1, 1],
                    bc_types=(1, 1, 1, 2), u_wall=((0, 0), (0, 0), (0, 0), (c["U"], 0)),
                    cs2=c["cs2"], collision=L.LBM_RC if cname == "RC" else L.LBM_RNR)
    lat.set_fields()
    lat.step(c["steps"])
    R = lat.residual()
    _, ux, uy = lat.moments()
    lat.close()
    nx, ny = c["nx"], c["ny"]
    got = np.concatenate([ux[:, nx // 2 - 1], ux[:, nx // 2], uy[ny // 2 - 1, :], uy[ny // 2, :]])
    want = np.array([float(v) for v in ref["ux_cols"][0] + ref["ux_cols"][1]
                     + ref["uy_rows"][0] + ref["uy_rows"][1]])
    err = float(np.abs(got - want).max() / np.abs(want).max())
    record_property("gpu_vs_oracle_centrelines", err)
    print(f"{run}: GPU vs oracle centrelines {err:.3e}, residual {R:.2e} "
          f"(oracle {ref['residual']:.2e})", flush=True)
    assert err < TOL64, err
    x, y, _ = primary_vortex(ux, uy, c["a"])
    px, py = printed_centres()[run]
    assert abs(x - px) < TOL_CENTRE and abs(y - py) < TOL_CENTRE, ((x, y), (px, py))
