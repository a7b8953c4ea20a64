"""The whole scheme on the paper's own lid-driven cavities (Table 3, a = 0.5)
against the primary-vortex centres it prints (Sec. 5.4): the moving lid of
Eq. 57-59, the corner links and both collisions together.

tests/golden/cavity_vortex_oracle.json holds the oracle's runs from rest
(Re 100: 40 000 steps, Re 1000: 250 000 steps, when the centre has settled
to within 1e-3 of its steady position), written by
tests/golden/make_cavity_vortex.py, which calls only the oracle.  The
printed centres are tests/golden/primary_vortex_printed.txt.  The Re 100 RC
run is repeated here and must reproduce the stored run bit for bit; the
Re 1000 runs (about 10 minutes each on 8 cores) are repeated only with
LBM_SLOW_PINS=1."""
import json
import os

import numpy as np
import pytest

from cavity_vortex import primary_vortex

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
TOL_CENTRE = 0.01  # the paper's own RC and RNR centres differ by up to 0.003


def printed_centres():
    out = {}
    with open(os.path.join(GOLDEN, "primary_vortex_printed.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            re_, method, x, y = line.split()
            out[f"re{re_}_{method}"] = (float(x), float(y))
    return out


def golden():
    with open(os.path.join(GOLDEN, "cavity_vortex_oracle.json")) as fh:
        return json.load(fh)


def test_printed_table_has_both_collisions_at_both_reynolds_numbers():
    assert sorted(printed_centres()) == ["re1000_RC", "re1000_RNR", "re100_RC", "re100_RNR"]


@pytest.mark.parametrize("run", ["re100_RC", "re100_RNR", "re1000_RC", "re1000_RNR"])
def test_oracle_primary_vortex_matches_the_paper(run):
    g = golden()["runs"][run]
    px, py = printed_centres()[run]
    x, y = g["centre"]
    assert abs(x - px) < TOL_CENTRE and abs(y - py) < TOL_CENTRE, (run, (x, y), (px, py))
    assert g["residual"] < 1e-6  # near the steady state


def _rerun(name, coll, orc):
    g = golden()
    c = g["cases"][name]
    p = orc.make_params(c["nx"], c["ny"], c["a"], c["cs2"], orc.paper_rates(c["tau"]),
                        collision=coll, bc=(1, 1, 1, 2),
                        u_wall=((0, 0), (0, 0), (0, 0), (c["U"], 0)))
    f = orc.run(p, orc.init(p), c["steps"])
    _, ux, uy = orc.moments(p, f)
    run = g["runs"][f"{name}_{'RC' if coll == orc.RC else 'RNR'}"]
    nx, ny = c["nx"], c["ny"]
    for k, i in enumerate((nx // 2 - 1, nx // 2)):
        assert np.array_equal(ux[:, i], np.array([float(v) for v in run["ux_cols"][k]]))
    for k, j in enumerate((ny // 2 - 1, ny // 2)):
        assert np.array_equal(uy[j, :], np.array([float(v) for v in run["uy_rows"][k]]))
    x, y, _ = primary_vortex(ux, uy, c["a"])
    assert (x, y) == tuple(run["centre"])


@pytest.mark.slow
def test_oracle_re100_run_reproduces_the_stored_run(orc):
    _rerun("re100", orc.RC, orc)


@pytest.mark.slow
@pytest.mark.skipif(os.environ.get("LBM_SLOW_PINS") != "1",
                    reason="250 000 steps of the 150 x 300 oracle (about 10 minutes); "
                           "set LBM_SLOW_PINS=1")
@pytest.mark.parametrize("coll", [0, 1])
def test_oracle_re1000_run_reproduces_the_stored_run(coll, orc):
    _rerun("re1000", coll, orc)
