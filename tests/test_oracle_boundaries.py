"""Pins of the oracle's streaming and boundary conditions (no GPU).

- Periodic streaming is a pure shift by (cx, cy) nodes (perfect shift, Sec. 3).
- Half-way bounce-back at a stationary wall returns the node's own outgoing
  population (Sec. 5.1).
- At a lid moving with (U, 0) the incoming populations follow Eq. 57-59:
  f4 = f~2, f7 = f~5 - rho_w cs2 U / (2 a^2), f8 = f~6 + rho_w cs2 U / (2 a^2).
"""
import numpy as np
import pytest

CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
OPP = np.array([0, 3, 4, 1, 2, 7, 8, 5, 6])


def _ft(shape, seed):
    return np.random.default_rng(seed).uniform(0.01, 0.5, (9,) + shape)


def test_periodic_stream_is_a_shift(orc):
    nx, ny = 7, 5
    p = orc.make_params(nx, ny, 0.5, 0.16, [1] * 9)
    ft = _ft((ny, nx), 1)
    f = orc.stream(p, ft)
    for k in range(9):
        assert np.array_equal(f[k], np.roll(ft[k], shift=(CY[k], CX[k]), axis=(0, 1)))


def test_stationary_walls_bounce_back(orc):
    nx, ny = 6, 5
    p = orc.make_params(nx, ny, 0.5, 0.16, [1] * 9, bc=(0, 0, 1, 1))
    ft = _ft((ny, nx), 2)
    f = orc.stream(p, ft)
    for k in range(9):
        for j in range(ny):
            for i in range(nx):
                sj = j - CY[k]
                if sj < 0 or sj >= ny:
                    assert f[k, j, i] == ft[OPP[k], j, i]
                else:
                    assert f[k, j, i] == ft[k, sj, (i - CX[k]) % nx]
    # closed box: streaming conserves mass exactly
    p2 = orc.make_params(nx, ny, 0.5, 0.16, [1] * 9, bc=(1, 1, 1, 1))
    f2 = orc.stream(p2, ft)
    assert f2.sum() == pytest.approx(ft.sum(), rel=1e-15)


@pytest.mark.parametrize("a,cs2", [(1.0, 1 / 3), (0.5, 0.16), (0.25, 0.04), (0.1, 0.005)])
def test_moving_lid_matches_eq57_59(orc, a, cs2):
    nx, ny, U, rho0 = 6, 4, 0.05, 1.0
    p = orc.make_params(nx, ny, a, cs2, [1] * 9, rho0=rho0, bc=(0, 0, 1, 2),
                        u_wall=((0, 0), (0, 0), (0, 0), (U, 0)))
    ft = _ft((ny, nx), 3)
    f = orc.stream(p, ft)
    j = ny - 1
    c = rho0 * cs2 * U / (2 * a * a)
    assert np.abs(f[4, j] - ft[2, j]).max() < 1e-16
    assert np.abs(f[7, j] - (ft[5, j] - c)).max() < 1e-16
    assert np.abs(f[8, j] - (ft[6, j] + c)).max() < 1e-16


def test_cavity_corner_links_take_the_lid(orc):
    """A link whose source lies above the top row is a lid link, also where
    it crosses a side wall (the corner convention)."""
    nx, ny, a, cs2, U = 5, 4, 0.5, 0.16, 0.1
    p = orc.make_params(nx, ny, a, cs2, [1] * 9, bc=(1, 1, 1, 2),
                        u_wall=((0, 0), (0, 0), (0, 0), (U, 0)))
    ft = _ft((ny, nx), 4)
    f = orc.stream(p, ft)
    c = cs2 * U / (2 * a * a)
    j = ny - 1
    # top-left corner, k = 8 (from (-1, ny)): lid term
    assert f[8, j, 0] == pytest.approx(ft[6, j, 0] + c, abs=1e-16)
    # top-right corner, k = 7 (from (nx, ny)): lid term
    assert f[7, j, nx - 1] == pytest.approx(ft[5, j, nx - 1] - c, abs=1e-16)
    # side-wall links below the lid are plain bounce-back
    assert f[1, 1, 0] == ft[3, 1, 0]
    assert f[5, j, 0] == ft[7, j, 0]
    # bottom corners: stationary
    assert f[5, 0, 0] == ft[7, 0, 0]
    assert f[6, 0, nx - 1] == ft[8, 0, nx - 1]


def test_density_gradient_wall_convention(orc):
    nx, ny, a = 5, 4, 0.5
    p = orc.make_params(nx, ny, a, 0.16, [1] * 9, bc=(1, 1, 0, 0))
    rho = np.random.default_rng(5).uniform(0.9, 1.1, (ny, nx))
    gx, gy = orc.density_gradient(p, rho)
    assert gx[2, 0] == pytest.approx((rho[2, 1] - rho[2, 0]) / 2)
    assert gx[2, nx - 1] == pytest.approx((rho[2, nx - 1] - rho[2, nx - 2]) / 2)
    assert gx[2, 2] == pytest.approx((rho[2, 3] - rho[2, 1]) / 2)
    assert gy[0, 2] == pytest.approx((rho[1, 2] - rho[ny - 1, 2]) / (2 * a))
