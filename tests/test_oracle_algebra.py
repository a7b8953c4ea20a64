"""Pins of the oracle's moment algebra against what the paper and the
mathematics fix (no GPU).

- T is built from the basis definition (Eq. 3) and checked against the matrix
  printed in Eq. 4 (one known erratum).
- T^{-1} (App. A, typed with one sign read differently) must invert T.
- F(u) (App. B) must reproduce the central moments of Eq. 43 computed by
  brute force, and F(-u) must invert it (the property stated with Eq. 55).
- Equilibria must reproduce Eq. 12 / Eq. 49, the Maxwellian product moments,
  the textbook D2Q9 weights at a = 1, cs2 = 1/3, and be positive exactly when
  cs2 < min(1, a^2).
"""
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
ASPECTS = [0.1, 0.2, 0.25, 0.3, 0.5, 0.8, 1.0, 2.0, 4.0]


def _load_printed(name, a):
    ns = {"a": a, "h1": 1 + a * a, "h2": 1 - a * a,
          "r1": -0.5 * (1 + 1 / (a * a)), "r2": -0.5 * (1 - 1 / (a * a))}
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append([float(eval(tok, {"__builtins__": {}}, ns)) for tok in line.split()])
    M = np.array(rows)
    assert M.shape == (9, 9)
    return M


@pytest.mark.parametrize("a", ASPECTS)
def test_T_matches_printed_eq4_except_erratum(orc, a):
    T = orc.T(a)
    P = _load_printed("eq4_T_printed.txt", a)
    diff = np.argwhere(np.abs(T - P) > 1e-14)
    if a == 1.0:
        assert diff.size == 0
    else:
        # only the entry e_x e_y^2 of e_5 differs: printed a, true a^2
        assert [tuple(d) for d in diff] == [(7, 5)]
        assert T[7, 5] == pytest.approx(a * a)


@pytest.mark.parametrize("a", ASPECTS)
def test_T_times_Tinv_is_identity(orc, a):
    T, Ti = orc.T(a), orc.Tinv(a)
    assert np.abs(T @ Ti - np.eye(9)).max() < 1e-12
    assert np.abs(Ti @ T - np.eye(9)).max() < 1e-12


@pytest.mark.parametrize("a", [0.25, 0.5, 2.0])
def test_printed_Tinv_differs_only_in_the_erratum(orc, a):
    P = _load_printed("appA_Tinv_printed.txt", a)
    Ti = orc.Tinv(a)
    diff = [tuple(d) for d in np.argwhere(np.abs(Ti - P) > 1e-14)]
    assert diff == [(0, 8)]
    assert Ti[0, 8] == pytest.approx(1 / (a * a))
    # the printed sign does not invert T, the read sign does
    assert np.abs(orc.T(a) @ P - np.eye(9)).max() > 1e-3


def test_F_inverse_is_F_of_minus_u(orc):
    g = np.random.default_rng(1)
    for _ in range(20):
        ux, uy = g.uniform(-0.3, 0.3, 2)
        assert np.abs(orc.F(ux, uy) @ orc.F(-ux, -uy) - np.eye(9)).max() < 1e-14


def _central_by_definition(f, a, ux, uy):
    """Eq. 43 summed directly over the velocity set, in the basis of Eq. 3."""
    ex = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], float)
    ey = a * np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], float)
    X, Y = ex - ux, ey - uy
    return np.array([
        f.sum(), (f * X).sum(), (f * Y).sum(),
        (f * (X ** 2 + Y ** 2)).sum(), (f * (X ** 2 - Y ** 2)).sum(), (f * X * Y).sum(),
        (f * X ** 2 * Y).sum(), (f * X * Y ** 2).sum(), (f * X ** 2 * Y ** 2).sum()])


@pytest.mark.parametrize("a", [0.25, 0.5, 1.0, 2.0])
def test_F_T_gives_central_moments_by_definition(orc, a):
    g = np.random.default_rng(2)
    for _ in range(10):
        f = g.uniform(0.01, 0.3, 9)
        ux, uy = g.uniform(-0.2, 0.2, 2)
        mc = orc.F(ux, uy) @ (orc.T(a) @ f)
        assert np.abs(mc - _central_by_definition(f, a, ux, uy)).max() < 1e-14


def _params(orc, a, cs2, **kw):
    return orc.make_params(4, 4, a, cs2, [1.0] * 9, **kw)


@pytest.mark.parametrize("a,cs2", [(1.0, 1 / 3), (0.5, 0.16), (0.25, 0.04), (2.0, 0.3)])
def test_equilibrium_raw_moments_are_eq12(orc, a, cs2):
    p = _params(orc, a, cs2)
    g = np.random.default_rng(3)
    for _ in range(10):
        rho = g.uniform(0.9, 1.1)
        ux, uy = g.uniform(-0.1, 0.1, 2)
        m = orc.T(a) @ orc.feq(p, rho, ux, uy)
        s = cs2
        # Eq. 12 as printed, except the m_8 coefficient of rho s (ux^2+uy^2)
        eq12 = np.array([rho, rho * ux, rho * uy, 2 * rho * s + rho * (ux * ux + uy * uy),
                         rho * (ux * ux - uy * uy), rho * ux * uy,
                         s * rho * uy + rho * ux * ux * uy, s * rho * ux + rho * ux * uy * uy,
                         rho * s * s + 1 * rho * s * (ux * ux + uy * uy) + rho * ux * ux * uy * uy])
        assert np.abs(m - eq12).max() < 1e-15
        # the Maxwellian's raw moment <xi_x^2 xi_y^2> = rho (s + ux^2)(s + uy^2)
        assert m[8] == pytest.approx(rho * (s + ux * ux) * (s + uy * uy), rel=1e-13)
        # the printed coefficient 3 would not match whenever u != 0
        printed_m8 = rho * s * s + 3 * rho * s * (ux * ux + uy * uy) + rho * ux * ux * uy * uy
        assert abs(printed_m8 - m[8]) > 1e-6 * rho * s * (ux * ux + uy * uy)


@pytest.mark.parametrize("a,cs2", [(1.0, 1 / 3), (0.5, 0.16), (0.25, 0.04)])
def test_equilibrium_central_moments_are_eq49(orc, a, cs2):
    p = _params(orc, a, cs2)
    rho, ux, uy = 1.03, 0.07, -0.04
    f = orc.feq(p, rho, ux, uy)
    mc = _central_by_definition(f, a, ux, uy)
    expect = np.array([rho, 0, 0, 2 * rho * cs2, 0, 0, 0, 0, rho * cs2 * cs2])
    assert np.abs(mc - expect).max() < 1e-15


def test_textbook_d2q9_weights_at_unit_aspect(orc):
    p = _params(orc, 1.0, 1 / 3)
    w = orc.feq(p, 1.0, 0.0, 0.0)
    expect = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    assert np.abs(w - expect).max() < 1e-15


@pytest.mark.parametrize("a", [0.1, 0.3, 0.5, 1.0, 2.0])
def test_rest_weights_positive_iff_cs2_below_min_1_a2(orc, a):
    lim = min(1.0, a * a)
    for cs2 in np.linspace(0.02, 1.5, 60):
        w = orc.feq(_params(orc, a, cs2), 1.0, 0.0, 0.0)
        if cs2 < lim * (1 - 1e-9):
            assert (w > 0).all(), (a, cs2)
        elif cs2 > lim * (1 + 1e-9):
            assert (w < 0).any(), (a, cs2)


def test_equilibrium_macroscopic_fields(orc):
    """sum feq = rho and sum feq e = rho u (no force)."""
    p = _params(orc, 0.5, 0.16)
    f = orc.feq(p, 0.97, 0.05, -0.03)
    r, ux, uy = orc.macro(p, f)
    assert (r, ux, uy) == pytest.approx((0.97, 0.05, -0.03), rel=1e-14)
