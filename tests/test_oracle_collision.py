"""Pins of the oracle's collision step (no GPU).

- Mass is conserved and momentum gains exactly F per collision, for any
  relaxation rates (the half-force variable change of Eq. 5-6 and the
  central source moments (0, Fx, Fy, 0, ...) of Sec. 4).
- A uniform equilibrium is a fixed point of collide + stream.
- With all rates 1 and the corrections switched off, the RC (Sec. 4) and RNR
  (Sec. 3) collisions coincide: both reduce to m~ = m^{eq,r} + Phi/2, which
  ties Eq. 12 and Eq. 13 to F^{-1} applied to Eq. 49 and to (0, Fx, Fy, 0...).
- The local strain-rate formulas (Eq. 37-38 with Eq. 40) invert the
  Chapman-Enskog non-equilibrium moments (Eq. 19-20 with Eq. 23-26
  substituted), and the isotropy corrections vanish at a = 1, cs2 = 1/3 as
  stated after Eq. 33.
"""
import numpy as np
import pytest

CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], float)
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], float)


def _random_state(orc, p, g, noise=0.05):
    rho = g.uniform(0.9, 1.1)
    ux, uy = g.uniform(-0.08, 0.08, 2)
    return orc.feq(p, rho, ux, uy) * (1 + noise * g.uniform(-1, 1, 9))


CASES = [(1.0, 1 / 3), (0.5, 0.16), (0.25, 0.04), (2.0, 0.3)]


@pytest.mark.parametrize("coll", [0, 1])
@pytest.mark.parametrize("a,cs2", CASES)
def test_mass_and_momentum_per_collision(orc, coll, a, cs2):
    g = np.random.default_rng(10)
    for _ in range(20):
        w = g.uniform(0.2, 1.9, 9)
        F = g.uniform(-1e-3, 1e-3, 2)
        p = orc.make_params(4, 4, a, cs2, w, force=F, collision=coll)
        f = _random_state(orc, p, g)
        gx, gy = g.uniform(-1e-3, 1e-3, 2)
        ft = orc.collide_node(p, f, gx, gy)
        assert ft.sum() == pytest.approx(f.sum(), abs=1e-14)
        assert (ft * CX).sum() == pytest.approx((f * CX).sum() + F[0], abs=1e-14)
        assert (ft * a * CY).sum() == pytest.approx((f * a * CY).sum() + F[1], abs=1e-14)


@pytest.mark.parametrize("coll", [0, 1])
@pytest.mark.parametrize("a,cs2", CASES)
def test_uniform_equilibrium_is_a_fixed_point(orc, coll, a, cs2):
    nx, ny = 6, 5
    w = [1.0, 1.0, 1.0, 0.9, 1.3, 1.3, 1.0, 1.0, 1.0]
    p = orc.make_params(nx, ny, a, cs2, w, collision=coll)
    rho = np.full((ny, nx), 1.02)
    ux = np.full((ny, nx), 0.04)
    uy = np.full((ny, nx), -0.03)
    f0 = orc.init(p, rho, ux, uy)
    f1 = orc.run(p, f0, 3)
    assert np.abs(f1 - f0).max() < 1e-15


@pytest.mark.parametrize("a,cs2", CASES)
def test_rc_equals_rnr_with_unit_rates_and_no_corrections(orc, a, cs2):
    g = np.random.default_rng(11)
    for _ in range(20):
        F = g.uniform(-1e-3, 1e-3, 2)
        prc = orc.make_params(4, 4, a, cs2, [1.0] * 9, force=F, collision=0, corrections=False)
        prn = orc.make_params(4, 4, a, cs2, [1.0] * 9, force=F, collision=1, corrections=False)
        f = _random_state(orc, prc, g)
        a1 = orc.collide_node(prc, f, 0.0, 0.0)
        a2 = orc.collide_node(prn, f, 0.0, 0.0)
        assert np.abs(a1 - a2).max() < 1e-15


@pytest.mark.parametrize("a,cs2", CASES)
def test_rc_and_rnr_differ_in_general(orc, a, cs2):
    """With non-unit rates the two frames give different post-collision
    populations (a plausible mix-up of the variants would pass the test
    above but fail here)."""
    g = np.random.default_rng(12)
    w = [1.0, 1.0, 1.0, 1.2, 1.5, 1.5, 0.8, 0.8, 0.8]
    prc = orc.make_params(4, 4, a, cs2, w, collision=0)
    prn = orc.make_params(4, 4, a, cs2, w, collision=1)
    f = _random_state(orc, prc, g)
    assert np.abs(orc.collide_node(prc, f, 0, 0) - orc.collide_node(prn, f, 0, 0)).max() > 1e-6


def _ce_nonequilibrium(a, s, w3, w4, rho, ux, uy, X, Y, gx, gy):
    """Eq. 19 and Eq. 20 with the corrections of Eq. 23-26 substituted:
    the non-equilibrium raw moments m3 - m3^{eq,r}, m4 - m4^{eq,r} produced by
    strain rates X = d ux/dx, Y = d uy/dy and a density gradient."""
    a2 = a * a
    k3, k4 = 1 / w3 - 0.5, 1 / w4 - 0.5
    m3s = k3 * ((-3 * s + 1) * rho * X + (-3 * s + a2) * rho * Y + (-3 * s + 1) * ux * gx
                + (-3 * s + a2) * uy * gy)
    m4s = k4 * ((-3 * s + 1) * rho * X + (3 * s - a2) * rho * Y + (-3 * s + 1) * ux * gx
                + (3 * s - a2) * uy * gy)
    m3G = -3 * rho * k3 * (ux * ux * X + uy * uy * Y)
    m4G = -3 * rho * k4 * (ux * ux * X - uy * uy * Y)
    n3 = -(1 / w3) * ((-s + 1) * rho * X + (-s + a2) * rho * Y + (-3 * s + 1) * ux * gx
                      + (-3 * s + a2) * uy * gy - 3 * rho * (ux * ux * X + uy * uy * Y)) + m3s + m3G
    n4 = -(1 / w4) * ((1 - s) * rho * X + (s - a2) * rho * Y + (-3 * s + 1) * ux * gx
                      - (-3 * s + a2) * uy * gy - 3 * rho * (ux * ux * X - uy * uy * Y)) + m4s + m4G
    return n3, n4, m3s + m3G, m4s + m4G


@pytest.mark.parametrize("a,cs2", CASES + [(0.1, 0.005)])
def test_strain_rate_inverts_chapman_enskog_moments(orc, a, cs2):
    g = np.random.default_rng(13)
    for _ in range(20):
        w = [1.0, 1.0, 1.0, g.uniform(0.5, 1.8), g.uniform(0.5, 1.9), 1.0, 1.0, 1.0, 1.0]
        w[5] = w[4]
        p = orc.make_params(4, 4, a, cs2, w)
        rho = g.uniform(0.95, 1.05)
        ux, uy = g.uniform(-0.08, 0.08, 2)
        X, Y = g.uniform(-1e-3, 1e-3, 2)
        gx, gy = g.uniform(-1e-4, 1e-4, 2)
        n3, n4, d3, d4 = _ce_nonequilibrium(a, cs2, w[3], w[4], rho, ux, uy, X, Y, gx, gy)
        # populations with these non-equilibrium parts in m3, m4 only
        dm = np.zeros(9)
        dm[3], dm[4] = n3, n4
        f = orc.feq(p, rho, ux, uy) + orc.Tinv(a) @ dm
        Xo, Yo = orc.strain_rate(p, f, gx, gy)
        assert Xo == pytest.approx(X, rel=1e-8, abs=1e-15)
        assert Yo == pytest.approx(Y, rel=1e-8, abs=1e-15)
        d3o, d4o = orc.corrections(p, f, gx, gy)
        assert d3o == pytest.approx(d3, rel=1e-8, abs=1e-16)
        assert d4o == pytest.approx(d4, rel=1e-8, abs=1e-16)


def test_isotropy_corrections_vanish_on_the_square_lattice(orc):
    """At a = 1, cs2 = 1/3 (and u = 0, so the Galilean term is zero too) the
    corrections vanish for any non-equilibrium state."""
    g = np.random.default_rng(14)
    p = orc.make_params(4, 4, 1.0, 1 / 3, [1, 1, 1, 1.1, 1.4, 1.4, 1, 1, 1])
    for _ in range(10):
        f0 = orc.feq(p, 1.0, 0.0, 0.0)
        dm = np.zeros(9)
        dm[3], dm[4] = g.uniform(-1e-3, 1e-3, 2)
        f = f0 + orc.Tinv(1.0) @ dm
        d3, d4 = orc.corrections(p, f, *g.uniform(-1e-4, 1e-4, 2))
        assert abs(d3) < 1e-18 and abs(d4) < 1e-18
    # but not on a rectangular lattice
    p2 = orc.make_params(4, 4, 0.5, 0.16, [1, 1, 1, 1.1, 1.4, 1.4, 1, 1, 1])
    f0 = orc.feq(p2, 1.0, 0.0, 0.0)
    dm = np.zeros(9)
    dm[3] = 1e-3
    d3, d4 = orc.corrections(p2, f0 + orc.Tinv(0.5) @ dm, 0.0, 0.0)
    assert abs(d3) > 1e-6


def test_corrections_off_switch(orc):
    g = np.random.default_rng(15)
    p = orc.make_params(4, 4, 0.5, 0.16, [1, 1, 1, 1.1, 1.4, 1.4, 1, 1, 1], corrections=False)
    f = _random_state(orc, p, g)
    assert orc.corrections(p, f, 1e-4, -1e-4) == (0.0, 0.0)
