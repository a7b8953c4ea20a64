"""Host logic of the studies, without a GPU: the bisections of the
stability module against known thresholds (the lattice runs replaced by a
rule), and the centreline extraction of the shallow-cavity comparison."""
import numpy as np
import pytest

from paper_2103_02119_amd import lbm as L
from paper_2103_02119_amd import shallow_cavity as SC
from paper_2103_02119_amd import stability as S


def lid_threshold(tau, a, coll):
    return 0.05 + 0.3 * (tau - 0.5) * a + (0.02 if coll == L.LBM_RC else 0.0)


@pytest.fixture
def fake_lid(monkeypatch):
    monkeypatch.setattr(S, "_lid_case", lambda nx, ny, a, tau, U, cs2: (a, tau, U))
    monkeypatch.setattr(S, "_survives", lambda cases, coll, steps, every, prec: np.array(
        [U < lid_threshold(tau, a, coll) for (a, tau, U) in cases]))


def test_lid_speed_bisection_brackets_the_threshold(fake_lid):
    rounds, u_max = 8, 0.6
    res = S.max_lid_velocity((0.52, 0.6, 1.0), rounds=rounds, u_max=u_max)
    assert len(res) == 3 * 3 * 2
    for r in res:
        t = lid_threshold(r["tau"], r["a"], L.LBM_RC if r["collision"] == "RC" else L.LBM_RNR)
        assert r["stable_U"] < t <= r["unstable_U"]
        assert r["unstable_U"] - r["stable_U"] <= u_max / 2 ** (rounds - 1) + 1e-15


def test_lid_speed_bisection_reports_a_stable_maximum(monkeypatch):
    monkeypatch.setattr(S, "_lid_case", lambda nx, ny, a, tau, U, cs2: U)
    monkeypatch.setattr(S, "_survives", lambda cases, coll, steps, every, prec:
                        np.ones(len(cases), bool))
    res = S.max_lid_velocity((0.6,), grids=((21, 21, 1.0),), rounds=4, u_max=0.5)
    assert all(r["stable_U"] == 0.5 and r["unstable_U"] is None for r in res)


def test_reynolds_bisection_brackets_the_threshold(monkeypatch):
    crit = {L.LBM_RC: 12000.0, L.LBM_RNR: 7000.0}
    U, cs2 = 0.2, 0.1
    monkeypatch.setattr(S, "_lid_case", lambda nx, ny, a, tau, u, c2: (nx, tau))
    monkeypatch.setattr(S, "_survives", lambda cases, coll, steps, every, prec: np.array(
        [U * nx / ((tau - 0.5) * cs2) < crit[coll] * nx / 100 for (nx, tau) in cases]))
    res = S.max_reynolds(grids=((100, 200), (200, 400)), rounds=14, re_lo=500.0, re_hi=60000.0,
                         U=U, cs2=cs2)
    for r in res:
        c = (crit[L.LBM_RC] if r["collision"] == "RC" else crit[L.LBM_RNR]) * r["nx"] / 100
        assert r["stable_Re"] < c <= r["unstable_Re"] * (1 + 1e-12)
        assert r["unstable_Re"] / r["stable_Re"] < 1.001
        assert r["tau_at_stable"] == pytest.approx(U * r["nx"] / r["stable_Re"] / cs2 + 0.5)


def test_shear_margin_bisection_brackets_the_threshold(monkeypatch):
    crit = {L.LBM_RC: 7.5e-3, L.LBM_RNR: 5.2e-3}
    monkeypatch.setattr(S, "_shear_survives",
                        lambda nx, ny, a, nu, cs2, coll, prec, steps, every, fields: nu > crit[coll])
    res = S.shear_layer_margin(nx=16, ny=64, rounds=10, nu_lo=1e-3, nu_hi=2e-2)
    for name, coll in (("RC", L.LBM_RC), ("RNR", L.LBM_RNR)):
        r = res[name]
        assert r["max_unstable_nu"] <= crit[coll] < r["min_stable_nu"]
        assert r["min_stable_nu"] / r["max_unstable_nu"] < 20 ** (1 / 2 ** 10) + 1e-12


def test_centrelines_pick_the_middle_columns_and_rows():
    nx, ny, U = 6, 5, 0.1
    ux = np.arange(ny * nx, dtype=float).reshape(ny, nx)
    uy = -np.arange(ny * nx, dtype=float).reshape(ny, nx)
    (y, u), (x, v) = SC.centrelines(nx, ny, ux, uy, U)
    assert np.allclose(y, (np.arange(ny) + 0.5) / ny) and np.allclose(x, (np.arange(nx) + 0.5) / nx)
    assert np.allclose(u, 0.5 * (ux[:, 2] + ux[:, 3]) / U)  # even nx: mean of the two middle columns
    assert np.allclose(v, uy[2, :] / U)                       # odd ny: the middle row
