"""Oracle pins for time-dependent flows (Sec. 5.2 and 5.3 validations):
impulsively started Couette flow against its Fourier series, and the
Womersley flow driven by F_m cos(w t) against the textbook solution of
du/dt = F(t) / rho + nu d2u/dy2 with no-slip plates (the paper's printed
formula is garbled; this is the standard one it paraphrases)."""
import numpy as np
import pytest

import oracle as O


def couette_series(y, t, U, H, nu, terms=400):
    n = np.arange(1, terms + 1)[:, None]
    return U * y / H + (2 * U / np.pi * ((-1.0) ** n / n) * np.sin(n * np.pi * y / H)
                        * np.exp(-nu * (n * np.pi / H) ** 2 * t)).sum(0)


@pytest.mark.parametrize("coll", [O.RC, O.RNR])
@pytest.mark.parametrize("a,ny", [(0.25, 40), (0.1, 100)])
def test_transient_couette_matches_the_series(coll, a, ny):
    nx, U, tau = 4, 0.02, 0.8
    cs2 = min(1 / 3, 0.64 * a * a)
    nu = cs2 * (tau - 0.5)
    H = ny * a
    p = O.make_params(nx, ny, a, cs2, O.paper_rates(tau), collision=coll, bc=(0, 0, 1, 2),
                      u_wall=((0, 0), (0, 0), (0, 0), (U, 0)))
    y = (np.arange(ny) + 0.5) * a
    f = O.init(p)
    t = 0
    for T in (0.02, 0.05, 0.1, 0.3, 1.0):
        n = int(round(T * H * H / nu)) - t
        f = O.run(p, f, n)
        t += n
        _, ux, uy = O.moments(p, f)
        err = np.abs(ux[:, 0] - couette_series(y, t, U, H, nu)).max() / U
        assert err < 0.01, (T, err)
        assert np.abs(uy).max() < 1e-5 * U  # weakly compressible transients only


def womersley(y, t, Fm, w, nu, H, rho=1.0):
    k = np.sqrt(1j * w / nu)
    u_hat = Fm / (1j * w * rho) * (1 - np.cosh(k * (y - H / 2)) / np.cosh(k * H / 2))
    return np.real(u_hat * np.exp(1j * w * t))


@pytest.mark.parametrize("coll", [O.RC, O.RNR])
def test_womersley_matches_the_closed_form(coll):
    nx, ny, a, tau = 4, 40, 0.25, 1.0
    cs2 = 0.04
    nu = cs2 * (tau - 0.5)
    H = ny * a
    Wo = 4.0
    w = (Wo / H) ** 2 * nu
    period = int(round(2 * np.pi / w))
    w = 2 * np.pi / period
    Fm = 1e-5
    p = O.make_params(nx, ny, a, cs2, O.paper_rates(tau), collision=coll, bc=(0, 0, 1, 1))
    y = (np.arange(ny) + 0.5) * a
    f = O.init(p)
    umax, worst = 0.0, 0.0
    for t in range(4 * period):
        # the step from t to t + 1 is driven by F(t + 1/2); the velocity at
        # t + 1 carries half of F(t + 1)
        p.force[0] = Fm * np.cos(w * (t + 0.5))
        f = O.run(p, f, 1)
        if t >= 3 * period and t % (period // 8) == 0:
            p.force[0] = Fm * np.cos(w * (t + 1))
            _, ux, _ = O.moments(p, f)
            ref = womersley(y, t + 1, Fm, w, nu, H)
            umax = max(umax, np.abs(ref).max())
            worst = max(worst, np.abs(ux[:, 0] - ref).max())
    assert worst / umax < 0.01, worst / umax
