"""Oracle pins for the local stress output (Eq. 37-39 with Eq. 30-33):
exact shear stress of steady Couette flow, the linear shear stress of the
Poiseuille channel, and the stresses of decaying shear waves and of the
Taylor-Green vortex against spectral derivatives of the velocity field."""
import numpy as np
import pytest

import oracle as O
from paper_2103_02119_amd import inputs as I


@pytest.mark.parametrize("coll", [O.RC, O.RNR])
@pytest.mark.parametrize("a", [1.0, 0.5, 0.25])
def test_couette_shear_stress(coll, a):
    nx, ny, U, tau = 4, 24, 0.01, 0.9
    cs2 = min(1 / 3, 0.64 * a * a)
    nu = cs2 * (tau - 0.5)
    H = ny * a
    p = O.make_params(nx, ny, a, cs2, O.paper_rates(tau), collision=coll, bc=(0, 0, 1, 2),
                      u_wall=((0, 0), (0, 0), (0, 0), (U, 0)))
    f = O.run(p, O.init(p), int(12 * H * H / nu))
    sxx, syy, sxy = O.stress(p, f)
    rho, _, _ = O.moments(p, f)
    assert np.abs(sxy / (rho * nu * U / H) - 1).max() < 1e-6
    # no normal stress in plane shear, up to the scheme's higher-order terms
    assert np.abs(sxx).max() < 2e-2 * nu * U / H and np.abs(syy).max() < 2e-2 * nu * U / H


@pytest.mark.parametrize("coll", [O.RC, O.RNR])
def test_poiseuille_shear_stress(coll):
    nx, ny, a, cs2, tau, Fx = 4, 32, 0.5, 0.16, 1.125, 1e-6
    nu = cs2 * (tau - 0.5)
    H = ny * a
    p = O.make_params(nx, ny, a, cs2, O.paper_rates(tau), force=(Fx, 0.0), collision=coll,
                      bc=(0, 0, 1, 1))
    f = O.run(p, O.init(p), int(8 * H * H / nu))
    _, _, sxy = O.stress(p, f)
    y = (np.arange(ny) + 0.5) * a
    ref = -Fx * (y - H / 2)
    assert np.abs(sxy[:, 0] - ref).max() / np.abs(ref).max() < 1e-2


def spectral_d(u, L, axis):
    k = np.fft.fftfreq(u.shape[axis], d=L / u.shape[axis]) * 2 * np.pi
    shape = [1, 1]
    shape[axis] = -1
    return np.real(np.fft.ifft(1j * k.reshape(shape) * np.fft.fft(u, axis=axis), axis=axis))


@pytest.mark.parametrize("a", [0.5, 0.25])
def test_shear_wave_and_taylor_green_stresses(a):
    nx, ny, tau = 64, int(64 / a), 0.8
    cs2 = min(1 / 3, 0.64 * a * a)
    nu = cs2 * (tau - 0.5)
    p = O.make_params(nx, ny, a, cs2, O.paper_rates(tau))
    f = O.run(p, O.init(p, *I.shear_wave(nx, ny, a, 0.01, "x")), 200)
    rho, ux, _ = O.moments(p, f)
    _, _, sxy = O.stress(p, f)
    ref = rho * nu * spectral_d(ux, ny * a, 0)
    assert np.abs(sxy - ref).max() / np.abs(ref).max() < 2e-2
    f = O.run(p, O.init(p, *I.taylor_green(nx, ny, a, 0.01, cs2)), 200)
    rho, ux, uy = O.moments(p, f)
    sxx, syy, sxy = O.stress(p, f)
    refs = (2 * rho * nu * spectral_d(ux, nx, 1), 2 * rho * nu * spectral_d(uy, ny * a, 0),
            rho * nu * (spectral_d(ux, ny * a, 0) + spectral_d(uy, nx, 1)))
    # the vortex's shear strain vanishes where kx = ky: errors against the stress scale
    scale = max(np.abs(r).max() for r in refs)
    for got, ref in zip((sxx, syy, sxy), refs):
        assert np.abs(got - ref).max() / scale < 1e-2


@pytest.mark.parametrize("coll", [O.RC, O.RNR])
@pytest.mark.parametrize("a", [1.0, 0.5, 0.25])
def test_sound_wave_normal_stresses_carry_the_bulk_viscosity(coll, a):
    """A travelling sound wave along x with zeta != nu (omega_3 != omega_4):
    tau_xx = rho (nu + zeta) d_x u_x and tau_yy = rho (zeta - nu) d_x u_x
    (Eq. 30-31 with div u = d_x u_x), against the spectral derivative of the
    velocity.  The error is mostly a uniform offset of second order in the
    amplitude and falls with the square of the resolution (1.4% at 64 nodes
    per wavelength, 0.7% at 128); a bulk term taken with nu instead of zeta
    would be off by 50%."""
    nx, ny = 128, 4
    cs2 = min(1 / 3, 0.64 * a * a)
    tau, tau_bulk = 0.8, 0.6
    rates = O.paper_rates(tau)
    rates[3] = 1 / tau_bulk
    nu, zeta = cs2 * (tau - 0.5), cs2 * (tau_bulk - 0.5)
    p = O.make_params(nx, ny, a, cs2, rates, collision=coll)
    A = 1e-3
    ux = np.tile(A * np.sin(2 * np.pi * np.arange(nx) / nx), (ny, 1))
    rho = 1 + ux / np.sqrt(cs2)
    f = O.run(p, O.init(p, rho, ux, np.zeros((ny, nx))), 3 * nx)
    r, u, _ = O.moments(p, f)
    sxx, syy, sxy = O.stress(p, f)
    X = spectral_d(u, nx, 1)
    scale = np.abs(r * (nu + zeta) * X).max()
    assert np.abs(sxx - r * (nu + zeta) * X).max() / scale < 1.5e-2
    assert np.abs(syy - r * (zeta - nu) * X).max() / scale < 1.5e-2
    assert np.abs(sxy).max() / scale < 1e-9
