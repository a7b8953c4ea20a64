"""Time-dependent validations on the GPU (Sec. 5.2, 5.3): the per-step
force schedule against the oracle, and the paper's own configurations of
the impulsively started Couette flow and the Womersley flow against their
closed forms."""
import numpy as np
import pytest

import oracle as O
from paper_2103_02119_amd import lbm as L

from test_oracle_transient import couette_series, womersley

pytestmark = pytest.mark.gpu


def announce(*args):
    print("case:", *args, flush=True)


@pytest.mark.parametrize("coll", [L.LBM_RC, L.LBM_RNR])
def test_forced_steps_match_the_oracle(coll):
    announce("step_forced parity", coll)
    nx, ny, a, tau, cs2 = 70, 40, 0.25, 1.0, 0.04
    rates = O.paper_rates(tau)
    p = O.make_params(nx, ny, a, cs2, rates, collision=coll, bc=(0, 0, 1, 1))
    lat = L.Lattice(nx, ny, a, rates, bc_types=(0, 0, 1, 1), cs2=cs2, collision=coll)
    w = 2 * np.pi / 400
    fx = 1e-5 * np.cos(w * (np.arange(900) + 0.5))
    fy = 3e-6 * np.sin(w * np.arange(900))
    lat.step_forced(fx, fy)
    f = O.init(p)
    for i in range(900):
        p.force[0], p.force[1] = fx[i], fy[i]
        f = O.run(p, f, 1)
    ref = lat.get_populations()
    assert np.abs(ref - f).max() / np.abs(f).max() < 1e-12
    lat.close()


@pytest.mark.parametrize("coll", [L.LBM_RC, L.LBM_RNR])
def test_transient_couette_at_the_paper_configuration(coll):
    """50 x 500 nodes, a = 0.1, U = 0.02, tau = 0.8, fluid at rest."""
    announce("couette 50x500", coll)
    nx, ny, a, U, tau = 50, 500, 0.1, 0.02, 0.8
    cs2 = 0.64 * a * a
    nu = cs2 * (tau - 0.5)
    H = ny * a
    lat = L.Lattice(nx, ny, a, O.paper_rates(tau), bc_types=(0, 0, 1, 2),
                    u_wall=((0, 0), (0, 0), (0, 0), (U, 0)), cs2=cs2, collision=coll)
    y = (np.arange(ny) + 0.5) * a
    t = 0
    for T in (0.01, 0.05, 0.2, 0.5):
        n = int(round(T * H * H / nu)) - t
        lat.step(n)
        t += n
        _, ux, _ = lat.moments()
        err = np.abs(ux.mean(1) - couette_series(y, t, U, H, nu)).max() / U
        print("T", T, "error / U", err, flush=True)
        assert err < 5e-3
    lat.close()


def test_womersley_at_the_paper_configuration():
    """400 nodes across H = 50 (a = 0.125), tau = 1, period 40 000 steps,
    F_m = 1e-5 (Wo = (H/2) sqrt(w / nu) = 4.4), RC."""
    announce("womersley 400")
    nx, ny, a, tau = 8, 400, 0.125, 1.0
    cs2 = 0.64 * a * a
    nu = cs2 * (tau - 0.5)
    H = ny * a
    period, Fm = 40_000, 1e-5
    w = 2 * np.pi / period
    lat = L.Lattice(nx, ny, a, O.paper_rates(tau), bc_types=(0, 0, 1, 1), cs2=cs2)
    y = (np.arange(ny) + 0.5) * a
    spin = 13 * period
    lat.step_forced(Fm * np.cos(w * (np.arange(spin) + 0.5)))
    worst, umax = 0.0, 0.0
    for k in range(8):
        t0 = spin + k * (period // 8)
        lat.step_forced(Fm * np.cos(w * (np.arange(t0, t0 + period // 8) + 0.5)))
        t = t0 + period // 8
        lat.set_force(Fm * np.cos(w * t))
        _, ux, _ = lat.moments()
        ref = womersley(y, t, Fm, w, nu, H)
        umax = max(umax, np.abs(ref).max())
        worst = max(worst, np.abs(ux.mean(1) - ref).max())
    print("womersley worst / peak", worst / umax, flush=True)
    assert worst / umax < 5e-3
    lat.close()


def test_shallow_cavity_rectangular_lattice_matches_the_square_one():
    """Sec. 5.5: H/L = 0.25, Re = 100; 100 x 125 nodes at a = 0.2 give the
    centreline profiles of 400 x 100 nodes at a = 1 with 3.2x fewer nodes."""
    from paper_2103_02119_amd import shallow_cavity as SC

    announce("shallow cavity")
    res = SC.compare(scale=1, tol=1e-8)
    print(res, flush=True)
    assert res["square"]["steps"] and res["rectangular"]["steps"]
    assert res["node_ratio"] == pytest.approx(3.2)
    assert res["max_abs_diff_u_vertical"] < 1e-2 and res["max_abs_diff_v_horizontal"] < 5e-2


@pytest.mark.parametrize("prec", [L.LBM_FP64, L.LBM_FP32_DEV])
def test_taylor_green_decay_at_full_size(prec):
    """1024 x 2048 nodes at a = 0.5 (a square physical box of side 1024),
    u0 = 0.02, nu = 0.1 (tau = 1.125 at cs2 = 0.16): after step 1000 the
    velocity amplitude decays at 2 nu k^2 within 1% (RC)."""
    from paper_2103_02119_amd import inputs as I

    announce("taylor-green 1024x2048", prec)
    nx, ny, a, cs2, nu, u0 = 1024, 2048, 0.5, 0.16, 0.1, 0.02
    tau = nu / cs2 + 0.5
    lat = L.Lattice(nx, ny, a, O.paper_rates(tau), cs2=cs2, precision=prec)
    lat.set_fields(*I.taylor_green(nx, ny, a, u0, cs2))
    lat.step(1000)
    _, ux0, _ = lat.moments()
    lat.step(19_000)
    _, ux1, _ = lat.moments()
    k = 2 * np.pi / nx
    rate = np.log(np.abs(ux0).max() / np.abs(ux1).max()) / 19_000
    print("decay rate / 2 nu k^2 =", rate / (2 * nu * k * k), flush=True)
    assert abs(rate / (2 * nu * k * k) - 1) < 1e-2
    lat.close()


def test_stream_copy_kernel_copies_every_byte():
    """The library's copy kernel (the bandwidth reference of the benchmark)
    moves every byte, including a tail shorter than one round of the grid."""
    import torch

    for nbytes in (16, 4096 * 16 + 48, (64 << 20) + 16 * 1234):
        print(f"case: stream copy {nbytes} bytes", flush=True)
        a = torch.randint(0, 256, (nbytes,), dtype=torch.uint8, device="cuda")
        b = torch.zeros_like(a)
        L.lbm_stream_copy(b.data_ptr(), a.data_ptr(), nbytes, 0,
                          torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        assert torch.equal(a, b)
