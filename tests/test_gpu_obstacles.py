"""GPU parity with obstacle masks: the HIP library against the oracle, with
solid nodes straddling 64-column segment boundaries, periodic seams, the
domain walls and the moving lid, single solid nodes, and tiles that the fast
interior path must hand to the generic one."""
import numpy as np
import pytest

import oracle as O
from paper_2103_02119_amd import inputs as I
from paper_2103_02119_amd import lbm as L

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
RATES = [1.0, 1.0, 1.0, 1.1, 1.3, 1.3, 1.0, 1.0, 1.0]
GENERAL = [1.0, 0.7, 1.2, 1.1, 1.3, 1.3, 0.9, 1.2, 1.4]
CASES = {
    "periodic": (0.5, 0.16, (0, 0, 0, 0), ((0, 0),) * 4, (1e-5, -2e-5)),
    "channel": (0.25, 0.04, (0, 0, 1, 1), ((0, 0),) * 4, (2e-6, 0.0)),
    "cavity": (0.5, 0.16, (1, 1, 1, 2), ((0, 0), (0, 0), (0, 0), (0.05, 0.0)), (0.0, 0.0)),
    "xmoving": (1.0, 1 / 3, (2, 2, 0, 0), ((0, 0.03), (0, -0.02), (0, 0), (0, 0)), (0.0, 0.0)),
}


def announce(*args):
    print("case:", *args, flush=True)


def rel(x, ref):
    return float(np.abs(x - ref).max() / max(np.abs(ref).max(), 1e-300))


def mask_for(nx, ny, seed):
    m = I.rect_obstacles(nx, ny, seed, nbox=6, wmax=8, hmax=6)
    m[ny // 2, 63] = 1        # the last column of a segment
    m[ny // 2 + 2, 64] = 1    # the first column of the next one
    m[1, nx // 2] = 1         # next to the bottom face
    m[ny - 1, nx // 3] = 1    # on the top row (the lid's row in a cavity)
    m[ny // 3, 0] = 1         # on the x-min column
    return m


def make(name, nx, ny, mask, coll=0, prec=0, rates=RATES, rows=0):
    a, cs2, bc, uw, F = CASES[name]
    p = O.make_params(nx, ny, a, cs2, rates, force=F, collision=coll, bc=bc, u_wall=uw,
                      solid=mask)
    lat = L.Lattice(nx, ny, a, rates, bc_types=bc, u_wall=uw, cs2=cs2, force=F,
                    collision=coll, precision=prec, rows_per_wave=rows)
    lat.set_mask(mask)
    return p, lat


def random_state(p, seed):
    rho, ux, uy = I.random_fields(seed, p.nx, p.ny)
    return O.init(p, rho, ux, uy) * I.relative_noise(seed, p.nx, p.ny, 1e-3)


@pytest.mark.parametrize("prec", [L.LBM_FP64, L.LBM_FP64_DEV])
@pytest.mark.parametrize("coll", [L.LBM_RC, L.LBM_RNR])
@pytest.mark.parametrize("name", list(CASES))
def test_obstacles_match_oracle(name, coll, prec):
    nx, ny = 150, 70
    announce("obstacles", name, coll, prec)
    m = mask_for(nx, ny, 31)
    p, lat = make(name, nx, ny, m, coll, prec)
    f0 = random_state(p, 40)
    lat.set_populations(f0)
    ref = O.init(p)  # solid nodes of the reference start at rest, as the library's do
    ref = np.where(m[None] != 0, ref, f0)
    for n in (1, 1, 3):
        lat.step(n)
        ref = O.run(p, ref, n)
        assert rel(lat.get_populations(), ref) < TOL64, n
    r_o, ux_o, uy_o = O.moments(p, ref)
    r_g, ux_g, uy_g = lat.moments()
    assert rel(r_g, r_o) < TOL64 and rel(ux_g, ux_o) < TOL64 and rel(uy_g, uy_o) < TOL64
    lat.close()


def test_general_rates_and_launch_shape_invariance():
    nx, ny = 150, 70
    m = mask_for(nx, ny, 32)
    outs = []
    for rows in (0, 1, 3, 16, 64):
        for prec in (L.LBM_FP64, L.LBM_FP32_DEV):
            announce("obstacle shapes", rows, prec)
            p, lat = make("cavity", nx, ny, m, prec=prec, rates=GENERAL, rows=rows)
            f0 = random_state(p, 41)
            lat.set_populations(f0)
            lat.step(4)
            got = lat.get_populations()
            if prec == L.LBM_FP64:
                ref = np.where(m[None] != 0, O.init(p), f0)
                assert rel(got, O.run(p, ref, 4)) < TOL64
            outs.append((prec, got))
            lat.close()
    for prec in (L.LBM_FP64, L.LBM_FP32_DEV):
        same = [g for q, g in outs if q == prec]
        for g in same[1:]:
            assert np.array_equal(g, same[0])


def test_sums_and_residual_cover_fluid_nodes_only():
    nx, ny = 150, 70
    m = mask_for(nx, ny, 33)
    fluid = m == 0
    for prec in (L.LBM_FP64, L.LBM_FP32_DEV):
        p, lat = make("channel", nx, ny, m, prec=prec)
        f0 = random_state(p, 42)
        lat.set_populations(f0)
        lat.step(5)
        ref0 = np.where(m[None] != 0, O.init(p), f0)
        f4 = O.run(p, ref0, 4)
        f5 = O.run(p, f4, 1)
        _, ux4, uy4 = O.moments(p, f4)
        r5, ux5, uy5 = O.moments(p, f5)
        mass = (r5 * fluid).sum()
        R_ref = np.sqrt((((ux5 - ux4) ** 2 + (uy5 - uy4) ** 2) * fluid).sum() /
                        ((ux5 ** 2 + uy5 ** 2) * fluid).sum())
        tol = 1e-13 if prec == L.LBM_FP64 else 1e-7
        assert abs(lat.sums()[0] - mass) / mass < tol
        assert lat.residual() == pytest.approx(R_ref, rel=1e-10 if prec == L.LBM_FP64 else 1e-3)
        lat.close()


def test_fp32_velocity_with_obstacles():
    nx, ny = 150, 70
    m = mask_for(nx, ny, 34)
    for coll in (L.LBM_RC, L.LBM_RNR):
        p, lat = make("cavity", nx, ny, m, coll, L.LBM_FP32_DEV)
        f0 = np.where(m[None] != 0, O.init(p), random_state(p, 43))
        lat.set_populations(f0)
        lat.step(50)
        _, ux_o, uy_o = O.moments(p, O.run(p, f0, 50))
        _, ux_g, uy_g = lat.moments()
        u = np.hypot(ux_o, uy_o).max()
        assert np.abs(ux_g - ux_o).max() / u < 1e-5 and np.abs(uy_g - uy_o).max() / u < 1e-5
        lat.close()


def test_mask_removal_and_batch_masks_match_single_lattices():
    nx, ny = 130, 40
    m1, m2 = mask_for(nx, ny, 35), mask_for(nx, ny, 36)
    a, cs2, bc, uw, F = CASES["cavity"]
    cases = [L.make_case(nx, ny, a, RATES, bc_types=bc, u_wall=uw, cs2=cs2) for _ in range(3)]
    b = L.Batch(cases, graph_steps=4)
    b.set_mask(0, m1)
    b.set_mask(2, m2)
    b.step(9)
    for c, m in enumerate((m1, None, m2)):
        lat = L.Lattice(nx, ny, a, RATES, bc_types=bc, u_wall=uw, cs2=cs2)
        lat.set_mask(m)
        lat.step(9)
        assert np.array_equal(b.get_populations(c), lat.get_populations()), c
        lat.close()
    # removing a mask brings back the plain lattice
    p, lat = make("cavity", nx, ny, m1)
    lat.set_mask(None)
    f0 = random_state(p, 44)
    lat.set_populations(f0)
    lat.step(3)
    p0 = O.make_params(nx, ny, a, cs2, RATES, bc=bc, u_wall=uw)
    assert rel(lat.get_populations(), O.run(p0, f0, 3)) < TOL64
    lat.close()
    b.close()


def test_full_size_cavity_with_obstacles_sampled():
    nx, ny, a, cs2, U = 512, 1024, 0.5, 0.16, 0.05
    rates = O.paper_rates(U * nx / 1000.0 / cs2 + 0.5)
    bc, uw = (1, 1, 1, 2), ((0, 0), (0, 0), (0, 0), (U, 0))
    m = I.rect_obstacles(nx, ny, 50, nbox=40, wmax=60, hmax=120, wrap=False)
    p = O.make_params(nx, ny, a, cs2, rates, bc=bc, u_wall=uw, solid=m)
    announce("full cavity obstacles")
    lat = L.Lattice(nx, ny, a, rates, bc_types=bc, u_wall=uw, cs2=cs2, precision=L.LBM_FP64)
    lat.set_mask(m)
    lat.set_fields(*I.random_fields(51, nx, ny, u_amp=0.05))
    lat.step(20)
    f_before = lat.get_populations()
    lat.step(1)
    got = lat.get_populations()
    scale = np.abs(f_before).max()
    g = np.random.default_rng(1)
    edge = np.argwhere((m == 0) & (np.roll(m, 1, 0) | np.roll(m, -1, 0) | np.roll(m, 1, 1)
                                   | np.roll(m, -1, 1)))
    pts = [tuple(edge[int(k)])[::-1] for k in g.choice(len(edge), 24, replace=False)]
    pts += [(int(g.integers(nx)), int(g.integers(ny))) for _ in range(16)]
    for i, j in pts:
        assert np.abs(got[:, j, i] - O.step_node(p, f_before, i, j)).max() / scale < TOL64
    lat.close()
