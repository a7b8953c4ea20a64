"""Oracle pins for obstacle masks (half-way bounce-back at solid nodes,
Sec. 5.2 with the wall at rest).

The pins tie the mask to the wall boundaries that the other oracle tests pin
to the paper (Poiseuille, Couette): a lattice whose outer rows / columns are
solid must evolve bit for bit like the same fluid region bounded by walls,
because a half-way wall and a solid layer put the reflection at the same
place and both replace the missing density neighbour by the node's own."""
import numpy as np

import oracle as O
from paper_2103_02119_amd import inputs as I

RATES = [1.0, 1.0, 1.0, 1.1, 1.3, 1.3, 1.0, 1.0, 1.0]
GENERAL = [1.0, 0.7, 1.2, 1.1, 1.3, 1.3, 0.9, 1.2, 1.4]


def state(p, seed):
    rho, ux, uy = I.random_fields(seed, p.nx, p.ny)
    return O.init(p, rho, ux, uy) * I.relative_noise(seed, p.nx, p.ny, 1e-3)


def embed_rows(f, pad):
    """(9, ny, nx) -> (9, ny + 2 pad, nx) with the new rows at rest."""
    out = np.zeros((9, f.shape[1] + 2 * pad, f.shape[2]))
    out[:, pad:-pad, :] = f
    return out


def test_solid_rows_are_walls():
    for coll in (O.RC, O.RNR):
        for rates in (RATES, GENERAL):
            nx, ny, a, cs2 = 24, 10, 0.5, 0.16
            pw = O.make_params(nx, ny, a, cs2, rates, force=(1e-5, 0.0), collision=coll,
                               bc=(0, 0, 1, 1))
            mask = np.zeros((ny + 2, nx), np.uint8)
            mask[0, :] = mask[-1, :] = 1
            pm = O.make_params(nx, ny + 2, a, cs2, rates, force=(1e-5, 0.0), collision=coll,
                               solid=mask)
            f0 = state(pw, 3)
            fw = O.run(pw, f0, 7)
            fm = O.run(pm, embed_rows(f0, 1), 7)
            assert np.array_equal(fm[:, 1:-1, :], fw)


def test_solid_columns_are_walls_and_solid_frame_is_a_box():
    nx, ny, a, cs2 = 12, 20, 2.0, 0.3
    pw = O.make_params(nx, ny, a, cs2, GENERAL, force=(0.0, 2e-5), bc=(1, 1, 0, 0))
    mask = np.zeros((ny, nx + 2), np.uint8)
    mask[:, 0] = mask[:, -1] = 1
    pm = O.make_params(nx + 2, ny, a, cs2, GENERAL, force=(0.0, 2e-5), solid=mask)
    f0 = state(pw, 4)
    fpad = np.zeros((9, ny, nx + 2))
    fpad[:, :, 1:-1] = f0
    assert np.array_equal(O.run(pm, fpad, 6)[:, :, 1:-1], O.run(pw, f0, 6))
    # all four sides: a solid frame on a periodic lattice = a closed box of walls
    pb = O.make_params(nx, ny, a, cs2, RATES, bc=(1, 1, 1, 1))
    frame = np.ones((ny + 2, nx + 2), np.uint8)
    frame[1:-1, 1:-1] = 0
    pf = O.make_params(nx + 2, ny + 2, a, cs2, RATES, solid=frame)
    f0 = state(pb, 5)
    fpad = np.zeros((9, ny + 2, nx + 2))
    fpad[:, 1:-1, 1:-1] = f0
    assert np.array_equal(O.run(pf, fpad, 6)[:, 1:-1, 1:-1], O.run(pb, f0, 6))


def random_mask(nx, ny, seed, nbox=4):
    m = I.rect_obstacles(nx, ny, seed, nbox)  # boxes may straddle the periodic seams
    m[3, 5] = 1  # a single solid node
    return m


def test_mass_is_conserved_around_obstacles():
    nx, ny = 30, 22
    m = random_mask(nx, ny, 8)
    for coll in (O.RC, O.RNR):
        p = O.make_params(nx, ny, 0.5, 0.16, GENERAL, collision=coll, solid=m)
        f = state(p, 6)
        fluid = m == 0
        m0 = (f.sum(0) * fluid).sum()
        f = O.run(p, f, 40)
        assert abs((f.sum(0) * fluid).sum() - m0) / m0 < 1e-13
        # solid nodes hold the rest state
        rest = O.feq(p, 1.0, 0.0, 0.0)
        assert np.array_equal(f[:, ~fluid], np.repeat(rest[:, None], (~fluid).sum(), axis=1))


def test_rest_stays_at_rest_and_mirror_symmetry_holds():
    nx, ny, a, cs2 = 40, 21, 0.5, 0.16
    m = np.zeros((ny, nx), np.uint8)
    m[8:13, 10:14] = 1  # symmetric about the channel's mid row j = 10
    p = O.make_params(nx, ny, a, cs2, RATES, bc=(0, 0, 1, 1), solid=m)
    f = O.init(p)
    assert np.abs(O.run(p, f, 5) - f).max() < 1e-15  # rest is a fixed point (to rounding)
    pf = O.make_params(nx, ny, a, cs2, RATES, force=(1e-4, 0.0), bc=(0, 0, 1, 1), solid=m)
    _, ux, uy = O.moments(pf, O.run(pf, O.init(pf), 300))
    assert np.abs(ux - ux[::-1, :]).max() < 1e-15
    assert np.abs(uy + uy[::-1, :]).max() < 1e-15
    assert np.abs(uy).max() > 1e-6  # the obstacle deflects the flow


def test_step_node_agrees_with_the_field_step():
    nx, ny = 26, 18
    m = random_mask(nx, ny, 9)
    p = O.make_params(nx, ny, 0.5, 0.16, GENERAL, force=(1e-5, -1e-5), bc=(1, 1, 1, 2),
                      u_wall=((0, 0), (0, 0), (0, 0), (0.04, 0)), solid=m)
    f = state(p, 7)
    g = O.run(p, f, 1)
    for i, j in [(0, 0), (5, 3), (4, 3), (6, 3), (nx - 1, ny - 1), (12, 9), (3, ny - 1)]:
        assert np.array_equal(O.step_node(p, f, i, j), g[:, j, i])
