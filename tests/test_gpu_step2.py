"""Two collide-and-stream steps per launch (the temporally blocked tile
kernel) against one step per launch, and against the FP64 oracle.

The two-step kernel runs every node through the same loaders, collision and
storage rounding as the one-step kernels, so its results must be identical
bit for bit in every storage mode; the oracle bar is the usual 1e-12 (FP64).
Shapes span interior tiles (every pulled node four or more nodes from a
face), tiles on the x faces, tiles on the y faces and degenerate lattices
smaller than one tile, with periodic faces, walls and moving walls."""
import numpy as np
import pytest
import torch  # noqa: F401  (imported at collection: the first import on a fresh box is slow)

import oracle as O
from paper_2103_02119_amd import inputs as I
from paper_2103_02119_amd import lbm as L
from test_gpu_parity import CASES, RATES_GEN, RATES_HU, TOL64, announce, make, random_state, rel

pytestmark = pytest.mark.gpu

PRECS = [L.LBM_FP64, L.LBM_FP32_DEV, L.LBM_FP64_DEV, L.LBM_FP32_DEV_F64]
REG, STAGED = L.LBM_FORM_REGISTER, L.LBM_FORM_STAGED
# (precision, two-step form): the register form in every precision, the
# staged form (FP32 storage and arithmetic only) beside it
PREC_FORMS = [(p, REG) for p in PRECS] + [(L.LBM_FP32_DEV, STAGED)]


def pair(name, nx, ny, coll, prec, rates=RATES_HU, corr=True, form=REG):
    """Two lattices with the same parameters: one step per launch, two (in
    the given form of the two-step kernel)."""
    p, one = make(name, nx, ny, coll, prec, rates=rates, corr=corr)
    _, two = make(name, nx, ny, coll, prec, rates=rates, corr=corr)
    one.set_steps_per_launch(1)
    two.set_steps_per_launch(2)
    two.set_two_step_form(form)
    assert two.two_step_form() == form
    return p, one, two


def same_after(p, one, two, n, seed=2103):
    f0 = random_state(p, seed=seed)
    one.set_populations(f0)
    two.set_populations(f0)
    one.step(n)
    two.step(n)
    a, b = one.get_populations(), two.get_populations()
    return a, b, f0


@pytest.mark.parametrize("prec,form", PREC_FORMS)
@pytest.mark.parametrize("coll", [L.LBM_RC, L.LBM_RNR])
@pytest.mark.parametrize("name", list(CASES))
def test_two_steps_per_launch_bit_identical(name, coll, prec, form):
    nx, ny = 150, 70  # interior, x-face and y-face tiles, ragged last column of tiles
    announce("step2", name, coll, prec, form, nx, ny)
    p, one, two = pair(name, nx, ny, coll, prec, form=form)
    assert two.steps_per_launch() == 2 and one.steps_per_launch() == 1
    a, b, _ = same_after(p, one, two, 7)  # one step from the set state, then three pairs
    assert np.array_equal(a, b), (name, coll, prec, float(np.abs(a - b).max()))
    one.close()
    two.close()


@pytest.mark.parametrize("prec,form", [(L.LBM_FP64, REG), (L.LBM_FP32_DEV, REG),
                                       (L.LBM_FP32_DEV, STAGED)])
@pytest.mark.parametrize("coll", [L.LBM_RC, L.LBM_RNR])
@pytest.mark.parametrize("name", ["periodic", "cavity", "xmoving"])
def test_two_steps_general_rates_and_no_corrections(name, coll, prec, form):
    nx, ny = 97, 45
    for rates, corr in ((RATES_GEN, True), (RATES_HU, False), (RATES_GEN, False)):
        announce("step2", name, coll, prec, form, rates, corr)
        p, one, two = pair(name, nx, ny, coll, prec, rates=rates, corr=corr, form=form)
        a, b, _ = same_after(p, one, two, 5, seed=7)
        assert np.array_equal(a, b), (name, rates, corr)
        one.close()
        two.close()


@pytest.mark.parametrize("prec,form", [(L.LBM_FP64, REG), (L.LBM_FP32_DEV, REG),
                                       (L.LBM_FP32_DEV, STAGED)])
@pytest.mark.parametrize("shape", [(3, 3), (4, 3), (3, 5), (7, 4), (64, 4), (65, 6), (128, 3),
                                   (130, 9), (200, 17), (72, 24), (300, 41), (70, 25), (129, 49)])
@pytest.mark.parametrize("name", ["periodic", "cavity", "xwalls", "channel"])
def test_two_steps_degenerate_shapes(name, shape, prec, form):
    nx, ny = shape
    announce("step2", name, shape, prec, form)
    p, one, two = pair(name, nx, ny, 0, prec, form=form)
    a, b, _ = same_after(p, one, two, 5, seed=11)
    assert np.array_equal(a, b), (name, shape, prec)
    one.close()
    two.close()


@pytest.mark.parametrize("coll", [L.LBM_RC, L.LBM_RNR])
@pytest.mark.parametrize("name", ["periodic", "cavity", "box_all_moving", "channel"])
def test_two_steps_against_the_oracle(name, coll):
    nx, ny = 150, 70
    announce("step2 oracle", name, coll)
    p, lat = make(name, nx, ny, coll, L.LBM_FP64)
    lat.set_steps_per_launch(2)
    f0 = random_state(p, seed=5)
    lat.set_populations(f0)
    lat.step(9)
    ref = O.run(p, f0, 9)
    assert rel(lat.get_populations(), ref) < TOL64
    r_o, ux_o, uy_o = O.moments(p, ref)
    r_g, ux_g, uy_g = lat.moments()
    assert rel(r_g, r_o) < TOL64 and rel(ux_g, ux_o) < TOL64 and rel(uy_g, uy_o) < TOL64
    lat.close()


def test_step_counts_and_the_state_one_step_back():
    """An explicit 2 leaves the previous state unavailable after a pair; the
    automatic choice always ends a call with a one-step launch; a mask
    turns the two-step kernel off."""
    p, lat = make("cavity", 96, 40, 0, L.LBM_FP64)
    lat.set_fields(*I.random_fields(3, 96, 40))
    assert lat.steps_per_launch() == 2  # automatic: two on any lattice without a mask
    lat.set_steps_per_launch(1)
    assert lat.steps_per_launch() == 1
    lat.set_steps_per_launch(2)
    assert lat.steps_per_launch() == 2
    lat.step(1)
    lat.residual()
    lat.step(2)
    with pytest.raises(L.LbmError) as e:
        lat.residual()
    assert e.value.code == L.LBM_E_STATE
    with pytest.raises(L.LbmError) as e:
        lat.check_async()
    assert e.value.code == L.LBM_E_STATE
    lat.step(1)
    assert np.isfinite(lat.residual())
    lat.step(3)  # a pair, then one step
    assert np.isfinite(lat.residual())
    assert lat.steps_done == 7
    mask = np.zeros((40, 96), np.uint8)
    mask[10:14, 30:40] = 1
    lat.set_mask(mask)
    assert lat.steps_per_launch() == 1
    lat.set_mask(None)
    lat.set_steps_per_launch(0)
    assert lat.steps_per_launch() == 2
    with pytest.raises(L.LbmError):
        lat.set_steps_per_launch(3)
    lat.close()


def test_two_step_form_choice_and_validation():
    """The automatic form: staged for FP32 storage from 512 of its 64 x 24
    tiles up, register below and in every other precision; the staged form
    cannot be asked of another precision."""
    for (nx, ny, prec), want in (((150, 70, L.LBM_FP32_DEV), REG),
                                 ((512, 1024, L.LBM_FP32_DEV), REG),      # 344 tiles
                                 ((1024, 768, L.LBM_FP32_DEV), STAGED),   # 512 tiles
                                 ((1024, 1024, L.LBM_FP64), REG),
                                 ((1024, 1024, L.LBM_FP32_DEV_F64), REG)):
        p, lat = make("periodic", nx, ny, 0, prec)
        assert lat.two_step_form() == want, (nx, ny, prec)
        if prec != L.LBM_FP32_DEV:
            with pytest.raises(L.LbmError) as e:
                lat.set_two_step_form(STAGED)
            assert e.value.code == L.LBM_E_INVAL
        with pytest.raises(L.LbmError) as e:
            lat.set_two_step_form(3)
        assert e.value.code == L.LBM_E_INVAL
        lat.set_two_step_form(REG)
        assert lat.two_step_form() == REG
        lat.close()


@pytest.mark.parametrize("prec,form,want", [(L.LBM_FP32_DEV, L.LBM_FORM_AUTO, STAGED),
                                            (L.LBM_FP32_DEV, REG, REG),
                                            (L.LBM_FP64, L.LBM_FORM_AUTO, REG)])
def test_full_size_shear_layer_two_steps_bit_identical(prec, form, want):
    """The 2048 x 8192, a = 0.25 shear layer (the automatic choice takes two
    steps per launch, in FP32 storage the staged form) against one step per
    launch."""
    nx, ny, a, cs2, nu = 2048, 8192, 0.25, 0.04, 6e-3
    tau = nu / cs2 + 0.5
    rates = [1, 1, 1, 1, 1 / tau, 1 / tau, 1, 1, 1]
    announce("step2 shear 2048x8192", prec, form)
    fields = I.shear_layer(nx, ny, a, u0=0.04)
    out = []
    for k in (0, 1):
        lat = L.Lattice(nx, ny, a, rates, cs2=cs2, precision=prec)
        lat.set_steps_per_launch(k)
        lat.set_two_step_form(form)
        assert lat.steps_per_launch() == (2 if k == 0 else 1)
        assert lat.two_step_form() == want
        lat.set_fields(*fields)
        lat.step(6)  # one step from the set state, two pairs, one step
        lat.residual()
        out.append(lat.moments())
        lat.close()
    for u, v in zip(*out):
        assert np.array_equal(u, v)


def test_zero_steps_change_nothing():
    """The empty run: lbm_step(ctx, 0) and lbm_batch_step(b, 0) enqueue
    nothing, so the populations, the step count and the residual of the last
    step stay as they were, right after creation and mid-run."""
    from paper_2103_02119_amd import warmstart as WS

    announce("zero steps")
    p, lat = make("cavity", 70, 25, L.LBM_RC, L.LBM_FP32_DEV)
    lat.set_populations(random_state(p, seed=7))
    f0 = lat.get_populations()
    lat.step(0)
    assert lat.steps_done == 0 and np.array_equal(lat.get_populations(), f0)
    lat.step(3)
    f3, R3 = lat.get_populations(), lat.residual()
    lat.step(0)
    assert lat.steps_done == 3 and np.array_equal(lat.get_populations(), f3)
    assert lat.residual() == R3
    lat.close()
    b = L.Batch(WS.cavity_cases([dict(Re=400.0, r=0.5), dict(Re=900.0, r=1.0)], 64, 32, 0.05),
                precision=L.LBM_FP32_DEV)
    g0 = [b.get_populations(c) for c in range(2)]
    b.step(0)
    assert all(b.steps_done(c) == 0 and np.array_equal(b.get_populations(c), g0[c])
               for c in range(2))
    b.step(5)
    g5, R5 = [b.get_populations(c) for c in range(2)], b.residuals()
    b.step(0)
    assert all(b.steps_done(c) == 5 and np.array_equal(b.get_populations(c), g5[c])
               for c in range(2))
    assert np.array_equal(b.residuals(), R5)
    b.close()
