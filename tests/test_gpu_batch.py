"""GPU parity of the batch ABI (include/lbm_batch.h).

Every case of a batch must reproduce the oracle to the single-lattice bars,
and the single-lattice library bit for bit (the batch only changes how the
work is launched): through the first in-place step, graph replays and single
launches, deactivation, a state reset mid-run, the autotuner's trial
launches, and at the full 512-case sweep size."""
import numpy as np
import pytest

import oracle as O
from paper_2103_02119_amd import inputs as I
from paper_2103_02119_amd import lbm as L
from paper_2103_02119_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL64 = 1e-12

# (nx, ny, a, cs2, bc types, wall velocities, force, rates): ragged sizes,
# several segments, one-segment and 3-row cases, every boundary kind
SPECS = [
    (150, 70, 0.5, 0.16, (0, 0, 0, 0), ((0, 0),) * 4, (1e-5, -2e-5), [1, 1, 1, 1.1, 1.3, 1.3, 1, 1, 1]),
    (64, 40, 0.5, 0.16, (1, 1, 1, 2), ((0, 0), (0, 0), (0, 0), (0.05, 0)), (0, 0), [1, 1, 1, 1, 1.5, 1.5, 1, 1, 1]),
    (97, 33, 0.25, 0.04, (0, 0, 1, 1), ((0, 0),) * 4, (2e-6, 0), [1, 1, 1, 1, 1.8, 1.8, 1, 1, 1]),
    (33, 130, 2.0, 0.3, (1, 1, 0, 0), ((0, 0),) * 4, (0, 1e-5), [1, 1, 1, 0.9, 1.2, 1.2, 1, 1, 1]),
    (200, 3, 1.0, 1 / 3, (2, 2, 0, 0), ((0, 0.03), (0, -0.02), (0, 0), (0, 0)), (0, 0), [1, 1, 1, 1, 1.1, 1.1, 1, 1, 1]),
    (70, 66, 0.5, 0.16, (2, 2, 2, 2), ((0, 0.01), (0, -0.01), (-0.02, 0), (0.03, 0)), (0, 0), [1, 1, 1, 1.2, 1.6, 1.6, 1, 1, 1]),
]
GENERAL = [1.0, 0.7, 1.2, 1.1, 1.3, 1.3, 0.9, 1.2, 1.4]


def announce(*args):
    print("case:", *args, flush=True)


def cases_of(specs, rates_override=None):
    out = []
    for nx, ny, a, cs2, bc, uw, F, rates in specs:
        out.append(L.make_case(nx, ny, a, rates_override or rates, bc_types=bc, u_wall=uw,
                               cs2=cs2, force=F))
    return out


def oracle_params(spec, coll, rates_override=None):
    nx, ny, a, cs2, bc, uw, F, rates = spec
    return O.make_params(nx, ny, a, cs2, rates_override or rates, force=F, collision=coll,
                         bc=bc, u_wall=uw)


def single(spec, coll, prec, rates_override=None, rows=0):
    nx, ny, a, cs2, bc, uw, F, rates = spec
    return L.Lattice(nx, ny, a, rates_override or rates, bc_types=bc, u_wall=uw, cs2=cs2,
                     force=F, collision=coll, precision=prec, rows_per_wave=rows)


def random_state(p, seed):
    rho, ux, uy = I.random_fields(seed, p.nx, p.ny)
    return O.init(p, rho, ux, uy) * I.relative_noise(seed, p.nx, p.ny, 1e-3)


def rel(x, ref):
    return float(np.abs(x - ref).max() / max(np.abs(ref).max(), 1e-300))


@pytest.mark.parametrize("prec", [L.LBM_FP64, L.LBM_FP64_DEV])
@pytest.mark.parametrize("coll", [L.LBM_RC, L.LBM_RNR])
@pytest.mark.parametrize("general", [False, True])
def test_batch_matches_oracle_and_single_lattice(coll, prec, general):
    """11 steps with graph_steps 4: the first in-place step, two graph
    replays and two single launches."""
    announce("batch parity", coll, prec, general)
    ro = GENERAL if general else None
    b = L.Batch(cases_of(SPECS, ro), collision=coll, precision=prec, graph_steps=4)
    f0s = []
    for c, spec in enumerate(SPECS):
        f0 = random_state(oracle_params(spec, coll, ro), seed=100 + c)
        b.set_populations(c, f0)
        f0s.append(f0)
    b.step(11)
    for c, spec in enumerate(SPECS):
        p = oracle_params(spec, coll, ro)
        got = b.get_populations(c)
        assert rel(got, O.run(p, f0s[c], 11)) < TOL64, c
        lat = single(spec, coll, prec, ro)
        lat.set_populations(f0s[c])
        lat.step(11)
        assert np.array_equal(got, lat.get_populations()), c
        assert b.steps_done(c) == 11
        lat.close()
    b.close()


@pytest.mark.parametrize("prec", [L.LBM_FP32_DEV, L.LBM_FP32_DEV_F64])
def test_fp32_batch_is_bitwise_the_single_lattice(prec):
    announce("batch fp32", prec)
    b = L.Batch(cases_of(SPECS), precision=prec, graph_steps=6)
    for c, spec in enumerate(SPECS):
        rho, ux, uy = I.random_fields(200 + c, spec[0], spec[1])
        b.set_fields(c, rho, ux, uy)
    b.step(20)
    R = b.residuals()
    for c, spec in enumerate(SPECS):
        rho, ux, uy = I.random_fields(200 + c, spec[0], spec[1])
        lat = single(spec, L.LBM_RC, prec)
        lat.set_fields(rho, ux, uy)
        lat.step(20)
        assert np.array_equal(b.get_populations(c), lat.get_populations()), c
        assert R[c] == pytest.approx(lat.residual(), rel=1e-12)
        lat.close()
    b.close()


def test_residuals_activity_and_reset():
    """Per-case residuals against the single-lattice ones; an inactive case
    keeps its state and count; a case reset mid-run (in-place form while the
    others pull) restarts correctly."""
    announce("batch activity")
    b = L.Batch(cases_of(SPECS), graph_steps=4)
    assert np.all(b.residuals() == -1.0)
    b.step(6)
    active = [1, 0, 1, 1, 1, 1]
    b.set_active(active)
    b.step(9)
    b.set_fields(3)  # case 3 back to rest, in-place form
    b.step(5)
    R = b.residuals()
    expect_steps = [20, 6, 20, 20, 20, 20]
    for c, spec in enumerate(SPECS):
        assert b.steps_done(c) == expect_steps[c]
        lat = single(spec, L.LBM_RC, L.LBM_FP64)
        if c == 3:
            lat.step(15)
            lat.set_fields()
            lat.step(5)
        else:
            lat.step(expect_steps[c])
        assert np.array_equal(b.get_populations(c), lat.get_populations()), c
        assert R[c] == pytest.approx(lat.residual(), rel=1e-12, abs=1e-300), c
        lat.close()
    b.close()


def test_first_residual_after_one_step_and_blow_up_flag():
    announce("batch residual flags")
    b = L.Batch(cases_of(SPECS[:3]))
    b.step(1)
    R = b.residuals()
    for c, spec in enumerate(SPECS[:3]):
        lat = single(spec, L.LBM_RC, L.LBM_FP64)
        lat.step(1)
        assert R[c] == pytest.approx(lat.residual(), rel=1e-12, abs=1e-300)
        lat.close()
    # a non-finite population in case 1 only (a blown-up case, made on the host)
    f = b.get_populations(1)
    f[2, 5, 7] = np.nan
    b.set_populations(1, f)
    steps = b.run_to_steady(1e-30, 2, 4)
    assert steps[1] == -1
    assert steps[0] == -2 and steps[2] == -2
    R = b.residuals()
    assert np.isnan(R[1]) and np.isfinite(R[0]) and np.isfinite(R[2])
    b.close()


def test_autotune_does_not_advance_the_state():
    announce("batch autotune")
    b = L.Batch(cases_of(SPECS), graph_steps=4)
    b.step(3)
    before = [b.get_populations(c) for c in range(len(SPECS))]
    rows, wgs = b.autotune(2)
    assert rows in (2, 4, 8, 16) and wgs >= 1
    assert b.launch_shape()[:2] == (rows, wgs)
    for c in range(len(SPECS)):
        assert np.array_equal(b.get_populations(c), before[c])
        assert b.steps_done(c) == 3
    assert np.all(b.residuals() == -1.0)
    b.step(9)
    for c, spec in enumerate(SPECS):
        lat = single(spec, L.LBM_RC, L.LBM_FP64)
        lat.step(12)
        assert np.array_equal(b.get_populations(c), lat.get_populations()), c
        lat.close()
    b.close()


def test_run_to_steady_channels_reach_the_poiseuille_profile():
    """Three body-force channels of different heights and aspect ratios, run
    to a residual of 1e-10; each must sit on the oracle's steady profile."""
    announce("batch steady channels")
    specs = [(16, 12, 0.5, 0.16), (8, 24, 0.25, 0.04), (12, 10, 1.0, 1 / 3)]
    cases = [W.channel_case(nx, ny, a, 1.0, 1e-3, cs2=cs2) for nx, ny, a, cs2 in specs]
    b = L.Batch(cases)
    steps = b.run_to_steady(1e-10, 500, 400000)
    assert np.all(steps > 0), steps
    for c, (nx, ny, a, cs2) in enumerate(specs):
        k = cases[c]
        p = O.make_params(nx, ny, a, cs2, list(k.rates), force=(k.force[0], 0.0), bc=(0, 0, 1, 1))
        _, ux_o, _ = O.moments(p, O.run(p, O.init(p), int(steps[c])))
        _, ux_g, _ = b.moments(c)
        assert rel(ux_g, ux_o) < 1e-9, c
    b.close()


def test_full_sweep_512_cases_sampled():
    """The 512-case sweep (cavities and channels, nx 64..512, r in
    {0.25, 0.5, 1}, Re 100..5000) in FP32, autotuned: sampled cases against
    the single-lattice library bit for bit, and single nodes against the
    oracle."""
    params = I.batch_sweep()
    cases = W.sweep_cases(params)
    announce("batch sweep", len(cases))
    b = L.Batch(cases, precision=L.LBM_FP32_DEV)
    b.autotune(2)
    b.step(40)
    g = np.random.default_rng(5)
    for c in [0, 1, 511] + [int(v) for v in g.choice(512, 5, replace=False)]:
        k, pr = cases[c], params[c]
        lat = L.Lattice(k.nx, k.ny, k.r, list(k.rates), bc_types=list(k.bc.type),
                        u_wall=[tuple(k.bc.u_wall[f]) for f in range(4)], cs2=k.cs2,
                        force=(k.force[0], k.force[1]), precision=L.LBM_FP32_DEV)
        lat.step(40)
        got = b.get_populations(c)
        assert np.array_equal(got, lat.get_populations()), (c, pr)
        lat.close()
    # one more step of case 7 checked node by node against the oracle
    c = 7
    k = cases[c]
    p = O.make_params(k.nx, k.ny, k.r, k.cs2, list(k.rates), force=(k.force[0], k.force[1]),
                      bc=list(k.bc.type), u_wall=[tuple(k.bc.u_wall[f]) for f in range(4)])
    f_before = b.get_populations(c)
    b.set_active([1 if i == c else 0 for i in range(512)])
    b.step(1)
    got = b.get_populations(c)
    scale = np.abs(f_before).max()
    for i, j in [(0, 0), (k.nx - 1, k.ny - 1), (k.nx // 2, k.ny // 2), (1, k.ny - 1), (k.nx - 1, 1)]:
        assert np.abs(got[:, j, i] - O.step_node(p, f_before, i, j)).max() / scale < 1e-6
    b.close()


def test_batch_smooth_step_and_set_rates_match_single_lattices():
    announce("batch smooth step")
    b = L.Batch(cases_of(SPECS, GENERAL), graph_steps=4)
    b.step(5)
    b.set_rates(2, [1.0, 0.8, 1.1, 1.2, 1.4, 1.4, 0.9, 1.1, 1.3])
    b.smooth_step()
    b.step(6)
    for c, spec in enumerate(SPECS):
        lat = single(spec, L.LBM_RC, L.LBM_FP64, GENERAL)
        lat.step(5)
        if c == 2:
            lat.set_rates([1.0, 0.8, 1.1, 1.2, 1.4, 1.4, 0.9, 1.1, 1.3])
        lat.smooth_step()
        lat.step(6)
        assert np.array_equal(b.get_populations(c), lat.get_populations()), c
        assert b.steps_done(c) == 12
        lat.close()
    b.close()
    # a batch built for omega_6..8 = 1 keeps them
    b = L.Batch(cases_of(SPECS[:2]))
    with pytest.raises(L.LbmError) as e:
        b.set_rates(0, GENERAL)
    assert e.value.code == L.LBM_E_INVAL
    b.close()


@pytest.mark.parametrize("prec", [L.LBM_FP64, L.LBM_FP32_DEV])
def test_tile_kernel_batch_matches_single_lattices_and_falls_back_under_a_mask(prec):
    """The batched tile kernel (64 x 8 block tiles) gives every case bit for
    bit the populations of a single lattice, through the first in-place step
    and graph replays; a mask on one case returns the batch to the marching
    kernel, still bit for bit."""
    announce("batch tile kernel", prec)
    b = L.Batch(cases_of(SPECS), precision=prec, graph_steps=4, tile_kernel=True)
    assert b.uses_tile_kernel()
    b.step(11)
    for c, spec in enumerate(SPECS):
        lat = single(spec, L.LBM_RC, prec)
        lat.step(11)
        assert np.array_equal(b.get_populations(c), lat.get_populations()), c
        lat.close()
    nx, ny = b.shapes[0]
    mask = np.zeros((ny, nx), np.uint8)
    mask[ny // 3:ny // 3 + 3, nx // 2:nx // 2 + 4] = 1
    b.set_mask(0, mask)
    assert not b.uses_tile_kernel()
    b.step(5)
    lat = single(SPECS[0], L.LBM_RC, prec)
    lat.step(11)
    lat.set_mask(mask)
    lat.step(5)
    assert np.array_equal(b.get_populations(0), lat.get_populations())
    lat.close()
    b.close()


def test_tile_kernel_returns_when_the_masks_are_removed():
    announce("batch tile kernel after masks")
    b = L.Batch(cases_of(SPECS[:2]), graph_steps=4, tile_kernel=True)
    nx, ny = b.shapes[1]
    mask = np.zeros((ny, nx), np.uint8)
    mask[5:8, 10:14] = 1
    b.set_mask(1, mask)
    assert not b.uses_tile_kernel()
    b.step(6)
    b.set_mask(1, None)
    assert b.uses_tile_kernel()
    b.step(6)
    lat = single(SPECS[1], L.LBM_RC, L.LBM_FP64)
    lat.set_mask(mask)
    lat.step(6)
    lat.set_mask(None)
    lat.step(6)
    assert np.array_equal(b.get_populations(1), lat.get_populations())
    lat.close()
    b.close()


@pytest.mark.parametrize("prec,form", [(L.LBM_FP64, L.LBM_FORM_AUTO),
                                       (L.LBM_FP32_DEV, L.LBM_FORM_REGISTER),
                                       (L.LBM_FP32_DEV, L.LBM_FORM_STAGED)])
@pytest.mark.parametrize("coll", [L.LBM_RC, L.LBM_RNR])
@pytest.mark.parametrize("general", [False, True])
def test_two_steps_per_launch_batch_is_bitwise_the_one_step_batch(prec, form, coll, general):
    """Pairs of steps per launch (graph replays of pairs, single pair
    launches and the closing single steps), through a deactivated case and a
    case reset mid-run, against the same batch at one step per launch:
    populations, step counts and residuals bit for bit.  A mask turns the
    pairs off."""
    announce("batch two-step", prec, form, coll, general)
    rates = GENERAL if general else None
    bs = [L.Batch(cases_of(SPECS, rates), collision=coll, precision=prec, graph_steps=4,
                  steps_per_launch=k, two_step_form=form) for k in (1, 0)]
    assert bs[0].steps_per_launch() == 1 and bs[1].steps_per_launch() == 2
    want = form if form != L.LBM_FORM_AUTO else L.LBM_FORM_REGISTER  # FP64: register
    assert bs[1].two_step_form() == want
    for b in bs:
        for c, spec in enumerate(SPECS):
            b.set_fields(c, *I.random_fields(300 + c, spec[0], spec[1]))
        b.step(14)  # the in-place step, three graph replays of two pairs, one step
        b.set_active([1, 1, 0, 1, 1, 1])
        b.step(6)   # one replay, two single steps
        b.set_fields(4)
        b.step(9)   # the in-place step, one replay, one pair, two single steps
    for c in range(len(SPECS)):
        assert bs[0].steps_done(c) == bs[1].steps_done(c)
        assert np.array_equal(bs[0].get_populations(c), bs[1].get_populations(c)), c
    assert np.array_equal(bs[0].residuals(), bs[1].residuals())
    nx, ny = bs[1].shapes[2]
    mask = np.zeros((ny, nx), np.uint8)
    mask[ny // 2:ny // 2 + 2, 5:9] = 1
    bs[1].set_mask(2, mask)
    assert bs[1].steps_per_launch() == 1
    bs[1].set_mask(2, None)
    assert bs[1].steps_per_launch() == 2
    for b in bs:
        b.close()


def test_two_step_batch_autotune_and_run_to_steady():
    """The autotuner's two-step trials leave the state as it was; a run to
    steady state with pairs of steps stops at the same step, with the same
    residuals, as at one step per launch."""
    announce("batch two-step autotune and steady")
    bs = [L.Batch(cases_of(SPECS[:3]), graph_steps=8, steps_per_launch=k) for k in (1, 0)]
    for b in bs:
        b.step(5)
    before = [bs[1].get_populations(c) for c in range(3)]
    rows, wgs = bs[1].autotune(2)
    assert rows == 8 and wgs >= 1 and bs[1].launch_shape()[:2] == (8, wgs)
    for c in range(3):
        assert np.array_equal(bs[1].get_populations(c), before[c])
    steps = [b.run_to_steady(1e-6, 50, 3000) for b in bs]
    assert np.array_equal(steps[0], steps[1])
    for c in range(3):
        assert np.array_equal(bs[0].get_populations(c), bs[1].get_populations(c)), c
    assert np.array_equal(bs[0].residuals(), bs[1].residuals())
    for b in bs:
        b.close()


def test_two_step_batch_form_choice_and_autotune_in_fp32():
    """FP32 storage: the staged form by default, the register form on
    request, the staged form refused for FP64; the autotuner's choice of form
    and grid keeps the results bit for bit those of one step per launch."""
    announce("batch two-step form choice")
    b = L.Batch(cases_of(SPECS[:3]), precision=L.LBM_FP32_DEV)
    assert b.two_step_form() == L.LBM_FORM_STAGED
    b.close()
    with pytest.raises(L.LbmError):
        L.Batch(cases_of(SPECS[:3]), precision=L.LBM_FP64, two_step_form=L.LBM_FORM_STAGED)
    bs = [L.Batch(cases_of(SPECS), precision=L.LBM_FP32_DEV, graph_steps=8, steps_per_launch=k)
          for k in (1, 0)]
    for b in bs:
        b.step(3)
    rows, wgs = bs[1].autotune(2)
    form = bs[1].two_step_form()
    assert (rows, form) in ((8, L.LBM_FORM_REGISTER), (24, L.LBM_FORM_STAGED))
    assert bs[1].launch_shape()[:2] == (rows, wgs)
    for b in bs:
        b.step(40)
    for c in range(len(SPECS)):
        assert np.array_equal(bs[0].get_populations(c), bs[1].get_populations(c)), c
    assert np.array_equal(bs[0].residuals(), bs[1].residuals())
    for b in bs:
        b.close()
