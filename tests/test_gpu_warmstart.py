"""The learned warm start end to end on small cavities (64 x 32 nodes):
steady fields from the batched solver, training on the GPU kernels, and the
plain lattice Boltzmann scheme deciding convergence.

At this size the cavities converge from rest within a few ten thousand
steps once the smoothing step has removed the impulsive start's staggered
mode, and 150 training fields are too few for the network to beat that, so
the first test asks for what holds at any size: the trained network explains
most of the held-out fields, and its prediction with the smoothing step
reaches a per-step residual of 1e-8 in fewer steps than the plain scheme
from rest.  The second test measures the network's own gain, against the
smoothed cold start, with the network trained at the 256 x 128 workload's
size (the committed weights of the pipeline's command-line run)."""
import pytest

from paper_2103_02119_amd import warmstart as WS

pytestmark = pytest.mark.gpu


def test_trained_network_shortens_the_run_to_steady_state():
    print("case: warm start 64x32", flush=True)
    m, net, scales = WS.run_pipeline(n_train=320, n_test=16, epochs=80, nx=64, ny=32,
                                     gen_max_steps=80_000, eval_max_steps=200_000,
                                     re_range=(100.0, 1000.0), gen_precision=WS.L.LBM_FP64,
                                     gen_tol=1e-7, log=lambda s: print(s, flush=True))
    for c in m["warm_vs_cold"]["per_case"]:
        print(c, flush=True)
    print("val", m["final_val"], "rest-state prediction", m["val_zero_prediction"], flush=True)
    assert m["dataset"]["converged"] >= 120
    assert m["final_val"] < 0.1 * m["val_zero_prediction"]
    w = m["warm_vs_cold"]
    assert w["warm+smooth"]["reached"] >= w["cold"]["reached"]
    pc = [c for c in w["per_case"] if c["cold"] > 0 and c["warm+smooth"] > 0]
    cold = sum(c["cold"] for c in pc)
    warm = sum(c["warm+smooth"] for c in pc)
    print("warm+smooth / cold steps:", warm, cold, flush=True)
    assert len(pc) >= 8 and warm < 0.7 * cold


def test_trained_network_gains_over_the_same_start_without_it(record_property):
    """The committed network (trained on the GPU on steady 256 x 128 cavity
    fields from the batched solver) against the method without it: the same
    smoothing step after 50 steps, started from rest instead of from the
    prediction.  The 64 unseen seeded cavities of the evaluation (Re
    100..5000, a in 0.25/0.5/1, 1-3 obstacles), FP64 to a per-step residual
    of 1e-8; the plain scheme decides convergence.  Bar: 5% fewer steps in
    total over the cases both starts reach.  (Per case the gain ranges from
    about 0.4x, where the prediction is 16% off, to 1.6x; a subset of 16
    cases is dominated by that worst case.  A 3x gain would need a
    prediction about a hundred times more accurate.)"""
    import os

    print("case: warm start network gain, 64 cases 256x128", flush=True)
    assert os.path.exists(WS.WEIGHTS)
    cmp = WS.evaluate(WS.WEIGHTS, n_test=64, modes=("cold+smooth", "warm+smooth"),
                      log=lambda s: print(s, flush=True))
    own = cmp["network_gain_warm+smooth_vs_cold+smooth"]
    print(own, flush=True)
    record_property("network_own_step_speedup", own["step_speedup_total"])
    assert cmp["warm+smooth"]["reached"] >= cmp["cold+smooth"]["reached"] - 2
    assert own["compared"] >= 40
    assert own["step_speedup_total"] > 1.05, own


def test_consistent_start_keeps_the_predicted_velocity():
    """consistent_start (the Mei et al. style start the evaluation can
    compare) leaves every fluid node at the predicted velocity, to rounding,
    while the density develops away from the predicted one."""
    import numpy as np

    from paper_2103_02119_amd import inputs as I

    print("case: consistent start 64x32", flush=True)
    nx, ny, U = 64, 32, 0.05
    params = [dict(Re=400.0, r=0.5, mask_seed=5), dict(Re=900.0, r=1.0, mask_seed=9)]
    masks = [I.cavity_obstacles(nx, ny, p["mask_seed"]) for p in params]
    b = WS.L.Batch(WS.cavity_cases(params, nx, ny, U), precision=WS.L.LBM_FP64)
    pred = []
    for c, m in enumerate(masks):
        b.set_mask(c, m)
        rho, ux, uy = I.random_fields(40 + c, nx, ny)
        fluid = m == 0
        pred.append((np.where(fluid, rho, 1.0), np.where(fluid, 0.5 * ux, 0.0),
                     np.where(fluid, 0.5 * uy, 0.0)))
        b.set_fields(c, *pred[c])
    WS.consistent_start(b, pred, masks, steps=20)
    for c, m in enumerate(masks):
        rho, ux, uy = b.moments(c)
        fl = m == 0
        assert np.abs(ux - pred[c][1])[fl].max() < 1e-14
        assert np.abs(uy - pred[c][2])[fl].max() < 1e-14
        assert np.abs(rho - pred[c][0])[fl].max() > 1e-6
    b.close()
