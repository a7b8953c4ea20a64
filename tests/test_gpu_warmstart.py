"""The learned warm start end to end on small cavities (64 x 32 nodes):
steady fields from the batched solver, training on the GPU kernels, and the
plain lattice Boltzmann scheme as the judge of the result.  The network must
shorten the way to a residual of 1e-8 against the same procedure started
from rest."""
import numpy as np
import pytest

from paper_2103_02119_amd import warmstart as WS

pytestmark = pytest.mark.gpu


def test_trained_network_shortens_the_run_to_steady_state():
    print("case: warm start 64x32", flush=True)
    m, net, scales = WS.run_pipeline(n_train=320, n_test=16, epochs=60, nx=64, ny=32,
                                     gen_max_steps=60_000, eval_max_steps=200_000,
                                     re_range=(100.0, 1000.0), log=lambda s: print(s, flush=True))
    assert m["dataset"]["converged"] >= 160
    assert m["final_val"] < 0.05
    w = m["warm_vs_cold"]
    assert w["warm+smooth"]["reached"] >= w["cold+smooth"]["reached"] - 1
    pc = [c for c in w["per_case"] if c["cold+smooth"] > 0 and c["warm+smooth"] > 0]
    cold = sum(c["cold+smooth"] for c in pc)
    warm = sum(c["warm+smooth"] for c in pc)
    print("warm / cold steps:", warm, cold, flush=True)
    assert len(pc) >= 8 and warm < 0.9 * cold
