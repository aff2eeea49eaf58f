"""lbm_conservation_noalloc (the entry point that allocates nothing: its
reduction scratch is the library's static per-GPU device array) against
lbm_conservation on the same state, bit for bit, over two calls in a row of
which the second has a smaller grid, in both precisions."""
import numpy as np
import pytest
import torch

from paper_1303_4624_amd import Simulation, _lib as L
from synth_inputs import smooth_ic

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp64", "fp32s"])
def test_noalloc_conservation_equals_bound_scratch(precision):
    print("case no-alloc conservation", precision, flush=True)
    for model, extent, steps in (("D3Q95", (96, 40, 36), 5), ("D3Q95", (20, 6, 5), 3),
                                 ("D2Q33", (70, 9), 4)):
        rho, U, th = smooth_ic(extent, seeds=(1, 2, 3, 4, 5)[:len(extent) + 2], amp_u=0.03)
        sim = Simulation(model, extent, 1.3, precision=precision)
        sim.init_fields(rho, U, th * sim.T0)
        sim.step(steps)
        want = L.lbm_conservation(sim.ctx, sim.D)
        got = L.lbm_conservation_noalloc(sim.ctx, sim.D)
        again = L.lbm_conservation_noalloc(sim.ctx, sim.D)
        sim.close()
        print(model, extent, want, got, flush=True)
        assert np.array_equal(got, want) and np.array_equal(again, want)
        assert np.isfinite(got).all() and got[0] > 0
