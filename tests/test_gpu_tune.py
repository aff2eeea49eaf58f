"""The forward steps' two block orders (lbm_tune_step, lbm_set_block_order):
the order only decides which blocks run on which XCD, so every result is
bit-identical under both, through single steps, tuning, graph replay,
checkpointed runs, restores and the adjoint."""
import pytest
import torch

from paper_1303_4624_amd import Simulation
from paper_1303_4624_amd import _lib as L
from synth_inputs import smooth_ic

pytestmark = pytest.mark.gpu

# Extents chosen so that the alternative order is active (the grid holds a
# multiple of 8 slabs of blocks): ragged rows, packed rows in float64 and for
# a lower-order set, and 2D rows.
CASES = [
    ("D3Q95", (70, 24, 16), "fp32s"),    # 24 blocks per z-plane, 16 planes
    ("D3Q95", (128, 16, 8), "fp64"),     # two rows per block
    ("D2Q33", (96, 40), "fp32s"),        # one block per row
    ("D3Q19", (64, 16, 16), "fp64"),     # eight rows per block
]


def _say(*a):
    print(*a, flush=True)


def _state(s):
    torch.cuda.synchronize()
    return s.get_populations()


def _pair(model, extent, precision, **kw):
    D = len(extent)
    rho, U, th = smooth_ic(extent, seeds=tuple(range(71, 71 + D + 2)), amp_u=0.03)
    a = Simulation(model, extent, 1.6, precision=precision, **kw)
    b = Simulation(model, extent, 1.6, precision=precision, **kw)
    for s in (a, b):
        s.init_fields(rho, U, th * s.T0)
    return a, b, (rho, U, th)


@pytest.mark.parametrize("model,extent,precision", CASES)
def test_tuned_steps_equal_plain_steps(model, extent, precision):
    _say("case", model, extent, precision)
    a, b, _ = _pair(model, extent, precision)
    try:
        order = a.tune_step(8)
        b.step(8)
        _say("order kept", order)
        assert order in (0, 1)
        assert torch.equal(_state(a), _state(b))
        a.step(5)
        b.step(5)
        assert torch.equal(_state(a), _state(b))
        # both orders, explicitly, over an odd number of steps
        for order in (1, 0, 1):
            a.set_block_order(order)
            a.step(3)
            b.step(3)
            assert torch.equal(_state(a), _state(b)), order
    finally:
        a.close()
        b.close()


@pytest.mark.parametrize("model,extent,precision", CASES[:2])
def test_checkpoints_adjoint_and_graphs_under_the_other_order(model, extent, precision):
    # order 1 in the checkpointed forward run and in the adjoint's
    # recomputation; the adjoint's own kernels keep order 0 either way
    _say("case", model, extent, precision)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        a, b, (rho, U, th) = _pair(model, extent, precision, stream=stream)
        try:
            a.set_block_order(1)
            n, k, keep = 10, 4, 1
            out = []
            for s in (a, b):
                r0, u0, t0 = [x.clone() for x in s.moments()]
                ck = s.run_checkpointed(n, k, keep)
                r = s.moments()[0]
                g = 2.0 * (r - 1.0)
                dT, dw = s.adjoint(n, k, ck, r0, u0, t0, g, keep=keep)
                s.restore_checkpoint(n, k, ck, 1, keep=keep)
                out.append((_state(s), dT.clone(), dw))
            assert torch.equal(out[0][0], out[1][0])
            assert torch.equal(out[0][1], out[1][1]) and out[0][2] == out[1][2]
            a.set_graph_steps(4)
            a.step(9)
            b.step(9)
            assert torch.equal(_state(a), _state(b))
        finally:
            a.close()
            b.close()
    torch.cuda.synchronize()


@pytest.mark.parametrize("model,extent,precision", [CASES[0], CASES[2]])
def test_in_place_tuned_steps_equal_plain_steps(model, extent, precision):
    _say("case", model, extent, precision)
    a, b, _ = _pair(model, extent, precision, streaming="aa")
    try:
        order = a.tune_step(13)          # pairs of (push, local) steps, and one more
        b.step(13)
        _say("order kept", order)
        assert order in (0, 1)
        assert torch.equal(_state(a), _state(b))
        for order in (1, 0):
            a.set_block_order(order)
            a.step(3)
            b.step(3)
            assert torch.equal(_state(a), _state(b)), order
        assert a.tune_step(7) == order   # in place: fewer than 8 steps do not tune
        b.step(7)
        assert torch.equal(_state(a), _state(b))
    finally:
        a.close()
        b.close()


def test_short_runs_do_not_tune():
    model, extent = "D3Q95", (70, 24, 16)
    a, b, _ = _pair(model, extent, "fp32s")
    try:
        a.set_block_order(1)
        assert a.tune_step(3) == 1       # fewer than 4 steps: the order stays
        b.step(3)
        assert torch.equal(_state(a), _state(b))
        with pytest.raises(L.LBMError) as ex:
            a.set_block_order(2)
        assert ex.value.status == L.LBM_E_INVALID
        with pytest.raises(L.LBMError) as ex:
            a.tune_step(-1)
        assert ex.value.status == L.LBM_E_INVALID
    finally:
        a.close()
        b.close()
