"""The lower-order 3D 19- and 15-velocity sets (order of accuracy m = 2,
second-order Hermite equilibrium; the construction's lower-order models named
after Formula (10)) run through the same kernel template as D3Q95, checked
against the FP64 oracle on the same seeded inputs.  Bars: FP64 within 1e-12
relative (fields), FP32-shifted within 1e-5 after 200 steps, pure streaming
bitwise, in-place streaming bit-identical to two-buffer streaming, the FP64
adjoint within 1e-11 of the oracle's autograd gradient."""
import numpy as np
import pytest
import torch

from gpu_helpers import gpu_run, new_sim, oracle_run, rel_errors
from oracle import lbm as olbm, velocity_sets as ovs
from synth_inputs import grid_shape, smooth_ic, smooth_noise

pytestmark = pytest.mark.gpu

MODELS = ["D3Q19", "D3Q15"]


def _say(*a):
    print(*a, flush=True)


def _double_riemann(extent):
    # rho = 1, theta = 1 outside x in [nx/4, 3nx/4), rho = 0.8, theta = 0.9 inside
    shape = grid_shape(extent)
    nx = extent[0]
    x = np.arange(nx)
    inside = (x >= nx // 4) & (x < 3 * nx // 4)
    rho = np.broadcast_to(np.where(inside, 0.8, 1.0), shape).copy()
    th = np.broadcast_to(np.where(inside, 0.9, 1.0), shape).copy()
    U = np.zeros((3,) + shape)
    return rho, U, th


@pytest.mark.parametrize("model", MODELS)
@pytest.mark.parametrize("extent,steps,ic", [((40, 24, 16), 60, "smooth"),
                                             ((128, 4, 4), 150, "riemann"),
                                             ((70, 5, 3), 9, "smooth"),     # ragged rows
                                             ((64, 6, 4), 7, "smooth"),     # packed rows
                                             ((1, 1, 1), 3, "smooth")])
def test_fp64_matches_oracle(model, extent, steps, ic):
    _say("case", model, extent, steps, ic)
    if ic == "riemann":
        rho, U, th = _double_riemann(extent)
    elif np.prod(extent) > 8:
        rho, U, th = smooth_ic(extent, seeds=(91, 92, 93, 94, 95), amp_u=0.03, amp_rho=0.03,
                               amp_theta=0.03)
    else:
        rng = np.random.default_rng(4)
        rho, U, th = (1 + 0.05 * rng.standard_normal((1, 1, 1)),
                      0.03 * rng.standard_normal((3, 1, 1, 1)),
                      1 + 0.02 * rng.standard_normal((1, 1, 1)))
    g = gpu_run(model, extent, 1.3, rho, U, th, steps)
    o = oracle_run(model, rho, U, th, steps, 1.3)
    er, eu, et = rel_errors(g, o, g[3])
    _say("errors", er, eu, et)
    assert er <= 1e-12 and eu <= 1e-12 and et <= 1e-12


@pytest.mark.parametrize("model", MODELS)
def test_streaming_is_an_exact_permutation(model):
    v = ovs.velocity_set(model)
    extent = (9, 4, 3)
    shape = grid_shape(extent)
    f0 = torch.arange(1, v.Q * int(np.prod(shape)) + 1, dtype=torch.float64).reshape((v.Q,) + shape)
    sim = new_sim(model, extent, 0.0)
    sim.set_populations(f0.cuda())
    sim.step(3)
    got = sim.get_populations().cpu()
    sim.close()
    assert torch.equal(got, olbm.stream(v, olbm.stream(v, olbm.stream(v, f0))))


@pytest.mark.parametrize("model", MODELS)
def test_fp32_shifted_matches_oracle_after_200_steps(model):
    extent = (40, 24, 16)
    rho, U, th = smooth_ic(extent, seeds=(1, 2, 3, 4, 5))
    g = gpu_run(model, extent, 1.5, rho, U, th, 200, precision="fp32s", rho0=1.0)
    o = oracle_run(model, rho, U, th, 200, 1.5)
    er, eu, et = rel_errors(g, o, g[3])
    _say("errors", model, er, eu, et)
    assert er <= 1e-5 and eu <= 1e-5 and et <= 1e-5


@pytest.mark.parametrize("model", MODELS)
@pytest.mark.parametrize("precision", ["fp64", "fp32s"])
def test_in_place_streaming_is_bit_identical(model, precision):
    from paper_1303_4624_amd import Simulation
    extent = (70, 6, 5)
    rho, U, th = smooth_ic(extent, seeds=(11, 12, 13, 14, 15), amp_u=0.04)
    out = []
    for scheme in ("ab", "aa"):
        sim = Simulation(model, extent, 1.6, precision=precision, streaming=scheme)
        sim.init_fields(rho, U, th * sim.T0)
        sim.step(7)
        out.append([x.cpu().numpy() for x in sim.moments()] + [sim.get_populations().cpu().numpy()])
        sim.close()
    for a, b in zip(*out):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("model", MODELS)
def test_fp64_adjoint_matches_oracle_autograd(model):
    v = ovs.velocity_set(model)
    extent, n, k, omega = (16, 10, 6), 9, 4, 1.4
    rho, U, th = smooth_ic(extent, seeds=(21, 22, 23, 24, 25), amp_u=0.03)
    target = rho * (1.0 + 0.05 * smooth_noise(extent, 26))
    L_o, gT_o, gw_o = olbm.loss_and_grad(v, rho, U, th * v.T0, omega, n, target)
    gT_o = gT_o.numpy()
    sim = new_sim(model, extent, omega, "fp64")
    sim.init_fields(rho, U, th * sim.T0)
    ck = sim.run_checkpointed(n, k, 1)
    r = sim.moments()[0]
    g = 2.0 * (r - torch.as_tensor(target, device="cuda"))
    dT, dw = sim.adjoint(n, k, ck, rho, U, th * sim.T0, g, keep=1)
    gT = dT.cpu().numpy()
    sim.close()
    eT = np.max(np.abs(gT - gT_o)) / np.max(np.abs(gT_o))
    ew = abs(dw - gw_o) / abs(gw_o)
    _say("adjoint", model, eT, ew)
    assert eT <= 1e-11 and ew <= 1e-11
