"""In-place (AA-pattern) streaming on the GPU: the same update as the
two-buffer path, bit for bit, at every step count (both storage forms), on
ragged and tiny grids, at the benchmark sizes, and against the oracle."""
import numpy as np
import pytest
import torch

from gpu_helpers import oracle_run, rel_errors
from paper_1303_4624_amd import Simulation, _lib as L
from synth_inputs import WORKLOADS, smooth_ic, tube_states, workload_ic

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _ic(extent, seed0=91):
    return smooth_ic(extent, seeds=tuple(range(seed0, seed0 + len(extent) + 2)), amp_u=0.03,
                     amp_rho=0.03, amp_theta=0.02)


def _pair(model, extent, precision, omega=1.6):
    ab = Simulation(model, extent, omega, precision=precision)
    aa = Simulation(model, extent, omega, precision=precision, streaming="aa")
    return ab, aa


def _same(ab, aa):
    for x, y in zip(ab.moments(), aa.moments()):
        assert torch.equal(x, y)
    assert torch.equal(ab.get_populations(), aa.get_populations())
    assert np.array_equal(ab.conservation(), aa.conservation())


@pytest.mark.parametrize("model,extent", [
    ("D3Q95", (300, 5, 3)),     # two chunks per row, ragged tail, wrap more than once
    ("D3Q95", (16, 8, 4)),
    ("D3Q95", (1, 1, 1)),       # every displacement lands on the cell itself
    ("D2Q33", (70, 3)),
    ("D2Q33", (33, 17)),
    ("D2Q33", (2, 1)),
    ("D3Q95", (64, 6, 4)),      # whole rows per block
    ("D2Q33", (128, 6)),
])
@pytest.mark.parametrize("precision", ["fp64", "fp32s"])
def test_in_place_equals_two_buffer_bitwise(model, extent, precision):
    _say("case", model, extent, precision)
    rho, U, th = _ic(extent)
    ab, aa = _pair(model, extent, precision)
    try:
        for s in (ab, aa):
            s.init_fields(rho, U, th * s.T0)
        _same(ab, aa)
        for n in (1, 1, 1, 3, 4):           # odd and even counts: both storage forms
            ab.step(n)
            aa.step(n)
            _same(ab, aa)
    finally:
        ab.close()
        aa.close()


@pytest.mark.parametrize("model,extent", [("D3Q95", (24, 10, 6)), ("D2Q33", (40, 12))])
def test_in_place_matches_oracle_and_set_populations(model, extent):
    _say("case", model, extent)
    rho, U, th = _ic(extent, 95)
    steps = 7
    o = oracle_run(model, rho, U, th, steps, 1.3)
    aa = Simulation(model, extent, 1.3, precision="fp64", streaming="aa")
    try:
        aa.init_fields(rho, U, th * aa.T0)
        aa.step(steps)
        g = [x.cpu().numpy() for x in aa.moments()] + [aa.T0]
        errs = rel_errors(g, o, aa.T0)
        _say("errors", errs)
        assert max(errs) <= 1e-12
        # set the populations while the state is in the pushed form, read back
        f = aa.get_populations()
        aa.set_populations(f)
        assert torch.equal(aa.get_populations(), f)
        ab = Simulation(model, extent, 1.3, precision="fp64")
        ab.set_populations(f)
        for n in (1, 2):
            ab.step(n)
            aa.step(n)
            _same(ab, aa)
        ab.close()
    finally:
        aa.close()


@pytest.mark.parametrize("model,extent,n_lo,n_hi", [
    ("D3Q95", (5, 3, 40), 5, 5),
    ("D3Q95", (7, 2, 33), 5, 2),      # thinner than the stencil at the top
    ("D3Q95", (300, 2, 24), 0, 5),    # one held end; two chunks per row, ragged tail
    ("D2Q33", (7, 33), 4, 4),
    ("D2Q33", (5, 28), 3, 0),
    ("D3Q19", (6, 4, 12), 2, 3),      # lower-order sets: displacements of 1
    ("D3Q15", (5, 3, 9), 1, 1),
])
@pytest.mark.parametrize("precision", ["fp64", "fp32s"])
def test_in_place_with_held_planes_equals_two_buffer_bitwise(model, extent, n_lo, n_hi,
                                                             precision):
    # The held cells store f^eq of their state into the locations they own in
    # either storage form; waves from the centre reach the held planes.
    _say("case", model, extent, n_lo, n_hi, precision)
    D = len(extent)
    rho, U, th = _ic(extent, 61)
    ab, aa = _pair(model, extent, precision, omega=1.4)
    try:
        lo = (2.0,) + (0.0,) * D + (1.0 * ab.T0,)
        hi = (1.0,) + (0.01,) * D + (1.1 * ab.T0,)
        for s in (ab, aa):
            s.init_fields(rho, U, th * s.T0)
            s.set_fixed_planes(n_lo, n_hi, lo, hi)
        for n in (1, 1, 2, 5, 8):          # both storage forms
            ab.step(n)
            aa.step(n)
            _same(ab, aa)
        for s in (ab, aa):                 # back to periodic, in the pushed form
            s.set_fixed_planes(0, 0)
        for n in (3, 2):
            ab.step(n)
            aa.step(n)
            _same(ab, aa)
    finally:
        ab.close()
        aa.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32s"])
def test_paper_tube_in_place_equals_two_buffer_bitwise(precision):
    w = WORKLOADS["d3q95_11x11x800_tube"]
    _say("case", w.name, precision)
    (lr, lt), (rr, rt) = tube_states(w)
    nh = int(w.extra["hold"])
    rho, U, th = workload_ic(w)
    ab, aa = _pair(w.model, w.extent, precision, omega=w.omega)
    try:
        for s in (ab, aa):
            s.init_fields(rho, U, th * s.T0)
            s.set_fixed_planes(nh, nh, (lr, 0.0, 0.0, 0.0, lt * s.T0),
                               (rr, 0.0, 0.0, 0.0, rt * s.T0))
            s.step(w.steps - 1)
        _same(ab, aa)
        ab.step(1)
        aa.step(1)
        _same(ab, aa)
    finally:
        ab.close()
        aa.close()


@pytest.mark.parametrize("model,extent,n,k,keep,precision,pre", [
    ("D3Q95", (20, 10, 8), 10, 3, 1, "fp32s", 0),
    ("D3Q95", (20, 10, 8), 10, 3, 99, "fp64", 1),    # starts in the pushed form
    ("D2Q33", (20, 12), 13, 4, 2, "fp32s", 1),
    ("D3Q95", (7, 5, 4), 3, 2, 1, "fp64", 2),
    ("D3Q19", (12, 8, 6), 9, 3, 1, "fp32s", 1),
    ("D3Q15", (10, 6, 5), 8, 4, 2, "fp64", 0),
])
def test_in_place_checkpoints_and_adjoint_equal_two_buffer_bitwise(model, extent, n, k, keep,
                                                                   precision, pre):
    # The in-place run copies its snapshots out in the two-buffer form and
    # stores the same moments, so the adjoint sees the same checkpoints.
    _say("case", model, extent, n, k, keep, precision, pre)
    rho, U, th = _ic(extent, 41)
    tgt = 1.0 + 0.01 * smooth_ic(extent, seeds=tuple(range(51, 51 + len(extent) + 2)))[0]
    ab, aa = _pair(model, extent, precision, omega=1.3)
    try:
        out = []
        for s in (ab, aa):
            T = th * s.T0
            s.init_fields(rho, U, T)
            s.step(pre)
            r0, u0, t0 = [x.clone() for x in s.moments()]
            ck = s.run_checkpointed(n, k, keep)
            r = s.moments()[0]
            g = 2.0 * (r - torch.as_tensor(tgt, device=r.device))
            dT, dw = s.adjoint(n, k, ck, r0, u0, t0, g, keep=keep)
            out.append((s.get_populations(), dT, dw))
        (fa, dTa, dwa), (fb, dTb, dwb) = out
        _say("dL/domega", dwa, dwb)
        assert torch.equal(fa, fb) and torch.equal(dTa, dTb) and dwa == dwb
        _same(ab, aa)
    finally:
        ab.close()
        aa.close()


def test_in_place_lbmfunction_matches_oracle():
    from oracle import lbm as olbm, velocity_sets as ovs
    from paper_1303_4624_amd import LBMFunction
    extent, n, k = (16, 8, 8), 10, 4
    rho, U, th = _ic(extent, 11)
    v = ovs.velocity_set("D3Q95")
    target = np.full(rho.shape, 1.0)
    _, gT_o, gw_o = olbm.loss_and_grad(v, rho, U, th * v.T0, 1.3, n, target)
    sim = Simulation("D3Q95", extent, 1.3, precision="fp64", streaming="aa")
    try:
        T = torch.tensor(th * sim.T0, device="cuda", requires_grad=True)
        w = torch.tensor(1.3, dtype=torch.float64, device="cuda", requires_grad=True)
        r = LBMFunction.apply(T, w, sim, torch.tensor(rho, device="cuda"),
                              torch.tensor(U, device="cuda"), n, k, 1)
        ((r - 1.0) ** 2).sum().backward()
        eT = np.max(np.abs(T.grad.cpu().numpy() - gT_o.numpy())) / np.max(np.abs(gT_o.numpy()))
        ew = abs(float(w.grad) - gw_o) / abs(gw_o)
        _say("errors", eT, ew)
        assert eT <= 1e-9 and ew <= 1e-9
    finally:
        sim.close()


def test_in_place_scheme_is_chosen_before_bind():
    ext = (8, 6, 20)
    rho, U, th = _ic(ext)
    aa = Simulation("D3Q95", ext, 1.3, precision="fp64", streaming="aa")
    try:
        aa.init_fields(rho, U, th * aa.T0)
        with pytest.raises(L.LBMError) as ex:
            L.lbm_set_streaming(aa.ctx, L.LBM_STREAM_AB)    # already bound
        assert ex.value.status == L.LBM_E_STATE
    finally:
        aa.close()


@pytest.mark.parametrize("model,extent,precision", [
    ("D3Q95", (384,) * 3, "fp32s"),
    ("D2Q33", (8192,) * 2, "fp32s"),
    ("D3Q95", (256,) * 3, "fp64"),
])
def test_in_place_equals_two_buffer_at_benchmark_size(model, extent, precision):
    _say("case", model, extent, precision)
    rho, U, th = smooth_ic(extent)
    out = {}
    for scheme in ("ab", "aa"):
        s = Simulation(model, extent, 1.8, precision=precision, streaming=scheme)
        s.init_fields(rho, U, th * s.T0)
        s.step(3)
        out[scheme] = [x.clone() for x in s.moments()]
        s.close()
        del s
        torch.cuda.empty_cache()
    for x, y in zip(out["ab"], out["aa"]):
        assert torch.equal(x, y)


def test_largest_grid_in_place_matches_oracle_on_sampled_cells():
    # 768^3 D3Q95 FP32-shifted: 172 GB of populations, a grid only in-place
    # streaming fits in HBM.  Sampled cells (corners and seams included)
    # against the oracle on periodic patches, as for the benchmark grids.
    from oracle import equilibrium as oeq, lbm as olbm, velocity_sets as ovs
    from synth_inputs import tiled_smooth_ic
    from test_gpu_parity import _centers, _patch
    extent, steps, omega = (768, 768, 768), 3, 1.8
    _say("case largest grid", extent)
    rho, U, th = tiled_smooth_ic(extent, (192, 192, 192))
    sim = Simulation("D3Q95", extent, omega, precision="fp32s", streaming="aa")
    try:
        sim.init_fields(rho, U, th * sim.T0)
        sim.step(steps)
        r_g, u_g, t_g = sim.moments()
        T0 = sim.T0
        centers = _centers(extent)
        samples = [(float(r_g[c[::-1]]), u_g[(slice(None),) + c[::-1]].cpu().numpy(),
                    float(t_g[c[::-1]])) for c in centers]
        del r_g, u_g, t_g
    finally:
        sim.close()
        torch.cuda.empty_cache()
    v = ovs.velocity_set("D3Q95")
    R = 5 * steps + 1
    worst = 0.0
    for c, (rg, ug, tg) in zip(centers, samples):
        pr = _patch(rho, c, R)
        pu = np.stack([_patch(U[a], c, R) for a in range(3)])
        pt = _patch(th, c, R)
        f = olbm.run(v, olbm.init_populations(v, pr, pu, pt * v.T0), omega, steps)
        ro, uo, to = oeq.moments(v, f)
        ro, uo, to = float(ro[R, R, R]), uo[:, R, R, R].numpy(), float(to[R, R, R])
        worst = max(worst, abs(rg - ro) / abs(ro), np.max(np.abs(ug - uo)) / 0.1, abs(tg - to) / T0)
    _say("worst sampled error", worst)
    assert worst <= 1e-6
