"""The shock tube of the results section on the GPU: end planes held at the
equilibria of C_L and C_R (lbm_set_fixed_planes), sides periodic.  Parity
with the oracle element by element on tubes whose waves reach the held
planes, and the paper-size 11 x 11 x 800 tube against the oracle and the
exact Riemann plateaus."""
import numpy as np
import pytest
import torch

from gpu_helpers import new_sim, rel_errors
from oracle import equilibrium as oeq, lbm as olbm, riemann as orm, velocity_sets as ovs
from paper_1303_4624_amd import Simulation, _lib as L
from synth_inputs import WORKLOADS, smooth_ic, smooth_noise, tube_ic, tube_states, workload_ic

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
FP32S_TOL = 1e-5
# plateau means (the quantity the experiment compares) against the oracle's
PLATEAU_TOL = 1e-6


def _say(*a):
    print(*a, flush=True)


def _state(rho, theta, T0, D, u=0.0):
    return (rho,) + (u,) * D + (theta * T0,)


def _gpu(model, extent, omega, rho, U, th, steps, hold, precision="fp64"):
    sim = new_sim(model, extent, omega, precision)
    n_lo, n_hi, lo, hi = hold(sim.T0)
    sim.init_fields(rho, U, th * sim.T0)
    sim.set_fixed_planes(n_lo, n_hi, lo, hi)
    sim.step(steps)
    r, u, t = [x.cpu().numpy() for x in sim.moments()]
    f = sim.get_populations().cpu()
    T0 = sim.T0
    sim.close()
    return r, u, t, T0, f


def _oracle(model, rho, U, th, steps, omega, hold):
    v = ovs.velocity_set(model)
    f = olbm.run(v, olbm.init_populations(v, rho, U, th * v.T0), omega, steps, hold(v.T0))
    r, u, t = oeq.moments(v, f)
    return r.numpy(), u.numpy(), t.numpy(), f, v


@pytest.mark.parametrize("model,extent,steps,n_lo,n_hi", [
    # waves from the centre reach and reflect off the held planes
    ("D3Q95", (5, 3, 40), 30, 5, 5),
    ("D3Q95", (7, 2, 33), 25, 5, 2),     # asymmetric, thinner than the stencil at the top
    ("D3Q95", (300, 2, 24), 10, 0, 5),   # one held end; rows span two chunks, ragged tail
    ("D2Q33", (7, 33), 30, 4, 4),
    ("D2Q33", (5, 28), 20, 3, 0),
    ("D3Q95", (64, 2, 24), 10, 5, 5),    # whole rows per block: held and free rows in one block
])
def test_held_tube_matches_oracle_elementwise(model, extent, steps, n_lo, n_hi):
    _say("case", model, extent, steps, n_lo, n_hi)
    D = len(extent)
    rho, U, th = tube_ic(extent, extent[-1] // 2, (2.0, 1.0), (1.0, 1.1))
    # a smooth perturbation so that no two nodes of a plane agree
    pr, pU, pth = smooth_ic(extent, seeds=(71, 72, 73, 74, 75), amp_u=0.02, amp_rho=0.02,
                            amp_theta=0.02)
    rho, U, th = rho * pr, U + pU, th * pth

    def hold(T0):
        return (n_lo, n_hi, _state(2.0, 1.0, T0, D), _state(1.0, 1.1, T0, D, 0.01))

    r, u, t, T0, f = _gpu(model, extent, 1.4, rho, U, th, steps, hold)
    ro, uo, to, fo, v = _oracle(model, rho, U, th, steps, 1.4, hold)
    er, eu, et = rel_errors((r, u, t), (ro, uo, to), T0)
    want = olbm.collide(v, fo, 1.4)    # the library stores post-collision populations
    ef = float(torch.max(torch.abs(f - want)) / torch.max(torch.abs(want)))
    _say("errors", er, eu, et, ef)
    assert max(er, eu, et, ef) <= FP64_TOL
    r32, u32, t32, _, _ = _gpu(model, extent, 1.4, rho, U, th, steps, hold, "fp32s")
    e32 = rel_errors((r32, u32, t32), (ro, uo, to), T0)
    _say("fp32s errors", *e32)
    assert max(e32) <= FP32S_TOL


@pytest.mark.parametrize("wname,plateaus", [
    ("d3q95_11x11x800_tube", ((300, 480), (540, 700))),
    ("d2q33_11x800_tube", ((340, 390), (470, 580))),
])
@pytest.mark.parametrize("precision,tol", [("fp64", FP64_TOL), ("fp32s", FP32S_TOL)])
def test_paper_tube_matches_oracle_and_exact_plateaus(wname, plateaus, precision, tol):
    # The sides are periodic and the initial state is uniform across them, so
    # the oracle's one-node-wide tube is the exact answer for every node of a
    # plane; the GPU must also keep every plane uniform.
    w = WORKLOADS[wname]
    _say("case", wname, precision, w.extent, w.steps)
    D = len(w.extent)
    (lr, lt), (rr, rt) = tube_states(w)
    nh = int(w.extra["hold"])

    def hold(T0):
        return (nh, nh, _state(lr, lt, T0, D), _state(rr, rt, T0, D))

    rho, U, th = workload_ic(w)
    r, u, t, T0, _ = _gpu(w.model, w.extent, w.omega, rho, U, th, w.steps, hold, precision)
    ext1 = (1,) * (D - 1) + (w.extent[-1],)
    r1, U1, th1 = workload_ic(w, ext1)
    ro, uo, to, _, v = _oracle(w.model, r1, U1, th1, w.steps, w.omega, hold)
    axes = tuple(range(1, D))
    for a, b in ((r, ro), (t, to)):
        assert np.all(a == a[(slice(None),) + (slice(0, 1),) * (D - 1)]), "plane not uniform"
    er, eu, et = rel_errors((r, u, t), (np.broadcast_to(ro, r.shape),
                                        np.broadcast_to(uo, u.shape),
                                        np.broadcast_to(to, t.shape)), T0)
    zmax = int(np.argmax(np.abs(r - np.broadcast_to(ro, r.shape)).max(axis=axes)))
    _say("errors", er, eu, et, "largest rho difference at plane", zmax)
    assert max(er, eu, et) <= tol
    (a, b), (c, d) = plateaus
    ro1, to1 = ro.reshape(-1), to.reshape(-1)
    rz = r.mean(axis=axes)
    tz = t.mean(axis=axes)
    pdev = max(abs(rz[a:b].mean() / ro1[a:b].mean() - 1), abs(rz[c:d].mean() / ro1[c:d].mean() - 1),
               abs(tz[a:b].mean() / to1[a:b].mean() - 1), abs(tz[c:d].mean() / to1[c:d].mean() - 1))
    _say("plateau deviation from the oracle", pdev)
    assert pdev <= PLATEAU_TOL
    st = orm.star_state((lr, 0.0, lr * lt * T0), (rr, 0.0, rr * rt * T0),
                        orm.monatomic_gamma(D))
    dev = (rz[a:b].mean() / st.rho_l - 1, rz[c:d].mean() / st.rho_r - 1,
           tz[a:b].mean() / (st.p / st.rho_l) - 1, tz[c:d].mean() / (st.p / st.rho_r) - 1)
    _say("plateau deviations", dev)
    assert max(abs(x) for x in dev) < 2e-3


@pytest.mark.parametrize("model,extent,n,k,n_lo,n_hi", [
    ("D3Q95", (5, 3, 40), 12, 5, 5, 5),
    ("D2Q33", (7, 33), 10, 4, 4, 4),
    ("D3Q95", (64, 2, 24), 8, 3, 5, 5),   # whole rows per block: held and free rows in one
])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("fp32s", 1e-5)])
def test_held_tube_temperature_gradient_matches_oracle_autograd(model, extent, n, k, n_lo, n_hi,
                                                                precision, tol):
    # The held cells' post-collision values are constants: the adjoint state
    # is zero there, and the initial field on the held planes still matters
    # through the first step.  The omega gradient is refused with held planes.
    _say("case", model, extent, n, k, n_lo, n_hi, precision)
    D = len(extent)
    rho, U, th = tube_ic(extent, extent[-1] // 2, (2.0, 1.0), (1.0, 1.1))
    pr, pU, pth = smooth_ic(extent, seeds=(51, 52, 53, 54, 55), amp_u=0.02, amp_rho=0.02,
                            amp_theta=0.02)
    rho, U, th = rho * pr, U + pU, th * pth
    v = ovs.velocity_set(model)
    lo, hi = _state(2.0, 1.0, v.T0, D), _state(1.0, 1.1, v.T0, D, 0.01)
    target = 1.3 + 0.01 * smooth_noise(extent, 56)
    _, gT_o, _ = olbm.loss_and_grad(v, rho, U, th * v.T0, 1.4, n, target, (n_lo, n_hi, lo, hi))
    gT_o = gT_o.numpy()
    out = []
    for streaming, keep in (("ab", 1), ("ab", 99), ("aa", 1)):
        sim = Simulation(model, extent, 1.4, precision=precision, streaming=streaming)
        try:
            sim.init_fields(rho, U, th * sim.T0)
            sim.set_fixed_planes(n_lo, n_hi, lo, hi)
            ck = sim.run_checkpointed(n, k, keep)
            r = sim.moments()[0]
            g = 2.0 * (r - torch.as_tensor(target, device=r.device))
            with pytest.raises(L.LBMError) as ex:
                sim.adjoint(n, k, ck, rho, U, th * sim.T0, g, keep=keep)
            assert ex.value.status == L.LBM_E_UNSUPPORTED
            dT, dw = sim.adjoint(n, k, ck, rho, U, th * sim.T0, g, keep=keep, want_omega=False)
            assert dw is None
            out.append(dT.cpu().numpy())
        finally:
            sim.close()
    err = np.max(np.abs(out[0] - gT_o)) / np.max(np.abs(gT_o))
    _say("dT error", err)
    assert err <= tol
    # kept moments and in-place forward runs give the same gradient bit for bit
    assert np.array_equal(out[0], out[1]) and np.array_equal(out[0], out[2])


def test_held_planes_clear_to_periodic():
    ext = (6, 4, 20)
    rho, U, th = smooth_ic(ext, seeds=(81, 82, 83, 84, 85), amp_u=0.03)
    sim = new_sim("D3Q95", ext, 1.3)
    ref = new_sim("D3Q95", ext, 1.3)
    try:
        st = _state(1.0, 1.0, sim.T0, 3)
        sim.init_fields(rho, U, th * sim.T0)
        sim.set_fixed_planes(5, 5, st, st)
        sim.set_fixed_planes(0, 0)
        sim.step(7)
        ref.init_fields(rho, U, th * ref.T0)
        ref.step(7)
        assert torch.equal(sim.get_populations(), ref.get_populations())
    finally:
        sim.close()
        ref.close()


def _crossing(z, y, level, from_right=True):
    """Position where y crosses `level`, linearly interpolated (scanning from
    the right end when from_right)."""
    idx = range(len(y) - 2, -1, -1) if from_right else range(len(y) - 1)
    for i in idx:
        a, b = y[i] - level, y[i + 1] - level
        if a == 0:
            return float(z[i])
        if a * b < 0:
            return float(z[i] + (z[i + 1] - z[i]) * a / (a - b))
    return float("nan")


@pytest.mark.parametrize("wname,plateaus", [
    ("d3q95_11x11x800_tube", ((300, 480), (540, 700))),
    ("d2q33_11x800_tube", ((340, 390), (470, 580))),
])
def test_paper_tube_axis_profiles_against_exact_solution(wname, plateaus):
    # The experiment's comparison (the shock-tube paragraph and the caption of
    # its figure): density and temperature along the tube's central axis
    # against the analytical Riemann solution.  Writes the profiles beside the
    # exact ones (gpurun_out/figure1_<workload>.csv and a summary), and bounds
    # the plateau deviations and the front positions.
    import os
    w = WORKLOADS[wname]
    D = len(w.extent)
    (lr, lt), (rr, rt) = tube_states(w)
    nh = int(w.extra["hold"])
    rho, U, th = workload_ic(w)
    prof = {}
    for precision in ("fp64", "fp32s"):
        def hold(T0):
            return (nh, nh, _state(lr, lt, T0, D), _state(rr, rt, T0, D))
        r, u, t, T0, _ = _gpu(w.model, w.extent, w.omega, rho, U, th, w.steps, hold, precision)
        axis = (slice(None),) + tuple(n // 2 for n in w.extent[:-1])[::-1]
        prof[precision] = (r[axis], t[axis] / T0, u[(D - 1,) + axis])
    L_ = w.extent[-1]
    z = np.arange(L_, dtype=np.float64)
    z0 = L_ // 2 - 0.5                 # the initial interface lies between planes L/2 - 1 and L/2
    g = orm.monatomic_gamma(D)
    left, right = (lr, 0.0, lr * lt * T0), (rr, 0.0, rr * rt * T0)
    er, eu, ep = orm.sample(left, right, g, (z - z0) / w.steps)
    eth = ep / er / T0
    st = orm.star_state(left, right, g)
    lh, lt_, rt_, rh = orm.wave_speeds(left, right, g)
    r64, th64, u64 = prof["fp64"]
    (a, b), (c, d) = plateaus
    dev = {"rho_L*": r64[a:b].mean() / st.rho_l - 1, "rho_R*": r64[c:d].mean() / st.rho_r - 1,
           "theta_L*": th64[a:b].mean() / (st.p / st.rho_l / T0) - 1,
           "theta_R*": th64[c:d].mean() / (st.p / st.rho_r / T0) - 1}
    # where the density crosses a level, measured and in the exact profile
    # (sampled 100 times finer); a shock or the contact crosses at its
    # discontinuity, the fan at the given fraction of its density drop
    zf = np.linspace(0, L_ - 1, 100 * (L_ - 1) + 1)
    erf = orm.sample(left, right, g, (zf - z0) / w.steps)[0]
    fan = lambda q: lr - q * (lr - st.rho_l)
    levels = {"shock": (0.5 * (st.rho_r + rr), True), "contact": (0.5 * (st.rho_l + st.rho_r), True),
              "fan 2 %": (fan(0.02), False), "fan 50 %": (fan(0.5), False),
              "fan 98 %": (fan(0.98), False)}
    fronts = {k_: (_crossing(z, r64, lev, fr), _crossing(zf, erf, lev, fr))
              for k_, (lev, fr) in levels.items()}
    assert abs(fronts["shock"][1] - (z0 + rh * w.steps)) < 0.02
    assert abs(fronts["contact"][1] - (z0 + st.u * w.steps)) < 0.02
    out = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "gpurun_out")
    os.makedirs(out, exist_ok=True)
    with open(os.path.join(out, f"figure1_{wname}.csv"), "w") as fh:
        fh.write("z,rho_fp64,theta_fp64,u_fp64,rho_fp32s,theta_fp32s,rho_exact,theta_exact,u_exact\n")
        r32, th32, _ = prof["fp32s"]
        for i in range(L_):
            fh.write(f"{i},{r64[i]:.10g},{th64[i]:.10g},{u64[i]:.10g},{r32[i]:.10g},"
                     f"{th32[i]:.10g},{er[i]:.10g},{eth[i]:.10g},{eu[i]:.10g}\n")
    with open(os.path.join(out, f"figure1_{wname}_summary.txt"), "w") as fh:
        fh.write(f"{wname}: {w.extent}, omega {w.omega}, t = {w.steps}, gamma {g:.6g}, "
                 f"interface at z = {z0}\n")
        fh.write("plateau means (FP64 GPU) against the exact solution:\n")
        for k_, v_ in dev.items():
            fh.write(f"  {k_:9s} {v_:+.3e}\n")
        fh.write("density crossings (FP64 GPU) vs the exact profile, cells (shock, contact: half-way\n"
                 "between the states they join; fan: the fraction of its density drop):\n")
        for k_, (m_, x_) in fronts.items():
            fh.write(f"  {k_:9s} measured {m_:8.2f} exact {x_:8.2f} diff {m_ - x_:+6.2f}\n")
        fh.write(f"FP32-shifted vs FP64 on the axis: rho {np.abs(r32 - r64).max():.2e}, "
                 f"theta {np.abs(th32 - th64).max():.2e}\n")
    _say("plateau deviations", dev)
    _say("fronts", fronts)
    assert max(abs(x) for x in dev.values()) < 2e-3
    # the fronts sit where the exact solution puts them; viscosity (nu =
    # T0 (1/omega - 1/2)) only smears them, which moves the outer edges of the
    # fan by about sqrt(nu t) ~ 8 cells, not its middle
    assert abs(fronts["shock"][0] - fronts["shock"][1]) < 3
    assert abs(fronts["contact"][0] - fronts["contact"][1]) < 3
    assert abs(fronts["fan 50 %"][0] - fronts["fan 50 %"][1]) < 3
    assert abs(fronts["fan 2 %"][0] - fronts["fan 2 %"][1]) < 15
    assert abs(fronts["fan 98 %"][0] - fronts["fan 98 %"][1]) < 15
