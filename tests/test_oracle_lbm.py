"""Pins of the oracle's update rule: streaming is an exact permutation (brute
force), collision invariants, conservation, fixed point, mirror symmetry,
shear viscosity against the BGK closed form, the Riemann-problem plateaus of
the shock-tube experiment, and the gradient machinery."""
import itertools

import numpy as np
import pytest
import torch

from conftest import read_golden
from oracle import equilibrium as eq, lbm, riemann as rm, velocity_sets as vs
from synth_inputs import WORKLOADS, grid_shape, smooth_ic, tube_ic, tube_states, workload_ic

MODELS = ["D2Q33", "D3Q95"]


def _ids(Q, shape):
    n = Q * int(np.prod(shape))
    return torch.arange(1, n + 1, dtype=torch.float64).reshape((Q,) + tuple(shape))


@pytest.mark.parametrize("name,extent", [("D2Q33", (5, 3)), ("D2Q33", (1, 2)),
                                         ("D3Q95", (4, 3, 2)), ("D3Q95", (7, 1, 6))])
def test_streaming_is_exact_permutation_brute_force(name, extent):
    # omega = 0 makes the update pure streaming.  Every value must land at
    # ((x + e_i) mod n) per axis, computed here with Python loops.
    v = vs.velocity_set(name)
    shape = grid_shape(extent)
    f = _ids(v.Q, shape)
    out = lbm.stream(v, f)
    assert torch.equal(lbm.step(v, f, 0.0), out)
    for i in range(v.Q):
        for x in itertools.product(*[range(n) for n in extent]):
            dst = tuple((x[a] + int(v.e[i, a])) % extent[a] for a in range(v.D))
            assert out[(i,) + tuple(reversed(dst))] == f[(i,) + tuple(reversed(x))]
    assert torch.equal(out.flatten().sort().values, f.flatten())


@pytest.mark.parametrize("name", MODELS)
def test_collision_conserves_mass_momentum_energy_per_cell(name):
    v = vs.velocity_set(name)
    rng = np.random.default_rng(5)
    shape = grid_shape((6, 5) if v.D == 2 else (4, 3, 2))
    rho = 1 + 0.1 * rng.random(shape)
    U = 0.05 * rng.standard_normal((v.D,) + shape)
    T = v.T0 * (1 + 0.05 * rng.standard_normal(shape))
    f = lbm.init_populations(v, rho, U, T)
    f = f * (1 + 0.05 * torch.as_tensor(rng.standard_normal(f.shape)))   # off equilibrium
    post = lbm.collide(v, f, 1.7)
    E = torch.as_tensor(v.e, dtype=torch.float64)
    for mom in [torch.ones(v.Q)] + [E[:, a] for a in range(v.D)] + [(E * E).sum(1)]:
        a = torch.einsum("q,q...->...", mom.double(), f)
        b = torch.einsum("q,q...->...", mom.double(), post)
        assert torch.allclose(a, b, rtol=0, atol=1e-14)


@pytest.mark.parametrize("name", MODELS)
def test_uniform_equilibrium_is_fixed_point(name):
    v = vs.velocity_set(name)
    shape = grid_shape((4, 4) if v.D == 2 else (3, 3, 3))
    U = np.zeros((v.D,) + shape)
    U[0] = 0.03
    f = lbm.init_populations(v, np.full(shape, 1.2), U, np.full(shape, 1.01 * v.T0))
    g = lbm.run(v, f, 1.3, 5)
    assert torch.allclose(g, f, rtol=1e-13, atol=0)


@pytest.mark.parametrize("name", MODELS)
def test_conserved_sums_closed_form(name):
    # Uniform equilibrium: mass rho N, momentum rho U N, energy N rho (D T + |U|^2) / 2.
    v = vs.velocity_set(name)
    ext = (3, 2) if v.D == 2 else (3, 2, 2)
    shape = grid_shape(ext)
    N = int(np.prod(shape))
    Uc = np.array([0.02, -0.01, 0.03][: v.D])
    U = np.broadcast_to(Uc.reshape((v.D,) + (1,) * v.D), (v.D,) + shape).copy()
    T = 1.05 * v.T0
    f = lbm.init_populations(v, np.full(shape, 1.1), U, np.full(shape, T))
    c = lbm.conserved(v, f).numpy()
    want = np.concatenate([[1.1 * N], 1.1 * N * Uc, [N * 1.1 * (v.D * T + Uc @ Uc) / 2]])
    assert np.allclose(c, want, rtol=1e-14, atol=1e-15)


def test_conservation_over_500_steps_d2q33_double_riemann():
    w = WORKLOADS["d2q33_128x4_riemann2"]
    v = vs.velocity_set(w.model)
    rho, U, th = workload_ic(w)
    f = lbm.init_populations(v, rho, U, th * v.T0)
    c0 = lbm.conserved(v, f)
    f = lbm.run(v, f, w.omega, w.steps)
    c1 = lbm.conserved(v, f)
    scale = torch.tensor([c0[0], c0[0], c0[0], c0[-1]])
    assert torch.all((c1 - c0).abs() / scale <= 1e-13)


def test_mirror_symmetry_d3q95():
    # Reflecting the initial fields in x (and negating U_x) reflects the result.
    v = vs.velocity_set("D3Q95")
    ext = (12, 5, 4)
    rho, U, th = smooth_ic(ext, seeds=(21, 22, 23, 24, 25), amp_u=0.03)
    f = lbm.run(v, lbm.init_populations(v, rho, U, th * v.T0), 1.6, 6)
    r1, u1, t1 = eq.moments(v, f)
    # reflection x -> (nx - 1 - x) maps the periodic grid onto itself
    rho_m = rho[..., ::-1].copy()
    U_m = U[..., ::-1].copy()
    U_m[0] = -U_m[0]
    th_m = th[..., ::-1].copy()
    g = lbm.run(v, lbm.init_populations(v, rho_m, U_m, th_m * v.T0), 1.6, 6)
    r2, u2, t2 = eq.moments(v, g)
    assert torch.allclose(r2, r1.flip(-1), rtol=1e-13, atol=0)
    assert torch.allclose(t2, t1.flip(-1), rtol=1e-13, atol=0)
    assert torch.allclose(u2[0], -u1[0].flip(-1), rtol=0, atol=1e-15)
    assert torch.allclose(u2[1:], u1[1:].flip(-1), rtol=0, atol=1e-15)


@pytest.mark.parametrize("name", MODELS)
@pytest.mark.parametrize("omega", [0.8, 1.5])
def test_shear_wave_decays_at_bgk_viscosity(name, omega):
    # Navier-Stokes closed form for BGK: nu = T0 (1/omega - 1/2); a shear wave
    # U_y = A sin(kx) decays as exp(-nu k^2 t) up to O(k^2) lattice corrections.
    v = vs.velocity_set(name)
    nx = 64
    ext = (nx, 1) if v.D == 2 else (nx, 1, 1)
    shape = grid_shape(ext)
    x = np.broadcast_to(np.arange(nx), shape)
    k = 2 * np.pi / nx
    U = np.zeros((v.D,) + shape)
    U[1] = 1e-4 * np.sin(k * x)
    f = lbm.init_populations(v, np.ones(shape), U, np.full(shape, v.T0))

    def amp(f):
        _, u, _ = eq.moments(v, f)
        return float((u[1].numpy() * np.sin(k * x)).sum() * 2 / x.size)

    f = lbm.run(v, f, omega, 20)
    a1 = amp(f)
    f = lbm.run(v, f, omega, 100)
    a2 = amp(f)
    rate = -np.log(a2 / a1) / 100
    nu = v.T0 * (1 / omega - 0.5)
    assert abs(rate / (nu * k * k) - 1) < 0.02


def test_riemann_textbook_values():
    for row in read_golden("toro_riemann_tests.txt"):
        a, b = row.split("|")
        a = [float(x) for x in a.split()]
        b = [float(x) for x in b.split()]
        st = rm.star_state(a[:3], a[3:], 1.4)
        for got, want in zip([st.p, st.u, st.rho_l, st.rho_r], b):
            assert abs(got - want) <= 1e-4 * abs(want) + 1e-5, (got, want)


def test_riemann_rankine_hugoniot_and_isentrope():
    # right shock: mass and momentum fluxes continuous in the shock frame;
    # left rarefaction: p / rho^gamma constant.
    g = 5.0 / 3.0
    L, R = (1.0, 0.0, 1.0), (0.5, 0.0, 0.4)
    st = rm.star_state(L, R, g)
    _, _, _, s = rm.wave_speeds(L, R, g)
    m1 = R[0] * (R[1] - s)
    m2 = st.rho_r * (st.u - s)
    assert abs(m1 - m2) < 1e-12
    assert abs((R[0] * (R[1] - s) ** 2 + R[2]) - (st.rho_r * (st.u - s) ** 2 + st.p)) < 1e-12
    assert abs(L[2] / L[0] ** g - st.p / st.rho_l ** g) < 1e-12
    rho, u, p = rm.sample(L, R, g, np.linspace(-3, 3, 61))
    assert np.all(np.diff(p[:30]) <= 1e-12)


def test_riemann_plateaus_of_d3q95_shock_tube():
    # The experiment compares plateaus with the exact solution; here on the
    # 512x4x4 periodic tube at t = 40, before the waves from the centre and
    # from the periodic seam meet.
    w = WORKLOADS["d3q95_512x4x4_riemann"]
    v = vs.velocity_set(w.model)
    rho, U, th = workload_ic(w)
    f = lbm.run(v, lbm.init_populations(v, rho, U, th * v.T0), w.omega, 40)
    r, u, T = eq.moments(v, f)
    r = r[0, 0].numpy()
    T = T[0, 0].numpy()
    ux = u[0, 0, 0].numpy()
    st = rm.star_state((1.0, 0.0, v.T0), (0.5, 0.0, 0.5 * 0.8 * v.T0), rm.monatomic_gamma(3))
    assert abs(r[225:261].mean() / st.rho_l - 1) < 0.01
    assert abs(r[300:336].mean() / st.rho_r - 1) < 0.01
    assert abs(T[225:261].mean() / (st.p / st.rho_l) - 1) < 0.01
    assert abs(T[300:336].mean() / (st.p / st.rho_r) - 1) < 0.01
    assert abs(ux[225:336].mean() / st.u - 1) < 0.01


def test_autograd_gradient_matches_central_differences():
    v = vs.velocity_set("D2Q33")
    ext = (10, 6)
    rho, U, th = smooth_ic(ext, seeds=(31, 32, 33, 34), amp_u=0.02)
    T = th * v.T0
    target = 1.0 + 0.01 * np.cos(np.arange(60).reshape(6, 10))
    L, gT, gw = lbm.loss_and_grad(v, rho, U, T, 1.3, 8, target)
    rng = np.random.default_rng(0)
    d = rng.standard_normal(T.shape)
    eps = 1e-6 * v.T0

    def loss(Tf, om):
        with torch.no_grad():
            r = lbm.forward_density(v, rho, U, torch.as_tensor(Tf), om, 8)
            return float(lbm.density_loss(r, torch.as_tensor(target)))

    fd = (loss(T + eps * d, 1.3) - loss(T - eps * d, 1.3)) / (2 * eps)
    an = float((gT.numpy() * d).sum())
    assert abs(fd - an) <= 1e-6 * abs(an)
    fdw = (loss(T, 1.3 + 1e-6) - loss(T, 1.3 - 1e-6)) / 2e-6
    assert abs(fdw - gw) <= 1e-6 * abs(gw)


def test_autograd_gradient_with_held_planes_matches_central_differences():
    # The tube's end planes: the held values are constants, so the gradient
    # with respect to T_init comes only through the first step's gathers from
    # them and through the free cells; central differences of the forward run
    # (no autograd) check it, and T_init on a held plane after the first step
    # matters only through that first step.
    v = vs.velocity_set("D2Q33")
    ext = (5, 14)
    rho, U, th = tube_ic(ext, 7, (2.0, 1.0), (1.0, 1.1))
    pr, pU, pth = smooth_ic(ext, seeds=(41, 42, 43, 44), amp_u=0.02, amp_rho=0.02,
                            amp_theta=0.02)
    rho, U, th = rho * pr, U + pU, th * pth
    T = th * v.T0
    hold = (4, 4, (2.0, 0.0, 0.0, v.T0), (1.0, 0.0, 0.0, 1.1 * v.T0))
    target = 1.2 + 0.01 * np.cos(np.arange(70).reshape(14, 5))
    L, gT, gw = lbm.loss_and_grad(v, rho, U, T, 1.3, 5, target, hold)
    eps = 1e-6 * v.T0

    def loss(Tf):
        with torch.no_grad():
            r = lbm.forward_density(v, rho, U, torch.as_tensor(Tf), 1.3, 5, hold)
            return float(lbm.density_loss(r, torch.as_tensor(target)))

    rng = np.random.default_rng(1)
    d = rng.standard_normal(T.shape)
    fd = (loss(T + eps * d) - loss(T - eps * d)) / (2 * eps)
    an = float((gT.numpy() * d).sum())
    assert abs(fd - an) <= 1e-6 * abs(an)
    # a held-plane cell: nonzero (its initial value feeds the first step)
    e = np.zeros(T.shape)
    e[1, 2] = 1.0
    fd1 = (loss(T + eps * e) - loss(T - eps * e)) / (2 * eps)
    assert abs(fd1 - float(gT[1, 2])) <= 1e-6 * abs(fd1) and abs(fd1) > 0


def test_adjoint_pairing_is_invariant_in_time():
    # The step f -> S C(f) is homogeneous of degree one (U and T are ratios of
    # moments), so <dL/df^t, f^t> is the same at every t.
    v = vs.velocity_set("D2Q33")
    ext = (9, 5)
    rho, U, th = smooth_ic(ext, seeds=(41, 42, 43, 44), amp_u=0.03)
    fs = [lbm.init_populations(v, rho, U, th * v.T0).requires_grad_(True)]
    for _ in range(6):
        fs.append(lbm.step(v, fs[-1], 1.4))
        fs[-1].retain_grad()
    target = torch.as_tensor(1.0 + 0.02 * np.sin(np.arange(45.0)).reshape(5, 9))
    L = lbm.density_loss(fs[-1].sum(0), target)
    L.backward()
    pairs = [float((f.grad * f.detach()).sum()) for f in fs]
    # The pairing is a sum whose terms cancel about 1e5-fold (here
    # |pair| ~ 1.1e-5 against sum |terms| ~ 1.1), so its float64 rounding
    # scales with sum |terms|, not with |pair|: measured 1.2e-17 * sum |terms|.
    # A step that is not homogeneous moves the pairing by O(|pair|), i.e.
    # 1e-5 * sum |terms|, ten orders above this bar.
    scale = max(float((f.grad * f.detach()).abs().sum()) for f in fs)
    assert abs(pairs[-1]) > 1e-7 * scale
    assert max(abs(p - pairs[-1]) for p in pairs) <= 1e-15 * scale


# -- the shock tube with end planes held at C_L and C_R (results section) ----

def _tube_hold(w, T0, n=None):
    (lr, lt), (rr, rt) = tube_states(w)
    D = len(w.extent)
    n = int(w.extra["hold"]) if n is None else n
    return (n, n, (lr,) + (0.0,) * D + (lt * T0,), (rr,) + (0.0,) * D + (rt * T0,))


@pytest.mark.parametrize("wname,plateaus", [
    # (start, stop) of the left and right plateaus at t = 120, between the
    # rarefaction tail, the contact and the shock of the exact solution
    ("d3q95_11x11x800_tube", ((300, 480), (540, 700))),
    ("d2q33_11x800_tube", ((340, 390), (470, 580))),
])
def test_tube_with_held_end_planes_reaches_exact_riemann_plateaus(wname, plateaus):
    # The experiment's claim: density and temperature agree with the exact
    # solution of the Riemann problem on the plateaus.  The sides are periodic
    # and the initial state is uniform across them, so one node per plane
    # represents the 11-wide tube exactly.
    w = WORKLOADS[wname]
    v = vs.velocity_set(w.model)
    ext = (1,) * (len(w.extent) - 1) + (w.extent[-1],)
    rho, U, th = workload_ic(w, ext)
    f = lbm.run(v, lbm.init_populations(v, rho, U, th * v.T0), w.omega, w.steps,
                _tube_hold(w, v.T0))
    r, u, T = eq.moments(v, f)
    r = r.reshape(-1).numpy()
    T = T.reshape(-1).numpy()
    uz = u[-1].reshape(-1).numpy()
    (lr, lt), (rr, rt) = tube_states(w)
    st = rm.star_state((lr, 0.0, lr * lt * v.T0), (rr, 0.0, rr * rt * v.T0),
                       rm.monatomic_gamma(v.D))
    (a, b), (c, d) = plateaus
    assert abs(r[a:b].mean() / st.rho_l - 1) < 2e-3
    assert abs(r[c:d].mean() / st.rho_r - 1) < 2e-3
    assert abs(T[a:b].mean() / (st.p / st.rho_l) - 1) < 2e-3
    assert abs(T[c:d].mean() / (st.p / st.rho_r) - 1) < 2e-3
    assert abs(uz[a:d].mean() / st.u - 1) < 2e-3
    # undisturbed ends: the held planes and their neighbours keep C_L / C_R
    assert np.allclose(r[:20], lr, rtol=1e-12) and np.allclose(r[-20:], rr, rtol=1e-12)


@pytest.mark.parametrize("name", MODELS)
def test_held_planes_close_the_periodic_seam(name):
    # Nodes gather from at most m = max|e_z| planes away.  With m planes held
    # at each end, what the far end holds reaches a node only through the
    # interior, at most m planes per step: after t steps nodes below
    # L - m - m t are identical for two different far-end states.  Holding
    # fewer planes lets the far end in through the seam at once.
    v = vs.velocity_set(name)
    m = int(np.abs(v.e[:, -1]).max())
    L = 60
    ext = (3,) * (v.D - 1) + (L,)
    rho, U, th = tube_ic(ext, L // 2, (2.0, 1.0), (1.0, 1.2))
    f0 = lbm.init_populations(v, rho, U, th * v.T0)
    lo = (2.0,) + (0.0,) * v.D + (v.T0,)
    hi_a = (1.0,) + (0.0,) * v.D + (1.2 * v.T0,)
    hi_b = (0.7,) + (0.05,) * v.D + (0.9 * v.T0,)
    for t in (1, 3, 5):
        fa = lbm.run(v, f0, 1.3, t, (m, m, lo, hi_a))
        fb = lbm.run(v, f0, 1.3, t, (m, m, lo, hi_b))
        cut = L - m - m * t
        assert torch.equal(fa[:, :cut], fb[:, :cut])
        assert not torch.equal(fa[:, cut:], fb[:, cut:])
        # the held planes carry f^eq of the held states
        ra, ua, Ta = eq.moments(v, fa)
        assert torch.allclose(ra[:m], torch.full_like(ra[:m], 2.0), rtol=1e-14)
        assert torch.allclose(Ta[-m:], torch.full_like(Ta[-m:], 1.2 * v.T0), rtol=1e-14)
    # the second step gathers the first step's held planes across the seam
    fa = lbm.run(v, f0, 1.3, 2, (m - 1, m - 1, lo, hi_a))
    fb = lbm.run(v, f0, 1.3, 2, (m - 1, m - 1, lo, hi_b))
    assert not torch.equal(fa[:, m - 1], fb[:, m - 1])


def test_held_planes_of_the_periodic_state_change_nothing():
    # Holding both ends at the state a uniform lattice already has is the
    # periodic run; holding zero planes is the periodic run for any state.
    v = vs.velocity_set("D2Q33")
    ext = (4, 30)
    shape = grid_shape(ext)
    st = (1.3, 0.02, -0.01, 0.9 * v.T0)
    f0 = lbm.init_populations(v, np.full(shape, st[0]),
                              np.stack([np.full(shape, st[1]), np.full(shape, st[2])]),
                              np.full(shape, st[3]))
    fp = lbm.run(v, f0, 1.1, 4)
    assert torch.allclose(lbm.run(v, f0, 1.1, 4, (4, 4, st, st)), fp, rtol=0, atol=1e-15)
    rho, U, th = smooth_ic(ext, seeds=(61, 62, 63, 64), amp_u=0.03)
    f1 = lbm.init_populations(v, rho, U, th * v.T0)
    assert torch.equal(lbm.run(v, f1, 1.1, 4, (0, 0, None, None)), lbm.run(v, f1, 1.1, 4))
