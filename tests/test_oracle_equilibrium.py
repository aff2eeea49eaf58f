"""Pins of the oracle's equilibrium and moments: Hermite tensors and coefficients
against Gauss-Hermite quadrature, discrete moments against the Maxwellian's
(Formula (1) up to m = 4), inversion, fixed point."""
import itertools

import numpy as np
import pytest
import torch

from oracle import equilibrium as eq, velocity_sets as vs

MODELS = ["D2Q33", "D3Q95"]


def _hermegauss_nd(D, n=10):
    z, wz = np.polynomial.hermite_e.hermegauss(n)
    wz = wz / np.sqrt(2 * np.pi)          # weights of the standard normal
    pts = np.array(list(itertools.product(z, repeat=D)))
    wts = np.prod(np.array(list(itertools.product(wz, repeat=D))), axis=1)
    return pts, wts


@pytest.mark.parametrize("D", [2, 3])
def test_hermite_tensors_orthogonality(D):
    # E[H^n H^m] under the standard normal: zero for n != m; for n = m the
    # symmetrised product of Kronecker deltas; E[H^n] = 0 for n >= 1.
    pts, wts = _hermegauss_nd(D)
    H = eq.hermite_tensors(torch.as_tensor(pts))
    Hf = [h.reshape(len(wts), -1).numpy() for h in H]
    for n in range(5):
        for m in range(5):
            G = np.einsum("p,pi,pj->ij", wts, Hf[n], Hf[m])
            if n != m:
                assert np.abs(G).max() < 1e-12
            else:
                # n! for the diagonal all-equal index, e.g. E[H2_xx^2] = 2
                idx_all_x = 0
                assert abs(G[idx_all_x, idx_all_x] - [1, 1, 2, 6, 24][n]) < 1e-12
                # trace over distinct orderings: number of index permutations
                assert np.allclose(G, G.T, atol=1e-12)
    # a mixed example: E[H2_xy H2_xy] = 1, E[H2_xy H2_yx] = 1
    G2 = np.einsum("p,pi,pj->ij", wts, Hf[2], Hf[2])
    assert abs(G2[1, 1] - 1) < 1e-12 and abs(G2[1, D] - 1) < 1e-12


@pytest.mark.parametrize("D", [2, 3])
def test_hermite_coefficients_are_projections_of_maxwellian(D):
    # a^(n) = int f_M(xi) H^(n)(xi) dxi with f_M = rho N(u, theta I): evaluate
    # by Gauss-Hermite quadrature of the shifted, scaled Gaussian.
    rng = np.random.default_rng(7)
    pts, wts = _hermegauss_nd(D, 12)
    for _ in range(3):
        rho = 0.5 + rng.random()
        u = 0.3 * rng.standard_normal(D)
        theta = 0.7 + 0.6 * rng.random()
        xi = u + np.sqrt(theta) * pts
        H = eq.hermite_tensors(torch.as_tensor(xi))
        A = eq.maxwell_hermite_coefficients(torch.tensor([rho], dtype=torch.float64),
                                             torch.as_tensor(u[None, :]),
                                             torch.tensor([theta - 1.0], dtype=torch.float64))
        for n in range(5):
            proj = rho * np.einsum("p,pi->i", wts, H[n].reshape(len(wts), -1).numpy())
            assert np.allclose(proj, A[n].reshape(-1).numpy(), atol=1e-12, rtol=1e-12), n


def _maxwell_moment_1d(mean, var, k):
    z, wz = np.polynomial.hermite_e.hermegauss(12)
    wz = wz / np.sqrt(2 * np.pi)
    return float(np.sum(wz * (mean + np.sqrt(var) * z) ** k))


def _random_states(rng, D, n, T0):
    rho = 0.5 + rng.random(n)
    U = 0.08 * rng.standard_normal((D, n))
    T = T0 * (0.8 + 0.4 * rng.random(n))
    return torch.as_tensor(rho), torch.as_tensor(U), torch.as_tensor(T)


@pytest.mark.parametrize("name", MODELS)
def test_discrete_moments_equal_maxwellian_up_to_order_4(name):
    v = vs.velocity_set(name)
    rng = np.random.default_rng(11)
    rho, U, T = _random_states(rng, v.D, 6, v.T0)
    f = eq.feq(v, rho, U, T).numpy()            # (Q, cells)
    E = v.e.astype(np.float64)
    worst = 0.0
    for n in range(5):
        for a in itertools.product(range(n + 1), repeat=v.D):
            if sum(a) != n:
                continue
            mono = np.prod(E ** np.array(a), axis=1)
            disc = mono @ f
            for c in range(f.shape[1]):
                cont = rho[c].item() * np.prod([_maxwell_moment_1d(U[al, c].item(), T[c].item(), a[al])
                                                for al in range(v.D)])
                scale = rho[c].item() * T[c].item() ** (n / 2)
                worst = max(worst, abs(disc[c] - cont) / scale)
    assert worst < 1e-12, worst


@pytest.mark.parametrize("name", MODELS)
def test_discrete_moments_miss_order_5(name):
    # Negative control: the 4th-order equilibrium does not reproduce the
    # Maxwellian's 5th-order moments once the flow is non-zero.
    v = vs.velocity_set(name)
    rho = torch.tensor([1.0])
    U = torch.zeros(v.D, 1)
    U[0, 0] = 0.1
    T = torch.tensor([v.T0 * 1.1])
    f = eq.feq(v, rho, U, T).numpy()[:, 0]
    E = v.e.astype(np.float64)
    a = (5,) + (0,) * (v.D - 1)
    disc = float(np.prod(E ** np.array(a), axis=1) @ f)
    cont = _maxwell_moment_1d(0.1, v.T0 * 1.1, 5)
    assert abs(disc - cont) / abs(cont) > 1e-4


@pytest.mark.parametrize("name", MODELS)
def test_moments_invert_equilibrium(name):
    v = vs.velocity_set(name)
    rng = np.random.default_rng(3)
    rho, U, T = _random_states(rng, v.D, 50, v.T0)
    r, u, t = eq.moments(v, eq.feq(v, rho, U, T))
    assert torch.allclose(r, rho, rtol=1e-14, atol=0)
    assert torch.allclose(u, U, rtol=0, atol=1e-15)
    assert torch.allclose(t, T, rtol=1e-14, atol=0)


@pytest.mark.parametrize("name", MODELS)
def test_rest_state_equilibrium_is_weights(name):
    v = vs.velocity_set(name)
    f = eq.feq(v, torch.tensor([1.3], dtype=torch.float64), torch.zeros(v.D, 1, dtype=torch.float64),
               torch.tensor([v.T0], dtype=torch.float64))
    assert np.allclose(f[:, 0].numpy(), 1.3 * v.w, rtol=1e-14, atol=0)


@pytest.mark.parametrize("name,theta_neg", [("D2Q33", 0.55), ("D3Q95", 0.6)])
def test_equilibrium_positivity_range(name, theta_neg):
    # Positive for the temperature range of every workload, negative well
    # below it (the paper gives no admissible range; this records where it ends).
    v = vs.velocity_set(name)
    ok = eq.min_feq_ratio(v, torch.tensor([1.0]), torch.zeros(v.D, 1), torch.tensor([0.8 * v.T0]))
    bad = eq.min_feq_ratio(v, torch.tensor([1.0]), torch.zeros(v.D, 1), torch.tensor([theta_neg * v.T0]))
    assert ok.item() > 0 and bad.item() < 0
