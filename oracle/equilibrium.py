"""Equilibrium and moments (Maxwellian and dimensionless variables; Formula (1);
polynomial equilibria f_i^eq = w_i P^(N)(v_i) with the m-th order Hermite
expansion, N = m: 4 for the models of Tables 2 and 3, 2 for the lower-order
3D 19- and 15-velocity sets).

Test infrastructure: see the package docstring.

Units.  Lattice units with dx = dt = 1, so the particle velocity of
population i is V_i = e_i (integer).  Temperatures are T = k_B T / m_g in
cells^2/step^2; the reference temperature is T0 = 1/(2c^2) and the lattice
sound-speed scale is c_s = sqrt(T0).  The Hermite variable is xi = V / c_s
(the paper's v scaled by sqrt(2)), u_hat = U / c_s and d = theta - 1 with
theta = T / T0.

Equilibrium.  The paper gives the form f_i^eq = w_i P^(4)(v_i) but does not
print the polynomial; it states that an m-th order model needs the m-th order
Hermite expansion f_HE^eq of the Maxwellian.  Here that expansion is written
out as its definition, the sum over n <= 4 of (1/n!) a^(n) : H^(n)(xi) with
the tensor Hermite polynomials H^(n) of the Gaussian weight exp(-xi^2/2) and
the Hermite coefficients a^(n) of the Maxwellian, in full tensor form
(D^n components per order, contracted with einsum).  Tests pin the
coefficients against numerical Gauss-Hermite projection of the Maxwellian and
the resulting discrete moments against the Maxwellian's moments of every
order <= 4.
"""
from __future__ import annotations

import torch

from .velocity_sets import VelocitySet


def _delta(D, dtype=torch.float64):
    return torch.eye(D, dtype=dtype)


def hermite_tensors(xi: torch.Tensor):
    """Tensor Hermite polynomials H^(0..4) at points xi (P, D).

    H0 = 1, H1_a = xi_a, H2_ab = xi_a xi_b - d_ab,
    H3_abc = xi_a xi_b xi_c - (xi_a d_bc + xi_b d_ac + xi_c d_ab),
    H4_abcd = xi_a xi_b xi_c xi_d - (six terms xi xi d) + (three terms d d).
    """
    P, D = xi.shape
    d = _delta(D, xi.dtype)
    ein = torch.einsum
    H0 = torch.ones(P, dtype=xi.dtype)
    H1 = xi
    H2 = ein("pa,pb->pab", xi, xi) - d
    H3 = (ein("pa,pb,pc->pabc", xi, xi, xi)
          - ein("pa,bc->pabc", xi, d) - ein("pb,ac->pabc", xi, d) - ein("pc,ab->pabc", xi, d))
    xx = ein("pa,pb->pab", xi, xi)
    H4 = (ein("pa,pb,pc,pd->pabcd", xi, xi, xi, xi)
          - ein("pab,cd->pabcd", xx, d) - ein("pac,bd->pabcd", xx, d) - ein("pad,bc->pabcd", xx, d)
          - ein("pbc,ad->pabcd", xx, d) - ein("pbd,ac->pabcd", xx, d) - ein("pcd,ab->pabcd", xx, d)
          + ein("ab,cd->abcd", d, d) + ein("ac,bd->abcd", d, d) + ein("ad,bc->abcd", d, d))
    return H0, H1, H2, H3, H4


def maxwell_hermite_coefficients(rho: torch.Tensor, u_hat: torch.Tensor, dth: torch.Tensor):
    """Hermite coefficients a^(0..4) of the Maxwellian at M points.

    rho (M,), u_hat (M, D), dth = theta - 1 (M,).  With u = u_hat:
    a0 = rho, a1 = rho u, a2 = rho (u u + dth I),
    a3 = rho (u u u + dth [u I]_3), a4 = rho (u u u u + dth [u u I]_6 + dth^2 [I I]_3).
    """
    M, D = u_hat.shape
    d = _delta(D, u_hat.dtype)
    ein = torch.einsum
    u = u_hat
    uu = ein("ma,mb->mab", u, u)
    a0 = rho
    a1 = rho[:, None] * u
    a2 = rho[:, None, None] * (uu + dth[:, None, None] * d)
    uI3 = ein("ma,bc->mabc", u, d) + ein("mb,ac->mabc", u, d) + ein("mc,ab->mabc", u, d)
    a3 = rho[:, None, None, None] * (ein("ma,mb,mc->mabc", u, u, u) + dth[:, None, None, None] * uI3)
    uuI6 = (ein("mab,cd->mabcd", uu, d) + ein("mac,bd->mabcd", uu, d) + ein("mad,bc->mabcd", uu, d)
            + ein("mbc,ad->mabcd", uu, d) + ein("mbd,ac->mabcd", uu, d) + ein("mcd,ab->mabcd", uu, d))
    II3 = ein("ab,cd->abcd", d, d) + ein("ac,bd->abcd", d, d) + ein("ad,bc->abcd", d, d)
    s = dth[:, None, None, None, None]
    a4 = rho[:, None, None, None, None] * (ein("ma,mb,mc,md->mabcd", u, u, u, u) + s * uuI6 + s * s * II3)
    return a0, a1, a2, a3, a4


def feq(vs: VelocitySet, rho: torch.Tensor, U: torch.Tensor, T: torch.Tensor,
        order: int = None) -> torch.Tensor:
    """Discrete equilibrium f_i^eq = w_i sum_{n<=N} (1/n!) a^(n) : H^(n)(xi_i).

    N = `order`, by default the model's order of accuracy m (N = m, as the
    paragraph after Formula (5) asks for N >= m): the Hermite sum is simply
    truncated after order N.  rho, T have the grid shape; U has shape
    (D, *grid).  Returns (Q, *grid).
    """
    N = vs.m if order is None else order
    if not 0 <= N <= 4:
        raise ValueError("equilibrium order must be 0..4")
    rho = torch.as_tensor(rho, dtype=torch.float64)
    U = torch.as_tensor(U, dtype=torch.float64)
    T = torch.as_tensor(T, dtype=torch.float64)
    grid = rho.shape
    D = vs.D
    cs = vs.T0 ** 0.5
    r = rho.reshape(-1)
    u = (U.reshape(D, -1) / cs).T.contiguous()
    dth = T.reshape(-1) / vs.T0 - 1.0
    xi = torch.as_tensor(vs.e, dtype=torch.float64) / cs
    H = hermite_tensors(xi)
    A = maxwell_hermite_coefficients(r, u, dth)
    fact = (1.0, 1.0, 2.0, 6.0, 24.0)
    Q = xi.shape[0]
    acc = None
    for n in range(N + 1):
        Hn = H[n].reshape(Q, -1)           # (Q, D^n)
        An = A[n].reshape(r.shape[0], -1)  # (M, D^n)
        term = (Hn @ An.T) / fact[n]        # (Q, M)
        acc = term if acc is None else acc + term
    w = torch.as_tensor(vs.w, dtype=torch.float64)
    return (w[:, None] * acc).reshape((Q,) + tuple(grid))


def moments(vs: VelocitySet, f: torch.Tensor):
    """rho = sum_i f_i, U = sum_i f_i e_i / rho, T = (sum_i f_i |e_i|^2 / rho - |U|^2) / D.

    The Maxwellian of the update rule has variance k_B T / m_g per axis, so
    these are the density, flow velocity and temperature it is built from.
    """
    e = torch.as_tensor(vs.e, dtype=torch.float64)
    rho = f.sum(0)
    j = torch.einsum("qa,q...->a...", e, f)
    U = j / rho
    e2 = (e * e).sum(1)
    E2 = torch.einsum("q,q...->...", e2, f)
    T = (E2 / rho - (U * U).sum(0)) / vs.D
    return rho, U, T


def min_feq_ratio(vs: VelocitySet, rho, U, T) -> torch.Tensor:
    """min_i f_i^eq / (w_i rho): negative where the equilibrium loses positivity."""
    f = feq(vs, rho, U, T)
    w = torch.as_tensor(vs.w, dtype=torch.float64)
    shape = (-1,) + (1,) * rho.dim()
    return (f / (w.reshape(shape) * rho)).min(0).values
