"""The lattice Boltzmann update rule and what is computed around it.

Test infrastructure: see the package docstring.

Update rule (the paragraph that opens the method):
    f_i(x + V_i dt, t + dt) = (1 - omega) f_i(x, t) + omega f_i^eq(x, t)
with V_i dt = e_i on the lattice and every axis periodic.  The oracle applies
it literally: collide at every node, then move each population i by e_i with
``torch.roll`` (which wraps by a true modulo, so displacements larger than an
extent are handled).  This is the same map as gathering from x - e_i.

Initial state: f = f^eq(rho, U, T) of the given fields, which is how the
paper's shock-tube experiment states its homogeneous initial conditions.

End conditions of the shock tube (results section): the two end planes
normal to the tube axis (the slowest grid axis) carry the fixed states C_L
and C_R while the side directions stay periodic.  Read here as reservoirs:
after every update the populations of the first n_lo and the last n_hi
planes are replaced by f^eq of the fixed state.  Since a node gathers from
up to max|e_z| planes away, holding that many planes at each end keeps the
periodic seam closed.
"""
from __future__ import annotations

from typing import Tuple

import torch

from .equilibrium import feq, moments
from .velocity_sets import VelocitySet


def to_tensor(a) -> torch.Tensor:
    return torch.as_tensor(a, dtype=torch.float64)


def init_populations(vs: VelocitySet, rho, U, T) -> torch.Tensor:
    """f(x, 0) = f^eq(rho, U, T) at every node."""
    return feq(vs, to_tensor(rho), to_tensor(U), to_tensor(T))


def collide(vs: VelocitySet, f: torch.Tensor, omega) -> torch.Tensor:
    """Post-collision populations (1 - omega) f_i + omega f_i^eq(rho, U, T of f)."""
    rho, U, T = moments(vs, f)
    return (1.0 - omega) * f + omega * feq(vs, rho, U, T)


def stream(vs: VelocitySet, post: torch.Tensor) -> torch.Tensor:
    """Move population i by e_i: out_i(x) = post_i(x - e_i), periodic.

    Grid axes of ``post`` are (..., y, x) after the population axis, so the
    displacement components are applied in reverse order.
    """
    D = vs.D
    dims = tuple(range(1, D + 1))
    outs = []
    for i in range(vs.Q):
        shifts = tuple(int(s) for s in reversed(vs.e[i].tolist()))
        outs.append(torch.roll(post[i], shifts=shifts, dims=tuple(d - 1 for d in dims)))
    return torch.stack(outs)


def hold_planes(vs: VelocitySet, f: torch.Tensor, n_lo: int, n_hi: int,
                state_lo=None, state_hi=None) -> torch.Tensor:
    """f with planes [0, n_lo) and [L - n_hi, L) of the slowest grid axis set
    to f^eq(state); a state is (rho, U_x, U_y[, U_z], T)."""
    D = vs.D
    f = f.clone()
    L = f.shape[1]
    plane = f.shape[2:]
    for lo, hi, st in ((0, n_lo, state_lo), (L - n_hi, L, state_hi)):
        if hi <= lo:
            continue
        st = [float(x) for x in st]
        rho = torch.full(plane, st[0], dtype=torch.float64)
        U = torch.stack([torch.full(plane, st[1 + a], dtype=torch.float64) for a in range(D)])
        T = torch.full(plane, st[D + 1], dtype=torch.float64)
        f[:, lo:hi] = feq(vs, rho, U, T).unsqueeze(1)
    return f


def step(vs: VelocitySet, f: torch.Tensor, omega, hold=None) -> torch.Tensor:
    """One update; ``hold`` = (n_lo, n_hi, state_lo, state_hi) applies the
    fixed end planes afterwards."""
    f = stream(vs, collide(vs, f, omega))
    if hold is not None:
        f = hold_planes(vs, f, *hold)
    return f


def run(vs: VelocitySet, f: torch.Tensor, omega, n: int, hold=None) -> torch.Tensor:
    for _ in range(n):
        f = step(vs, f, omega, hold)
    return f


def conserved(vs: VelocitySet, f: torch.Tensor) -> torch.Tensor:
    """Global mass, momentum (D components) and energy sum_x sum_i f_i |e_i|^2 / 2."""
    e = to_tensor(vs.e)
    mass = f.sum()
    mom = torch.einsum("qa,q...->a", e, f)
    energy = 0.5 * torch.einsum("q,q...->", (e * e).sum(1), f)
    return torch.cat([mass.reshape(1), mom, energy.reshape(1)])


def density_loss(rho_final: torch.Tensor, rho_target: torch.Tensor) -> torch.Tensor:
    """L = sum_x (rho_n(x) - rho*(x))^2."""
    return ((rho_final - rho_target) ** 2).sum()


def forward_density(vs: VelocitySet, rho0, U0, T_init: torch.Tensor, omega, n: int,
                    hold=None) -> torch.Tensor:
    f = feq(vs, to_tensor(rho0), to_tensor(U0), T_init)
    f = run(vs, f, omega, n, hold)
    return f.sum(0)


def loss_and_grad(vs: VelocitySet, rho0, U0, T_init, omega: float, n: int,
                  rho_target, hold=None) -> Tuple[float, torch.Tensor, float]:
    """Loss and its gradient with respect to the initial temperature field and
    omega, by float64 reverse-mode automatic differentiation through the
    initial equilibrium and n update steps (independent of any hand-written
    adjoint); `hold` as for step (end planes reset to a fixed equilibrium)."""
    T = to_tensor(T_init).clone().requires_grad_(True)
    w = torch.tensor(float(omega), dtype=torch.float64, requires_grad=True)
    rho_n = forward_density(vs, rho0, U0, T, w, n, hold)
    L = density_loss(rho_n, to_tensor(rho_target))
    L.backward()
    return float(L.detach()), T.grad.detach(), float(w.grad)
