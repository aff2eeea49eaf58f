"""torch.autograd.Function around the checkpointed forward run and the
hand-written adjoint of liblbm.

    rho_n = LBMFunction.apply(T_init, omega, sim, rho_init, U_init, n, k, keep)

Forward: f^0 = f^eq(rho_init, U_init, T_init), n update steps with a
checkpoint every k steps (the last `keep` segments also keep their step
moments), returns the final density (grid-shaped float64).
Backward: ``lbm_adjoint`` (recomputation per segment + transposed steps)
returns dL/dT_init and dL/domega.  rho_init and U_init are constants.
"""
from __future__ import annotations

import torch

from .sim import Simulation


class LBMFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, T_init: torch.Tensor, omega: torch.Tensor, sim: Simulation,
                rho_init: torch.Tensor, U_init: torch.Tensor, n: int, k: int, keep: int):
        sim.set_omega(float(omega))
        sim.init_fields(rho_init, U_init, T_init)
        ckpt = sim.run_checkpointed(n, k, keep)
        ctx.keep = keep
        rho, _, _ = sim.moments()
        ctx.sim = sim
        ctx.n, ctx.k = n, k
        ctx.omega = float(omega)
        ctx.save_for_backward(T_init, rho_init, U_init)
        ctx.ckpt = ckpt
        return rho

    @staticmethod
    def backward(ctx, grad_rho: torch.Tensor):
        T_init, rho_init, U_init = ctx.saved_tensors
        sim: Simulation = ctx.sim
        if sim.omega != ctx.omega:
            sim.set_omega(ctx.omega)
        want_T = ctx.needs_input_grad[0]
        want_w = ctx.needs_input_grad[1]
        dT, dw = sim.adjoint(ctx.n, ctx.k, ctx.ckpt, rho_init, U_init, T_init,
                             grad_rho.to(torch.float64).contiguous(), want_T=want_T,
                             want_omega=want_w, keep=ctx.keep)
        ctx.ckpt = None
        gw = torch.tensor(dw, dtype=torch.float64, device=grad_rho.device) if want_w else None
        return dT, gw, None, None, None, None, None, None
