"""Shared helpers of the GPU tests: run a workload through liblbm and through
the oracle on identical seeded inputs."""
import numpy as np
import torch

from oracle import equilibrium as oeq, lbm as olbm, velocity_sets as ovs

MODELS = {"D2Q33": (2, 33), "D3Q95": (3, 95)}


def gpu_available():
    return torch.cuda.is_available()


def new_sim(model, extent, omega, precision="fp64", rho0=1.0):
    from paper_1303_4624_amd import Simulation
    return Simulation(model, extent, omega, precision=precision, rho0=rho0)


def gpu_run(model, extent, omega, rho, U, theta, steps, precision="fp64", rho0=1.0):
    sim = new_sim(model, extent, omega, precision, rho0)
    sim.init_fields(rho, U, theta * sim.T0)
    sim.step(steps)
    r, u, t = sim.moments()
    torch.cuda.synchronize()
    out = (r.cpu().numpy(), u.cpu().numpy(), t.cpu().numpy(), sim.T0)
    sim.close()
    return out


def oracle_run(model, rho, U, theta, steps, omega):
    v = ovs.velocity_set(model)
    f = olbm.init_populations(v, rho, U, theta * v.T0)
    f = olbm.run(v, f, omega, steps)
    r, u, t = oeq.moments(v, f)
    return r.numpy(), u.numpy(), t.numpy(), f


def rel_errors(gpu, ora, T0):
    """max |d rho| / max rho, max |d U| / max |U|, max |d T| / T0."""
    r1, u1, t1 = gpu[:3]
    r2, u2, t2 = ora[:3]
    er = np.max(np.abs(r1 - r2)) / np.max(np.abs(r2))
    umax = max(np.max(np.abs(u2)), 1e-300)
    eu = np.max(np.abs(u1 - u2)) / umax
    et = np.max(np.abs(t1 - t2)) / T0
    return er, eu, et
