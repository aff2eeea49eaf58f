"""Seeded synthetic inputs shared by the CPU oracle, the tests and the benchmark.

This module holds workload definitions and random-field generators only.  It
contains none of the lattice Boltzmann arithmetic (no velocity sets, weights,
equilibria, moments or lattice temperature): temperatures are returned as the
dimensionless ratio theta = T / T0, and each consumer converts them with its
own T0.

Array conventions (shared by every consumer):
  * 3D scalar fields have shape (nz, ny, nx), 2D ones (ny, nx); x is the
    fastest (last) axis, C order.
  * Vector fields have shape (D, *grid) with components ordered (x, y[, z]).
  * Grid extents are written (nx, ny[, nz]).

The workloads stand in for the paper's only experiment, a shock tube with
homogeneous left/right states (Riemann problem), and for smooth thermal flows
at throughput sizes.  The paper uses no public dataset.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, Tuple

import numpy as np

__all__ = [
    "Workload",
    "WORKLOADS",
    "grid_shape",
    "smooth_noise",
    "smooth_ic",
    "riemann_ic",
    "double_riemann_ic",
    "tube_ic",
    "tube_states",
    "tiled_smooth_ic",
    "workload_ic",
    "fd_direction",
    "target_theta",
]


@dataclass(frozen=True)
class Workload:
    """One named workload: model, periodic grid, relaxation, step count, IC recipe."""

    name: str
    model: str                      # "D2Q33" or "D3Q95"
    extent: Tuple[int, ...]         # (nx, ny[, nz])
    omega: float
    steps: int
    ic: str                         # "double_riemann", "riemann", "smooth"
    precisions: Tuple[str, ...]     # "fp64", "fp32s"
    checkpoint_every: int = 0
    extra: Dict[str, float] = field(default_factory=dict)

    @property
    def cells(self) -> int:
        return int(np.prod(self.extent))


WORKLOADS: Dict[str, Workload] = {
    w.name: w
    for w in [
        # 2D 33-velocity model, double Riemann problem along x.
        Workload("d2q33_128x4_riemann2", "D2Q33", (128, 4), 1.0, 500,
                 "double_riemann", ("fp64",)),
        # 3D 95-velocity model, one Riemann problem along x.
        Workload("d3q95_512x4x4_riemann", "D3Q95", (512, 4, 4), 1.2, 400,
                 "riemann", ("fp64",)),
        # Smooth random thermal flow, FP32-shifted and FP64.
        Workload("d3q95_256c_smooth", "D3Q95", (256, 256, 256), 1.5, 1000,
                 "smooth", ("fp32s", "fp64")),
        # Throughput / roofline run.
        Workload("d3q95_384c_smooth", "D3Q95", (384, 384, 384), 1.8, 500,
                 "smooth", ("fp32s",)),
        # The shock tube of the results section: 11 x 11 x 800 nodes, the left
        # half (z < 400) at rho = p = 4, the right half at rho = p = 1, theta = 1
        # and at rest in both; the end planes held at those states
        # (extra["hold"] planes at each end), sides periodic, omega = 1.5.
        Workload("d3q95_11x11x800_tube", "D3Q95", (11, 11, 800), 1.5, 120,
                 "tube", ("fp64", "fp32s"), extra={"hold": 5}),
        # The same tube for the 2D model along y.
        Workload("d2q33_11x800_tube", "D2Q33", (11, 800), 1.5, 120,
                 "tube", ("fp64", "fp32s"), extra={"hold": 4}),
        # Forward + adjoint with checkpoints every 20 steps.
        Workload("d3q95_128c_adjoint", "D3Q95", (128, 128, 128), 1.4, 200,
                 "smooth", ("fp32s",), checkpoint_every=20),
    ]
}


def grid_shape(extent) -> Tuple[int, ...]:
    """Array shape (…, ny, nx) of a grid with extents (nx, ny[, nz])."""
    return tuple(int(n) for n in reversed(tuple(extent)))


def smooth_noise(extent, seed: int, kmax: float = 8.0) -> np.ndarray:
    """Gaussian noise low-pass filtered to integer wavenumbers |k| <= kmax.

    Standard normal values from ``numpy.random.default_rng(seed)`` on the
    grid, real FFT, every mode with Euclidean integer wavenumber above kmax
    and the k = 0 mode set to zero, inverse FFT, then scaled to unit RMS.
    Returns float64 of shape ``grid_shape(extent)``.
    """
    shape = grid_shape(extent)
    rng = np.random.default_rng(seed)
    g = rng.standard_normal(shape)
    spec = np.fft.rfftn(g)
    k2 = np.zeros(spec.shape)
    for ax, n in enumerate(shape):
        if ax == len(shape) - 1:
            k = np.fft.rfftfreq(n, d=1.0 / n)
        else:
            k = np.fft.fftfreq(n, d=1.0 / n)
        sh = [1] * len(shape)
        sh[ax] = k.size
        k2 = k2 + k.reshape(sh) ** 2
    spec[k2 > kmax * kmax] = 0.0
    spec.flat[0] = 0.0
    out = np.fft.irfftn(spec, s=shape, axes=tuple(range(len(shape))))
    rms = np.sqrt(np.mean(out * out))
    if rms > 0:
        out /= rms
    return out


def smooth_ic(extent, seeds=(1, 2, 3, 4, 5), amp_rho=0.01, amp_u=0.02,
              amp_theta=0.01):
    """rho = 1 + amp_rho g1, U_a = amp_u g_(2+a), theta = 1 + amp_theta g_last.

    U is in cells per step.  One seed per field: seeds[0] for rho,
    seeds[1..D] for the velocity components, seeds[-1] for theta.
    """
    D = len(extent)
    if len(seeds) < D + 2:
        raise ValueError("need D + 2 seeds")
    rho = 1.0 + amp_rho * smooth_noise(extent, seeds[0])
    U = np.stack([amp_u * smooth_noise(extent, seeds[1 + a]) for a in range(D)])
    theta = 1.0 + amp_theta * smooth_noise(extent, seeds[D + 1])
    return rho, U, theta


def tiled_smooth_ic(extent, tile, **kw):
    """smooth_ic on the grid ``tile`` repeated periodically to ``extent``
    (each extent a multiple of the tile's); for grids too large to filter
    in one FFT on the host."""
    if any(e % t for e, t in zip(extent, tile)):
        raise ValueError("extent must be a multiple of tile")
    rho, U, th = smooth_ic(tile, **kw)
    reps = tuple(e // t for e, t in zip(reversed(extent), reversed(tile)))
    return (np.tile(rho, reps), np.tile(U, (1,) + reps), np.tile(th, reps))


def _x_index(extent) -> np.ndarray:
    shape = grid_shape(extent)
    return np.broadcast_to(np.arange(extent[0]), shape)


def riemann_ic(extent, x_split, left, right):
    """Two homogeneous states at rest: x < x_split gets ``left``, else ``right``.

    ``left`` and ``right`` are (rho, theta) pairs.
    """
    x = _x_index(extent)
    rho = np.where(x < x_split, left[0], right[0]).astype(np.float64)
    theta = np.where(x < x_split, left[1], right[1]).astype(np.float64)
    U = np.zeros((len(extent),) + rho.shape)
    return rho, U, theta


def tube_ic(extent, split, left, right):
    """Two homogeneous states at rest split along the slowest axis (z in 3D,
    y in 2D): index < split gets ``left``, else ``right``; (rho, theta) pairs."""
    shape = grid_shape(extent)
    z = np.broadcast_to(np.arange(extent[-1]).reshape((-1,) + (1,) * (len(extent) - 1)), shape)
    rho = np.where(z < split, left[0], right[0]).astype(np.float64)
    theta = np.where(z < split, left[1], right[1]).astype(np.float64)
    U = np.zeros((len(extent),) + rho.shape)
    return rho, U, theta


def tube_states(w: Workload):
    """(left, right) (rho, theta) pairs of a tube workload."""
    return (4.0, 1.0), (1.0, 1.0)


def double_riemann_ic(extent, x_lo, x_hi, outer, inner):
    """``inner`` state for x_lo <= x < x_hi, ``outer`` elsewhere; U = 0."""
    x = _x_index(extent)
    mid = (x >= x_lo) & (x < x_hi)
    rho = np.where(mid, inner[0], outer[0]).astype(np.float64)
    theta = np.where(mid, inner[1], outer[1]).astype(np.float64)
    U = np.zeros((len(extent),) + rho.shape)
    return rho, U, theta


def workload_ic(w: Workload, extent=None):
    """Initial (rho, U, theta) of a workload, optionally on another extent.

    A different extent keeps the recipe (for example a small replica of a
    smooth workload for the oracle).
    """
    ext = tuple(extent) if extent is not None else w.extent
    if w.ic == "double_riemann":
        nx = ext[0]
        return double_riemann_ic(ext, nx // 4, 3 * nx // 4, (1.0, 1.0), (0.8, 0.9))
    if w.ic == "riemann":
        return riemann_ic(ext, ext[0] // 2, (1.0, 1.0), (0.5, 0.8))
    if w.ic == "smooth":
        return smooth_ic(ext)
    if w.ic == "tube":
        lo, hi = tube_states(w)
        return tube_ic(ext, ext[-1] // 2, lo, hi)
    raise ValueError(w.ic)


def fd_direction(extent, k: int) -> np.ndarray:
    """k-th finite-difference direction: unit-RMS smooth field, seed 100 + k."""
    return smooth_noise(extent, 100 + k)


def target_theta(extent, amp_theta=0.01) -> np.ndarray:
    """Temperature ratio of the run that produces a gradient test's target (seed 6)."""
    return 1.0 + amp_theta * smooth_noise(extent, 6)
