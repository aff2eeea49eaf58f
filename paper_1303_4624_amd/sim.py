"""Simulation: a context of liblbm with its device buffers held as torch tensors.

PyTorch supplies device memory and the stream; every step of the method runs
in the library's HIP kernels through the C ABI.
"""
from __future__ import annotations

from typing import Optional, Sequence, Tuple

import numpy as np
import torch

from . import _lib as L

# The 4th-order models of Tables 2 and 3, and the lower-order (m = 2) 3D
# 19- and 15-velocity sets built by the same construction.
MODELS = {"D2Q33": (2, 33), "D3Q95": (3, 95), "D3Q19": (3, 19), "D3Q15": (3, 15)}
PRECISIONS = {"fp64": L.LBM_FP64, "fp32s": L.LBM_FP32_SHIFTED}
STREAMING = {"ab": L.LBM_STREAM_AB, "aa": L.LBM_STREAM_AA}


def _dev_bytes(nbytes: int, device) -> torch.Tensor:
    # float64 elements keep the base 8-byte aligned; the caching allocator
    # hands out 512-byte aligned blocks.
    t = torch.empty((nbytes + 7) // 8, dtype=torch.float64, device=device)
    if t.data_ptr() % 256:
        raise RuntimeError("device allocation is not 256-byte aligned")
    return t


class Simulation:
    """One periodic lattice with a supported velocity set.

    model     : "D2Q33", "D3Q95" (4th order), "D3Q19" or "D3Q15" (2nd order)
    extent    : (nx, ny[, nz])
    omega     : relaxation frequency
    precision : "fp64" or "fp32s" (float32 deviations from w_i rho0)
    streaming : "ab" (two population buffers) or "aa" (one buffer, in place)
    """

    def __init__(self, model: str, extent: Sequence[int], omega: float,
                 precision: str = "fp64", rho0: float = 1.0, device="cuda",
                 stream: Optional[torch.cuda.Stream] = None, streaming: str = "ab"):
        if model not in MODELS:
            raise ValueError(f"unknown model {model}")
        self.model = model
        self.D, self.Q = MODELS[model]
        self.extent = tuple(int(n) for n in extent)
        if len(self.extent) != self.D:
            raise ValueError("extent must have D entries")
        self.N = int(np.prod(self.extent))
        self.precision = precision
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.e, self.w, self.c = L.lbm_velocity_set(self.D, self.Q)
        self.T0 = 1.0 / (2.0 * self.c * self.c)
        self.omega = float(omega)
        self.ctx = L.lbm_create(self.D, self.Q, self.e, self.w, self.c, self.extent, omega,
                                PRECISIONS[precision], rho0, self.stream.cuda_stream)
        if streaming not in STREAMING:
            raise ValueError(f"unknown streaming scheme {streaming}")
        self.streaming = streaming
        L.lbm_set_streaming(self.ctx, STREAMING[streaming])
        pop, scr = L.lbm_workspace_bytes(self.ctx)
        self.pop_bytes = pop
        self._fa = _dev_bytes(pop, self.device)
        self._fb = _dev_bytes(pop, self.device) if streaming == "ab" else None
        self._scratch = _dev_bytes(scr, self.device)
        with torch.cuda.device(self.device):
            L.lbm_bind(self.ctx, self._fa, self._fb, self._scratch)
        self.block_order = 0

    # -- shapes --------------------------------------------------------
    @property
    def grid_shape(self) -> Tuple[int, ...]:
        return tuple(reversed(self.extent))

    def _field(self, x, comps: int = 1) -> torch.Tensor:
        t = torch.as_tensor(x, dtype=torch.float64, device=self.device).contiguous()
        want = (self.N * comps,)
        if t.numel() != want[0]:
            raise ValueError(f"field has {t.numel()} values, expected {want[0]}")
        return t

    # -- stream ordering ------------------------------------------------
    # The library runs on self.stream; tensors are made and consumed on the
    # caller's current stream.  Each call first makes self.stream wait for
    # the current stream (inputs written there), then the current stream
    # wait for self.stream (outputs read there), and records every tensor
    # handed to the library on self.stream so that the caching allocator does
    # not reuse its memory while a kernel may still use it.
    def _call(self, fn, *args, tensors=()):
        cur = torch.cuda.current_stream(self.device)
        other = cur.cuda_stream != self.stream.cuda_stream
        if other:
            self.stream.wait_stream(cur)
        res = fn(*args)
        if other:
            for t in tensors:
                if isinstance(t, torch.Tensor) and t.is_cuda:
                    t.record_stream(self.stream)
            cur.wait_stream(self.stream)
        return res

    # -- C ABI wrappers -------------------------------------------------
    def init_fields(self, rho, U, T) -> None:
        r, u, t = self._field(rho), self._field(U, self.D), self._field(T)
        self._call(L.lbm_init_fields, self.ctx, r, u, t, tensors=(r, u, t))

    def set_populations(self, f) -> None:
        t = self._field(f, self.Q)
        self._call(L.lbm_set_populations, self.ctx, t, tensors=(t,))

    def get_populations(self) -> torch.Tensor:
        out = torch.empty((self.Q,) + self.grid_shape, dtype=torch.float64, device=self.device)
        self._call(L.lbm_get_populations, self.ctx, out, tensors=(out,))
        return out

    def step(self, n: int = 1) -> None:
        self._call(L.lbm_step, self.ctx, n)

    def tune_step(self, n: int) -> int:
        """step(n), bit for bit, timing on the way the two block orders of
        the forward step on these buffers and keeping the faster; returns
        the order kept (0: contiguous rows per XCD, 1: slabs in turn).
        Synchronises the library's stream when it tunes (n >= 4, two-buffer
        streaming)."""
        self.block_order = self._call(L.lbm_tune_step, self.ctx, n)
        return self.block_order

    def set_block_order(self, order: int) -> None:
        """Set the forward steps' block order (0 or 1) without timing."""
        L.lbm_set_block_order(self.ctx, order)
        self.block_order = order

    def moments(self):
        rho = torch.empty(self.grid_shape, dtype=torch.float64, device=self.device)
        U = torch.empty((self.D,) + self.grid_shape, dtype=torch.float64, device=self.device)
        T = torch.empty(self.grid_shape, dtype=torch.float64, device=self.device)
        self._call(L.lbm_moments, self.ctx, rho, U, T, tensors=(rho, U, T))
        return rho, U, T

    def conservation(self) -> np.ndarray:
        return self._call(L.lbm_conservation, self.ctx, self.D)

    def stream_copy(self, n: int = 1) -> None:
        """Measurement reference: n plain streaming copies of the state into
        the other population buffer (the bytes of a step, no gather or
        arithmetic); the state is unchanged."""
        self._call(L.lbm_stream_copy, self.ctx, n)

    def set_fixed_planes(self, n_lo: int, n_hi: int, state_lo=None, state_hi=None) -> None:
        """Hold the first n_lo / last n_hi planes of the slowest axis at
        f^eq(state) after every step; a state is (rho, U_x, U_y[, U_z], T)."""
        for s, n in ((state_lo, n_lo), (state_hi, n_hi)):
            if n and (s is None or len(s) != self.D + 2):
                raise ValueError(f"a held state needs D + 2 = {self.D + 2} values")
        L.lbm_set_fixed_planes(self.ctx, n_lo, n_hi, state_lo, state_hi)

    def set_graph_steps(self, steps: int) -> None:
        """Replay step() in HIP graphs of `steps` (even) steps; 0 turns it off.
        Needs a non-default stream (pass ``stream=torch.cuda.Stream()``; the
        calls order themselves against the caller's current stream)."""
        L.lbm_set_graph_steps(self.ctx, steps)

    def set_omega(self, omega: float) -> None:
        L.lbm_set_omega(self.ctx, omega)
        self.omega = float(omega)

    def run_checkpointed(self, n: int, k: int, keep: int = 1) -> torch.Tensor:
        """n steps with a snapshot every k steps; the last `keep` segments also
        keep their step moments (keep >= ceil(n/k): no recomputation later)."""
        nb = L.lbm_checkpoint_bytes(self.ctx, n, k, keep)
        ck = _dev_bytes(nb, self.device)
        self._call(L.lbm_run_checkpointed, self.ctx, n, k, keep, ck, nb, tensors=(ck,))
        return ck

    def restore_checkpoint(self, n: int, k: int, ckpt: torch.Tensor, slot: int,
                           keep: int = 1) -> None:
        """Continue from snapshot `slot` of run_checkpointed(n, k, keep) (the
        state at t = slot*k; slot = ceil(n/k): the final state)."""
        self._call(L.lbm_restore_checkpoint, self.ctx, n, k, keep, ckpt, ckpt.numel() * 8, slot,
                   tensors=(ckpt,))

    def adjoint(self, n: int, k: int, ckpt: torch.Tensor, rho_init, U_init, T_init,
                dL_drho_final, want_T: bool = True, want_omega: bool = True,
                workspace: Optional[torch.Tensor] = None, keep: int = 1):
        """(dL/dT_init as a grid-shaped tensor or None, dL/domega or None)."""
        wsb = L.lbm_adjoint_workspace_bytes(self.ctx, n, k, keep)
        if workspace is None or workspace.numel() * 8 < wsb:
            workspace = _dev_bytes(wsb, self.device)
        r, u, t = self._field(rho_init), self._field(U_init, self.D), self._field(T_init)
        g = self._field(dL_drho_final)
        dT = torch.empty(self.grid_shape, dtype=torch.float64, device=self.device) if want_T else None
        dw = self._call(L.lbm_adjoint, self.ctx, n, k, keep, ckpt, ckpt.numel() * 8, r, u, t, g,
                        workspace, wsb, dT, want_omega, tensors=(ckpt, r, u, t, g, workspace, dT))
        return dT, dw

    def close(self) -> None:
        if getattr(self, "ctx", None):
            L.lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
