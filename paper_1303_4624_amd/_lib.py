"""ctypes binding of liblbm.so with the names of the C ABI (include/lbm.h).

Argument marshalling only: every computation runs in the library's HIP
kernels.  Device buffers are passed as integer addresses (e.g.
``tensor.data_ptr()``) and streams as ``hipStream_t`` handles
(``torch.cuda.current_stream().cuda_stream``).  A non-zero status raises
:class:`LBMError`.  If the library is not built the first call raises
``RuntimeError`` -- there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence, Tuple

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "liblbm.so")

LBM_OK = 0
LBM_E_INVALID = -1
LBM_E_UNSUPPORTED = -2
LBM_E_DEVICE = -3
LBM_E_STATE = -4
LBM_E_NONFINITE = -5
LBM_FP64 = 0
LBM_FP32_SHIFTED = 1
LBM_STREAM_AB = 0
LBM_STREAM_AA = 1
LBM_MAX_Q = 95

EXPORTED = [
    "lbm_velocity_set", "lbm_equation_count", "lbm_model_build", "lbm_create", "lbm_workspace_bytes", "lbm_bind", "lbm_init_fields",
    "lbm_set_populations", "lbm_get_populations", "lbm_step", "lbm_tune_step", "lbm_set_block_order", "lbm_moments",
    "lbm_conservation", "lbm_conservation_noalloc", "lbm_stream_copy", "lbm_set_fixed_planes", "lbm_set_streaming", "lbm_set_graph_steps",
    "lbm_set_omega", "lbm_checkpoint_bytes", "lbm_run_checkpointed", "lbm_restore_checkpoint",
    "lbm_adjoint_workspace_bytes", "lbm_adjoint", "lbm_destroy", "lbm_status_str",
    "lbm_last_error",
]


class LBMError(RuntimeError):
    def __init__(self, status: int, func: str, detail: str):
        self.status = status
        super().__init__(f"{func}: {_status_str(status)} ({status}): {detail}")


_lib: Optional[ctypes.CDLL] = None
_c = ctypes
_vp = ctypes.c_void_p
_sz = ctypes.c_size_t
_pd = ctypes.POINTER(ctypes.c_double)
_pi32 = ctypes.POINTER(ctypes.c_int32)
_pi64 = ctypes.POINTER(ctypes.c_int64)
_psz = ctypes.POINTER(ctypes.c_size_t)

_SIGS = {
    "lbm_velocity_set": (_c.c_int, [_c.c_int, _c.c_int, _pi32, _pd, _pd]),
    "lbm_equation_count": (_c.c_int, [_c.c_int, _c.c_int, ctypes.POINTER(_c.c_int)]),
    "lbm_model_build": (_c.c_int, [_c.c_int, _c.c_int, _c.c_int, _pi32, _pd, _c.c_double, _c.c_int,
                                   _pi32, _pi32, _pd, _pd, ctypes.POINTER(_c.c_int), _pd]),
    "lbm_create": (_c.c_int, [ctypes.POINTER(_vp), _c.c_int, _c.c_int, _pi32, _pd, _c.c_double,
                              _pi64, _c.c_double, _c.c_int, _c.c_double, _vp]),
    "lbm_workspace_bytes": (_c.c_int, [_vp, _psz, _psz]),
    "lbm_bind": (_c.c_int, [_vp, _vp, _vp, _vp]),
    "lbm_init_fields": (_c.c_int, [_vp, _vp, _vp, _vp]),
    "lbm_set_populations": (_c.c_int, [_vp, _vp]),
    "lbm_get_populations": (_c.c_int, [_vp, _vp]),
    "lbm_step": (_c.c_int, [_vp, _c.c_int]),
    "lbm_tune_step": (_c.c_int, [_vp, _c.c_int, _c.POINTER(_c.c_int)]),
    "lbm_set_block_order": (_c.c_int, [_vp, _c.c_int]),
    "lbm_moments": (_c.c_int, [_vp, _vp, _vp, _vp]),
    "lbm_conservation": (_c.c_int, [_vp, _pd]),
    "lbm_conservation_noalloc": (_c.c_int, [_vp, _pd]),
    "lbm_stream_copy": (_c.c_int, [_vp, _c.c_int]),
    "lbm_set_fixed_planes": (_c.c_int, [_vp, _c.c_int, _c.c_int, _pd, _pd]),
    "lbm_set_streaming": (_c.c_int, [_vp, _c.c_int]),
    "lbm_set_graph_steps": (_c.c_int, [_vp, _c.c_int]),
    "lbm_set_omega": (_c.c_int, [_vp, _c.c_double]),
    "lbm_checkpoint_bytes": (_c.c_int, [_vp, _c.c_int, _c.c_int, _c.c_int, _psz]),
    "lbm_run_checkpointed": (_c.c_int, [_vp, _c.c_int, _c.c_int, _c.c_int, _vp, _sz]),
    "lbm_restore_checkpoint": (_c.c_int, [_vp, _c.c_int, _c.c_int, _c.c_int, _vp, _sz,
                                          _c.c_int]),
    "lbm_adjoint_workspace_bytes": (_c.c_int, [_vp, _c.c_int, _c.c_int, _c.c_int, _psz]),
    "lbm_adjoint": (_c.c_int, [_vp, _c.c_int, _c.c_int, _c.c_int, _vp, _sz, _vp, _vp, _vp, _vp,
                               _vp, _sz, _vp, _pd]),
    "lbm_destroy": (_c.c_int, [_vp]),
    "lbm_status_str": (_c.c_char_p, [_c.c_int]),
    "lbm_last_error": (_c.c_char_p, [_vp]),
}


def library() -> ctypes.CDLL:
    """Load liblbm.so (once); raises RuntimeError if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_1303_4624_amd.build` "
                "(the HIP library is required; there is no CPU fallback)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _status_str(status: int) -> str:
    return library().lbm_status_str(status).decode()


def _check(status: int, func: str, ctx=None) -> None:
    if status != LBM_OK:
        detail = library().lbm_last_error(ctx).decode()
        raise LBMError(status, func, detail)


def _addr(x) -> Optional[int]:
    """Device address of a tensor-like (``data_ptr()``) or an int; None -> NULL."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return int(x.data_ptr())


def lbm_status_str(status: int) -> str:
    return _status_str(status)


def lbm_last_error(ctx=None) -> str:
    return library().lbm_last_error(ctx).decode()


def lbm_velocity_set(D: int, Q: int) -> Tuple[np.ndarray, np.ndarray, float]:
    """Canonical velocities e (Q, D) int32, weights w (Q,) and c, solved by the library."""
    e = np.zeros((Q, D), dtype=np.int32)
    w = np.zeros(Q, dtype=np.float64)
    c = ctypes.c_double(0.0)
    st = library().lbm_velocity_set(D, Q, e.ctypes.data_as(_pi32), w.ctypes.data_as(_pd),
                                    ctypes.byref(c))
    _check(st, "lbm_velocity_set")
    return e, w, float(c.value)


def lbm_equation_count(m: int, D: int) -> int:
    n = ctypes.c_int(0)
    _check(library().lbm_equation_count(int(m), int(D), ctypes.byref(n)), "lbm_equation_count")
    return n.value


def lbm_model_build(D: int, m: int, reps, c_guess: float, w_guess=None):
    """(e int32[Q, D], group int32[Q], w float64[Q], c, residual) of the model
    whose groups are the orbits of ``reps`` (int[G][D])."""
    reps = np.ascontiguousarray(reps, dtype=np.int32).reshape(-1, D)
    G = reps.shape[0]
    wg = None if w_guess is None else np.ascontiguousarray(w_guess, dtype=np.float64)
    if wg is not None and wg.size != G:
        raise ValueError("w_guess needs one value per group")
    cap = G * (48 if D == 3 else 8)
    e = np.zeros((cap, D), dtype=np.int32)
    grp = np.zeros(cap, dtype=np.int32)
    w = np.zeros(cap, dtype=np.float64)
    c, Q, res = ctypes.c_double(0), ctypes.c_int(0), ctypes.c_double(0)
    st = library().lbm_model_build(D, int(m), G, reps.ctypes.data_as(_pi32),
                                   None if wg is None else wg.ctypes.data_as(_pd),
                                   float(c_guess), cap, e.ctypes.data_as(_pi32),
                                   grp.ctypes.data_as(_pi32), w.ctypes.data_as(_pd),
                                   ctypes.byref(c), ctypes.byref(Q), ctypes.byref(res))
    _check(st, "lbm_model_build")
    q = Q.value
    return e[:q].copy(), grp[:q].copy(), w[:q].copy(), c.value, res.value


def lbm_create(D: int, Q: int, e, w, c: float, extent: Sequence[int], omega: float,
               precision: int, rho0: float = 1.0, stream: int = 0) -> int:
    e = np.ascontiguousarray(e, dtype=np.int32)
    w = np.ascontiguousarray(w, dtype=np.float64)
    ext = np.ascontiguousarray(extent, dtype=np.int64)
    if e.size != Q * D or w.size != Q or ext.size != D:
        raise ValueError("e must be (Q, D), w (Q,), extent (D,)")
    h = _vp()
    st = library().lbm_create(ctypes.byref(h), D, Q, e.ctypes.data_as(_pi32),
                              w.ctypes.data_as(_pd), float(c), ext.ctypes.data_as(_pi64),
                              float(omega), int(precision), float(rho0), stream or None)
    _check(st, "lbm_create")
    return h.value


def lbm_workspace_bytes(ctx) -> Tuple[int, int]:
    pop, scr = _sz(0), _sz(0)
    _check(library().lbm_workspace_bytes(ctx, ctypes.byref(pop), ctypes.byref(scr)),
           "lbm_workspace_bytes", ctx)
    return pop.value, scr.value


def lbm_bind(ctx, f_a, f_b, scratch) -> None:
    _check(library().lbm_bind(ctx, _addr(f_a), _addr(f_b), _addr(scratch)), "lbm_bind", ctx)


def lbm_init_fields(ctx, rho, U, T) -> None:
    _check(library().lbm_init_fields(ctx, _addr(rho), _addr(U), _addr(T)), "lbm_init_fields", ctx)


def lbm_set_populations(ctx, f) -> None:
    _check(library().lbm_set_populations(ctx, _addr(f)), "lbm_set_populations", ctx)


def lbm_get_populations(ctx, f) -> None:
    _check(library().lbm_get_populations(ctx, _addr(f)), "lbm_get_populations", ctx)


def lbm_step(ctx, n: int) -> None:
    _check(library().lbm_step(ctx, int(n)), "lbm_step", ctx)


def lbm_tune_step(ctx, n: int) -> int:
    """lbm_step(n) that times the two block orders of the forward step on
    the way and keeps the faster; returns the order kept (0 or 1)."""
    m = _c.c_int(0)
    _check(library().lbm_tune_step(ctx, int(n), _c.byref(m)), "lbm_tune_step", ctx)
    return m.value


def lbm_set_block_order(ctx, order: int) -> None:
    _check(library().lbm_set_block_order(ctx, int(order)), "lbm_set_block_order", ctx)


def lbm_moments(ctx, rho=None, U=None, T=None) -> None:
    _check(library().lbm_moments(ctx, _addr(rho), _addr(U), _addr(T)), "lbm_moments", ctx)


def lbm_conservation(ctx, D: int) -> np.ndarray:
    out = np.zeros(D + 2, dtype=np.float64)
    _check(library().lbm_conservation(ctx, out.ctypes.data_as(_pd)), "lbm_conservation", ctx)
    return out


def lbm_stream_copy(ctx, n: int) -> None:
    _check(library().lbm_stream_copy(ctx, int(n)), "lbm_stream_copy", ctx)


def lbm_conservation_noalloc(ctx, D: int) -> np.ndarray:
    out = np.zeros(D + 2, dtype=np.float64)
    _check(library().lbm_conservation_noalloc(ctx, out.ctypes.data_as(_pd)),
           "lbm_conservation_noalloc", ctx)
    return out


def lbm_set_fixed_planes(ctx, n_lo: int, n_hi: int, state_lo=None, state_hi=None) -> None:
    """state_* : sequences (rho, U_x, U_y[, U_z], T) or None where the count is 0."""
    def arr(s):
        return None if s is None else np.ascontiguousarray(s, dtype=np.float64)
    lo, hi = arr(state_lo), arr(state_hi)
    _check(library().lbm_set_fixed_planes(
        ctx, int(n_lo), int(n_hi), None if lo is None else lo.ctypes.data_as(_pd),
        None if hi is None else hi.ctypes.data_as(_pd)), "lbm_set_fixed_planes", ctx)


def lbm_set_streaming(ctx, scheme: int) -> None:
    _check(library().lbm_set_streaming(ctx, int(scheme)), "lbm_set_streaming", ctx)


def lbm_set_graph_steps(ctx, steps: int) -> None:
    _check(library().lbm_set_graph_steps(ctx, int(steps)), "lbm_set_graph_steps", ctx)


def lbm_set_omega(ctx, omega: float) -> None:
    _check(library().lbm_set_omega(ctx, float(omega)), "lbm_set_omega", ctx)


def lbm_checkpoint_bytes(ctx, n: int, k: int, keep: int = 1) -> int:
    b = _sz(0)
    _check(library().lbm_checkpoint_bytes(ctx, int(n), int(k), int(keep), ctypes.byref(b)),
           "lbm_checkpoint_bytes", ctx)
    return b.value


def lbm_run_checkpointed(ctx, n: int, k: int, keep: int, ckpt, ckpt_bytes: int) -> None:
    _check(library().lbm_run_checkpointed(ctx, int(n), int(k), int(keep), _addr(ckpt),
                                          int(ckpt_bytes)), "lbm_run_checkpointed", ctx)


def lbm_restore_checkpoint(ctx, n: int, k: int, keep: int, ckpt, ckpt_bytes: int,
                           slot: int) -> None:
    _check(library().lbm_restore_checkpoint(ctx, int(n), int(k), int(keep), _addr(ckpt),
                                            int(ckpt_bytes), int(slot)),
           "lbm_restore_checkpoint", ctx)


def lbm_adjoint_workspace_bytes(ctx, n: int, k: int, keep: int = 1) -> int:
    b = _sz(0)
    _check(library().lbm_adjoint_workspace_bytes(ctx, int(n), int(k), int(keep), ctypes.byref(b)),
           "lbm_adjoint_workspace_bytes", ctx)
    return b.value


def lbm_adjoint(ctx, n: int, k: int, keep: int, ckpt, ckpt_bytes: int, rho_init, U_init, T_init,
                dL_drho_final, workspace, ws_bytes: int, dL_dT_init=None,
                want_omega: bool = True) -> Optional[float]:
    dw = ctypes.c_double(0.0)
    st = library().lbm_adjoint(ctx, int(n), int(k), int(keep), _addr(ckpt), int(ckpt_bytes),
                               _addr(rho_init), _addr(U_init), _addr(T_init),
                               _addr(dL_drho_final), _addr(workspace), int(ws_bytes),
                               _addr(dL_dT_init), ctypes.byref(dw) if want_omega else None)
    _check(st, "lbm_adjoint", ctx)
    return float(dw.value) if want_omega else None


def lbm_destroy(ctx) -> None:
    if ctx:
        library().lbm_destroy(ctx)
