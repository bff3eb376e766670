"""ctypes binding of ``liblbmwb.so`` (declared in ``include/lbmwb.h``).

Argument marshalling only: every step of the method runs in the HIP kernels
of the library.  Loading fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbmwb.so")

LBM_OK, LBM_EINVAL, LBM_EHIP, LBM_ENONFINITE, LBM_ESTATE = 0, -1, -2, -3, -4
PERIODIC, WALL = 0, 1
SNAPSHOT_HAS_PHI_MU = 1
LO_AUTO, LO_16, LO_32 = 0, 1, 2
THETA_NATIVE, THETA_TAU = 0, 1

# Every symbol include/lbmwb.h declares.
SYMBOLS = (
    "lbm_derive", "lbm_state_bytes", "lbm_workspace_bytes", "lbm_init", "lbm_step",
    "lbm_step_count", "lbm_moments", "lbm_last_diag", "lbm_get_state", "lbm_set_state",
    "lbm_timing", "lbm_kernel_times", "lbm_stream_copy", "lbm_destroy", "lbm_strerror",
    "lbm_last_error", "lbm_snapshot_bytes", "lbm_snapshot", "lbm_restore",
    "lbm_adjoint_workspace_bytes", "lbm_adjoint_attach", "lbm_adjoint_step", "lbm_adjoint_init",
    "lbm_adjoint_theta", "lbm_step_into", "lbm_adjoint_segment", "lbm_step_noalloc",
)


class LbmParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("use_sigma_W", ctypes.c_int32),
        ("phi_A", ctypes.c_double), ("phi_B", ctypes.c_double),
        ("rho_A", ctypes.c_double), ("rho_B", ctypes.c_double),
        ("nu_A", ctypes.c_double), ("nu_B", ctypes.c_double),
        ("kappa", ctypes.c_double), ("beta", ctypes.c_double),
        ("sigma", ctypes.c_double), ("W", ctypes.c_double),
        ("M", ctypes.c_double), ("alpha", ctypes.c_double),
        ("gx", ctypes.c_double), ("gy", ctypes.c_double),
        ("diag_every", ctypes.c_int32), ("kernel_path", ctypes.c_int32),
        ("nu_form", ctypes.c_int32), ("collision", ctypes.c_int32),
        ("mrt_f", ctypes.c_double * 4), ("mrt_g", ctypes.c_double * 2),
        ("lo_format", ctypes.c_int32), ("use_tau", ctypes.c_int32),
        ("tau_f", ctypes.c_double), ("tau_gA", ctypes.c_double), ("tau_gB", ctypes.c_double),
    ]


class LbmDerived(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in
                ("kappa", "beta", "sigma", "W", "tau_f", "tau_gA", "tau_gB", "alpha", "nu_A",
                 "nu_B")] + [("lo16", ctypes.c_int32), ("two_step", ctypes.c_int32)]


class LbmDiag(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in
                ("sum_phi", "source_sum", "kinetic_energy", "max_u", "min_rho", "max_rho",
                 "mu_min", "mu_max", "phi_min", "phi_max", "max_div_u", "laplace_dP")] + [
        ("n_nonfinite", ctypes.c_int64), ("n_bulk_A", ctypes.c_int64), ("n_bulk_B", ctypes.c_int64),
        ("step", ctypes.c_int64)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class LbmError(RuntimeError):
    def __init__(self, code: int, what: str, detail: str = ""):
        self.code = code
        msg = f"{what} failed: {code} ({strerror(code)})"
        if detail:
            msg += f": {detail}"
        super().__init__(msg)


_lib = None


def load() -> ctypes.CDLL:
    """Load the in-tree HIP library; raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2311_10827_amd.build` "
            "(there is no CPU fallback)")
    # torch ships its own HIP runtime; loaded first, it is the one the
    # library binds to, so both share one runtime (the library loaded before
    # torch made lbm_init fail with a HIP error on MI355X).
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    P = ctypes.POINTER(LbmParams)
    L.lbm_derive.argtypes = [P, ctypes.POINTER(LbmDerived)]
    L.lbm_derive.restype = ctypes.c_int
    L.lbm_state_bytes.argtypes = [P]
    L.lbm_state_bytes.restype = ctypes.c_size_t
    L.lbm_workspace_bytes.argtypes = [P]
    L.lbm_workspace_bytes.restype = ctypes.c_size_t
    L.lbm_init.argtypes = [ctypes.POINTER(vp), P, vp, vp, dp, dp, dp, vp]
    L.lbm_init.restype = ctypes.c_int
    L.lbm_step.argtypes = [vp, i64]
    L.lbm_step.restype = ctypes.c_int
    L.lbm_step_noalloc.argtypes = [vp, i64]
    L.lbm_step_noalloc.restype = ctypes.c_int
    L.lbm_step_count.argtypes = [vp]
    L.lbm_step_count.restype = i64
    L.lbm_moments.argtypes = [vp, dp, dp, dp, dp, dp, dp, ctypes.POINTER(LbmDiag)]
    L.lbm_moments.restype = ctypes.c_int
    L.lbm_last_diag.argtypes = [vp, ctypes.POINTER(LbmDiag)]
    L.lbm_last_diag.restype = ctypes.c_int
    L.lbm_get_state.argtypes = [vp, i32, i32, i32, i32, dp, dp, dp]
    L.lbm_get_state.restype = ctypes.c_int
    L.lbm_set_state.argtypes = [vp, dp, dp, dp, i64]
    L.lbm_set_state.restype = ctypes.c_int
    L.lbm_timing.argtypes = [vp, ctypes.c_int]
    L.lbm_timing.restype = ctypes.c_int
    L.lbm_kernel_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]
    L.lbm_kernel_times.restype = ctypes.c_int
    L.lbm_stream_copy.argtypes = [vp, vp, ctypes.c_size_t, vp]
    L.lbm_stream_copy.restype = ctypes.c_int
    L.lbm_destroy.argtypes = [vp]
    L.lbm_destroy.restype = ctypes.c_int
    L.lbm_strerror.argtypes = [ctypes.c_int]
    L.lbm_strerror.restype = ctypes.c_char_p
    L.lbm_last_error.argtypes = [vp]
    L.lbm_last_error.restype = ctypes.c_char_p
    L.lbm_snapshot_bytes.argtypes = [vp]
    L.lbm_snapshot_bytes.restype = ctypes.c_size_t
    L.lbm_snapshot.argtypes = [vp, vp]
    L.lbm_snapshot.restype = ctypes.c_int
    L.lbm_restore.argtypes = [vp, vp, i64]
    L.lbm_restore.restype = ctypes.c_int
    L.lbm_adjoint_workspace_bytes.argtypes = [P]
    L.lbm_adjoint_workspace_bytes.restype = ctypes.c_size_t
    L.lbm_adjoint_attach.argtypes = [vp, vp]
    L.lbm_adjoint_attach.restype = ctypes.c_int
    L.lbm_step_into.argtypes = [vp, vp, vp]
    L.lbm_step_into.restype = ctypes.c_int
    L.lbm_adjoint_step.argtypes = [vp, vp, vp, vp, ctypes.c_int]
    L.lbm_adjoint_step.restype = ctypes.c_int
    L.lbm_adjoint_segment.argtypes = [vp, ctypes.POINTER(vp), ctypes.c_int, vp, vp,
                                      ctypes.POINTER(ctypes.c_int)]
    L.lbm_adjoint_segment.restype = ctypes.c_int
    L.lbm_adjoint_init.argtypes = [vp, vp, vp, vp, vp, vp]
    L.lbm_adjoint_init.restype = ctypes.c_int
    L.lbm_adjoint_theta.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.c_int]
    L.lbm_adjoint_theta.restype = ctypes.c_int
    _lib = L
    return L


def strerror(code: int) -> str:
    try:
        return load().lbm_strerror(code).decode()
    except ImportError:
        return str(code)


def check(code: int, what: str, ctx=None) -> None:
    if code != LBM_OK:
        detail = ""
        if ctx:
            detail = (load().lbm_last_error(ctx) or b"").decode()
        raise LbmError(code, what, detail)
