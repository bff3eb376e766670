"""PyTorch-side wrapper of the C ABI: device memory and streams only.

PyTorch allocates the state and workspace buffers and provides the HIP
stream; every step of the method runs in ``liblbmwb.so``.
"""
from __future__ import annotations

import ctypes
from typing import Optional

import torch

from . import _lib
from ._lib import LbmDiag, LbmParams, LbmDerived, check

# viscosity across the interface (lbm_params.nu_form): nu, 1/nu or ln nu linear in phi
NU_LINEAR, NU_INVERSE, NU_EXP = 0, 1, 2
# collision operator (lbm_params.collision); MRT rates: mrt_f = f's (e, eps, q, p),
# mrt_g = g's ((rho, e, eps), q)
BGK, MRT = 0, 1


def make_params(workload=None, precision: int = 64, diag_every: int = 0, **over) -> LbmParams:
    """C parameter block from a workload preset (``inputs.Workload``) and overrides.

    A workload gives sigma and W; the library derives kappa and beta from them
    (use_sigma_W = 1) unless ``kappa`` and ``beta`` are passed explicitly.
    """
    kw = dict(nx=0, ny=0, bc_x=0, bc_y=0, precision=precision, use_sigma_W=0, phi_A=1.0,
              phi_B=-1.0, rho_A=1.0, rho_B=1.0, nu_A=0.1, nu_B=0.1, kappa=0.0, beta=0.0,
              sigma=0.0, W=0.0, M=0.1, alpha=1.0, gx=0.0, gy=0.0, diag_every=diag_every,
              kernel_path=0, nu_form=NU_LINEAR, collision=BGK, mrt_f=(1.0, 1.0, 1.0, 1.0),
              mrt_g=(1.0, 1.0), lo_format=_lib.LO_AUTO, use_tau=0, tau_f=0.0, tau_gA=0.0, tau_gB=0.0)
    if workload is not None:
        for k in ("nx", "ny", "bc_x", "bc_y", "phi_A", "phi_B", "rho_A", "rho_B", "nu_A", "nu_B",
                  "sigma", "W", "M", "alpha", "nu_form", "collision", "mrt_f", "mrt_g"):
            kw[k] = getattr(workload, k)
        kw["use_sigma_W"] = 1
    if "kappa" in over or "beta" in over:
        kw["use_sigma_W"] = 0
    kw.update(over)
    kw["mrt_f"] = (ctypes.c_double * 4)(*kw["mrt_f"])
    kw["mrt_g"] = (ctypes.c_double * 2)(*kw["mrt_g"])
    return LbmParams(**kw)


def derive(p: LbmParams) -> dict:
    d = LbmDerived()
    check(_lib.load().lbm_derive(ctypes.byref(p), ctypes.byref(d)), "lbm_derive")
    return {k: getattr(d, k) for k, _ in d._fields_}


def _dev_f64(a, shape, device) -> Optional[torch.Tensor]:
    if a is None:
        return None
    t = torch.as_tensor(a, dtype=torch.float64, device=device).contiguous()
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"expected shape {tuple(shape)}, got {tuple(t.shape)}")
    return t


def pick_state_buffers(params: LbmParams, phi0, tries: int = 3, steps: int = 4, device="cuda:0"):
    """State and workspace buffers for ``params``: up to ``tries``
    allocations, keeping the one on which ``steps`` steps from ``phi0`` run
    fastest.  How fast a large step runs depends, by up to about 10 % at
    16384^2 on MI355X, on where in HBM the state's pages land, which neither
    the library nor the caller chooses; a long run can afford this probe
    (a few steps per try).  A rejected allocation is released to the driver
    before the next try, so the next one gets pages of its own.  Returns
    (state, workspace, [ms per step of each try])."""
    L = _lib.load()
    nb = L.lbm_state_bytes(ctypes.byref(params))
    nw = L.lbm_workspace_bytes(ctypes.byref(params))
    if nb == 0 or nw == 0:
        raise _lib.LbmError(_lib.LBM_EINVAL, "lbm_state_bytes")
    dev = torch.device(device)
    best, times = None, []
    for _ in range(max(1, tries)):
        st = torch.empty(nb, dtype=torch.uint8, device=dev)
        ws = torch.empty(nw, dtype=torch.uint8, device=dev)
        sim = Sim(params, phi0, device=dev, state=st, workspace=ws)
        sim.step(2)
        sim.stream.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(sim.stream)
        sim.step(steps)
        e1.record(sim.stream)
        e1.synchronize()
        sim.close()
        times.append(e0.elapsed_time(e1) / steps)
        if best is None or times[-1] < best[2]:
            best = (st, ws, times[-1])
        else:
            del st, ws
        del sim
        torch.cuda.empty_cache()
    return best[0], best[1], times


def _caller_buffer(t: torch.Tensor, nbytes: int, device, what: str) -> torch.Tensor:
    if t.dtype != torch.uint8 or t.device != torch.device(device) or not t.is_contiguous():
        raise ValueError(f"{what}: expected a contiguous uint8 tensor on {device}")
    if t.numel() < nbytes or t.data_ptr() % 256:
        raise ValueError(f"{what}: needs {nbytes} bytes, 256-byte aligned")
    return t[:nbytes]


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _storage_dtype(precision: int):
    return torch.float64 if precision == 64 else torch.float32


class Sim:
    """One simulation context on one GPU."""

    def __init__(self, params: LbmParams, phi0, ux0=None, uy0=None, device="cuda:0", state=None,
                 workspace=None):
        """``state``/``workspace``: optional uint8 device tensors of at least
        ``lbm_state_bytes``/``lbm_workspace_bytes`` to use instead of new ones
        (256-byte aligned; the state is zeroed here)."""
        self.L = _lib.load()
        self.p = params
        self.derived = derive(params)
        self.device = torch.device(device)
        self.shape = (params.ny, params.nx)
        nb = self.L.lbm_state_bytes(ctypes.byref(params))
        nw = self.L.lbm_workspace_bytes(ctypes.byref(params))
        if nb == 0 or nw == 0:
            raise _lib.LbmError(_lib.LBM_EINVAL, "lbm_state_bytes")
        with torch.cuda.device(self.device):
            # zeroed so that the padding between rows and planes (never written
            # by the kernels) is defined and raw snapshots compare bytewise
            if state is None:
                self.state = torch.zeros(nb, dtype=torch.uint8, device=self.device)
            else:
                self.state = _caller_buffer(state, nb, self.device, "state").zero_()
            if workspace is None:
                self.workspace = torch.empty(nw, dtype=torch.uint8, device=self.device)
            else:
                self.workspace = _caller_buffer(workspace, nw, self.device, "workspace")
            self.stream = torch.cuda.current_stream(self.device)
            phi0 = _dev_f64(phi0, self.shape, self.device)
            ux0 = _dev_f64(ux0, self.shape, self.device)
            uy0 = _dev_f64(uy0, self.shape, self.device)
            ctx = ctypes.c_void_p()
            rc = self.L.lbm_init(ctypes.byref(ctx), ctypes.byref(params),
                                 ctypes.c_void_p(self.state.data_ptr()),
                                 ctypes.c_void_p(self.workspace.data_ptr()), _ptr(phi0), _ptr(ux0),
                                 _ptr(uy0), ctypes.c_void_p(self.stream.cuda_stream))
            check(rc, "lbm_init")
            self.ctx = ctx
            self._keep = (phi0, ux0, uy0)
            self.stream.synchronize()
            self._keep = None

    # -- lifecycle ---------------------------------------------------------
    def close(self):
        if getattr(self, "ctx", None):
            self.L.lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- time stepping -------------------------------------------------------
    def step(self, n: int = 1) -> "Sim":
        check(self.L.lbm_step(self.ctx, int(n)), "lbm_step", self.ctx)
        return self

    def step_noalloc(self, n: int = 1) -> "Sim":
        """The same steps through lbm_step_noalloc (diagnostic reductions in
        the library's per-GPU scratch; the call allocates nothing)."""
        check(self.L.lbm_step_noalloc(self.ctx, int(n)), "lbm_step_noalloc", self.ctx)
        return self

    @property
    def step_count(self) -> int:
        return int(self.L.lbm_step_count(self.ctx))

    def moments(self, diag: bool = True, fields: bool = True):
        """phi, mu, ux, uy, p, rho as FP64 device fields (fields=False: none,
        the library stages what its diagnostics need) and, with diag, the
        FP64 diagnostics under "diag"."""
        names = ("phi", "mu", "ux", "uy", "p", "rho")
        out = {k: torch.empty(self.shape, dtype=torch.float64, device=self.device)
               for k in names} if fields else {}
        d = LbmDiag()
        rc = self.L.lbm_moments(self.ctx, *(_ptr(out.get(k)) for k in names),
                                ctypes.byref(d) if diag else None)
        check(rc, "lbm_moments", self.ctx)
        if diag:
            out["diag"] = d.as_dict()
        return out

    def last_diag(self) -> dict:
        d = LbmDiag()
        rc = self.L.lbm_last_diag(self.ctx, ctypes.byref(d))
        if rc not in (_lib.LBM_OK, _lib.LBM_ENONFINITE):
            check(rc, "lbm_last_diag", self.ctx)
        r = d.as_dict()
        r["ok"] = rc == _lib.LBM_OK
        return r

    # -- state ---------------------------------------------------------------
    def get_state(self, window=None):
        """(f, g, Sp) pre-collision populations [9,h,w] and previous source [h,w]."""
        x0, y0, w, h = window if window is not None else (0, 0, self.p.nx, self.p.ny)
        f = torch.empty((9, h, w), dtype=torch.float64, device=self.device)
        g = torch.empty((9, h, w), dtype=torch.float64, device=self.device)
        Sp = torch.empty((h, w), dtype=torch.float64, device=self.device)
        check(self.L.lbm_get_state(self.ctx, x0, y0, w, h, _ptr(f), _ptr(g), _ptr(Sp)),
              "lbm_get_state", self.ctx)
        return f, g, Sp

    def set_state(self, f, g, Sp, step: int = 0) -> "Sim":
        sh9 = (9,) + self.shape
        f, g, Sp = _dev_f64(f, sh9, self.device), _dev_f64(g, sh9, self.device), _dev_f64(Sp, self.shape, self.device)
        check(self.L.lbm_set_state(self.ctx, _ptr(f), _ptr(g), _ptr(Sp), int(step)), "lbm_set_state", self.ctx)
        self.stream.synchronize()
        return self

    # -- timing ----------------------------------------------------------------
    def timing(self, enable: bool) -> None:
        check(self.L.lbm_timing(self.ctx, int(bool(enable))), "lbm_timing", self.ctx)

    def kernel_times(self):
        """(summed ms of the timed steps' kernels, number of steps)."""
        a, n = ctypes.c_double(), ctypes.c_int64()
        check(self.L.lbm_kernel_times(self.ctx, ctypes.byref(a), ctypes.byref(n)),
              "lbm_kernel_times", self.ctx)
        return a.value, n.value

    # -- snapshots (raw state) ----------------------------------------------

    def snapshot_bytes(self) -> int:
        return int(self.L.lbm_snapshot_bytes(self.ctx))

    def new_snapshot(self, zeroed: bool = True) -> torch.Tensor:
        """A snapshot buffer.  zeroed=False leaves the row and plane padding
        (never read by the kernels) undefined, which only matters to a
        bytewise comparison of raw snapshots."""
        alloc = torch.zeros if zeroed else torch.empty
        return alloc(self.snapshot_bytes(), dtype=torch.uint8, device=self.device)

    def snapshot(self, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        out = self.new_snapshot() if out is None else out
        check(self.L.lbm_snapshot(self.ctx, _ptr(out)), "lbm_snapshot", self.ctx)
        return out

    def restore(self, snap: torch.Tensor, step: int) -> "Sim":
        check(self.L.lbm_restore(self.ctx, _ptr(snap), int(step)), "lbm_restore", self.ctx)
        return self

    def step_into(self, src: torch.Tensor, dst: torch.Tensor) -> None:
        check(self.L.lbm_step_into(self.ctx, _ptr(src), _ptr(dst)), "lbm_step_into", self.ctx)

    # -- adjoint -------------------------------------------------------------
    def enable_adjoint(self) -> None:
        if getattr(self, "adj_ws", None) is not None:
            return
        nb = self.L.lbm_adjoint_workspace_bytes(ctypes.byref(self.p))
        self.adj_ws = torch.empty(nb, dtype=torch.uint8, device=self.device)
        check(self.L.lbm_adjoint_attach(self.ctx, _ptr(self.adj_ws)), "lbm_adjoint_attach", self.ctx)

    def new_adjoint(self) -> torch.Tensor:
        """Zeroed adjoint of a state: 19 planes (f_0..f_8, g_0..g_8, S_prev)."""
        return torch.zeros((19,) + self.shape, dtype=_storage_dtype(self.p.precision), device=self.device)

    def adjoint_step(self, state: torch.Tensor, lam_in: torch.Tensor, lam_out: torch.Tensor,
                     have_phi_mu: bool = False) -> None:
        flags = _lib.SNAPSHOT_HAS_PHI_MU if have_phi_mu else 0
        check(self.L.lbm_adjoint_step(self.ctx, _ptr(state), _ptr(lam_in), _ptr(lam_out), flags),
              "lbm_adjoint_step", self.ctx)

    def adjoint_segment(self, snaps, lam: torch.Tensor, tmp: torch.Tensor) -> int:
        """Recompute a checkpoint segment and run its adjoint steps natively.

        Returns 0 if dL/d(first state) is in ``lam``, 1 if in ``tmp``."""
        arr = (ctypes.c_void_p * len(snaps))(*[t.data_ptr() for t in snaps])
        which = ctypes.c_int()
        check(self.L.lbm_adjoint_segment(self.ctx, arr, len(snaps), _ptr(lam), _ptr(tmp),
                                         ctypes.byref(which)), "lbm_adjoint_segment", self.ctx)
        return which.value

    def adjoint_init(self, state0: torch.Tensor, phi0: torch.Tensor, lam0: torch.Tensor,
                     scratch: torch.Tensor) -> torch.Tensor:
        phi0 = _dev_f64(phi0, self.shape, self.device)
        out = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        check(self.L.lbm_adjoint_init(self.ctx, _ptr(state0), _ptr(phi0), _ptr(lam0), _ptr(scratch),
                                      _ptr(out)), "lbm_adjoint_init", self.ctx)
        self._keep_phi0 = phi0
        return out

    def adjoint_theta(self, reset: bool = True, basis: int = _lib.THETA_NATIVE):
        """Parameter gradient accumulated so far: dL/d(kappa, beta, alpha, tau_f,
        nu_A, nu_B) (THETA_NATIVE) or dL/d(kappa, beta, M, tau_f, tau_gA, tau_gB)
        (THETA_TAU), as the library forms them."""
        buf = (ctypes.c_double * 6)()
        check(self.L.lbm_adjoint_theta(self.ctx, int(basis), buf, int(bool(reset))), "lbm_adjoint_theta",
              self.ctx)
        return list(buf)


def stream_copy(dst: torch.Tensor, src: torch.Tensor) -> None:
    """Plain streaming copy kernel of the library (bandwidth probe)."""
    L = _lib.load()
    nbytes = src.numel() * src.element_size()
    rc = L.lbm_stream_copy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()), nbytes,
                           ctypes.c_void_p(torch.cuda.current_stream(src.device).cuda_stream))
    check(rc, "lbm_stream_copy")
