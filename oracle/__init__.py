"""ctypes wrapper around the FP64 CPU oracle (``oracle/lbm_oracle.cpp``).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark import this package.  The product library in
``paper_2311_10827_amd`` never imports it, and it imports nothing from there.

Arrays are numpy float64, C order:
  * fields ``[ny, nx]``;
  * populations ``[9, ny, nx]`` in the lattice order
    0 rest, 1 (+1,0), 2 (0,+1), 3 (-1,0), 4 (0,-1),
    5 (+1,+1), 6 (-1,+1), 7 (-1,-1), 8 (+1,-1).

The state is the pre-collision populations ``f`` (order parameter, the
paper's f_i), ``g`` (pressure/velocity, the paper's g_i), and ``Sp``, the
convection source u.grad(phi) of the previous step.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.cpp")
_LIB = os.path.join(_HERE, "liblbm_oracle.so")

PERIODIC, WALL = 0, 1
# viscosity across the interface: nu, 1/nu or ln nu linear in phi (Sec. 2.3.2)
NU_LINEAR, NU_INVERSE, NU_EXP = 0, 1, 2
# collision operator; MRT rates: f (e, eps, q, p), g ((rho, e, eps) together, q)
BGK, MRT = 0, 1


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (FP64, no FMA contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math",
               "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class OrcParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32),
        ("phi_A", ctypes.c_double), ("phi_B", ctypes.c_double),
        ("rho_A", ctypes.c_double), ("rho_B", ctypes.c_double),
        ("nu_A", ctypes.c_double), ("nu_B", ctypes.c_double),
        ("kappa", ctypes.c_double), ("beta", ctypes.c_double),
        ("M", ctypes.c_double), ("alpha", ctypes.c_double),
        ("gx", ctypes.c_double), ("gy", ctypes.c_double),
        ("nu_form", ctypes.c_int32),
        ("collision", ctypes.c_int32),
        ("mrt_f", ctypes.c_double * 4), ("mrt_g", ctypes.c_double * 2),
    ]


@dataclass
class Params:
    """Physical parameters in the paper's notation (phase A = paper l, B = v)."""
    nx: int
    ny: int
    bc_x: int = PERIODIC
    bc_y: int = PERIODIC
    phi_A: float = 1.0
    phi_B: float = -1.0
    rho_A: float = 1.0
    rho_B: float = 1.0
    nu_A: float = 0.1
    nu_B: float = 0.1
    kappa: float = 0.0
    beta: float = 0.0
    M: float = 0.1
    alpha: float = 1.0
    gx: float = 0.0
    gy: float = 0.0
    nu_form: int = NU_LINEAR
    collision: int = BGK
    mrt_f: tuple = (1.0, 1.0, 1.0, 1.0)
    mrt_g: tuple = (1.0, 1.0)

    def c(self) -> OrcParams:
        return OrcParams(self.nx, self.ny, self.bc_x, self.bc_y, self.phi_A, self.phi_B,
                         self.rho_A, self.rho_B, self.nu_A, self.nu_B, self.kappa, self.beta,
                         self.M, self.alpha, self.gx, self.gy, self.nu_form, self.collision,
                         (ctypes.c_double * 4)(*self.mrt_f), (ctypes.c_double * 2)(*self.mrt_g))

    @property
    def tau_f(self) -> float:
        return float(lib().orc_tau_f(ctypes.byref(self.c())))


_lib = None
_dp = ctypes.POINTER(ctypes.c_double)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(OrcParams)
        vp = ctypes.c_void_p
        L.orc_lattice.argtypes = [ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32), _dp, _dp]
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_get_threads.restype = ctypes.c_int
        L.orc_feq.argtypes = [P, ctypes.c_double, ctypes.c_double, _dp]
        L.orc_source.argtypes = [P, ctypes.c_double, _dp]
        L.orc_geq.argtypes = [P] + [ctypes.c_double] * 4 + [_dp]
        L.orc_forcing.argtypes = [P] + [ctypes.c_double] * 7 + [_dp]
        L.orc_macro.argtypes = [P, _dp] + [ctypes.c_double] * 5 + [_dp, _dp, _dp]
        L.orc_gradient.argtypes = [P, _dp, _dp, _dp]
        L.orc_laplacian.argtypes = [P, _dp, _dp]
        L.orc_chemical_potential.argtypes = [P, _dp, _dp]
        L.orc_tau_f.argtypes = [P]
        L.orc_tau_f.restype = ctypes.c_double
        L.orc_create.argtypes = [P]
        L.orc_create.restype = vp
        L.orc_destroy.argtypes = [vp]
        L.orc_init.argtypes = [vp, _dp, _dp, _dp]
        L.orc_step.argtypes = [vp, ctypes.c_int64]
        L.orc_moments.argtypes = [vp] + [_dp] * 7
        L.orc_get_state.argtypes = [vp, _dp, _dp, _dp]
        L.orc_set_state.argtypes = [vp, _dp, _dp, _dp]
        L.orc_tlm_create.argtypes = [P, _dp]
        L.orc_tlm_create.restype = vp
        L.orc_tlm_destroy.argtypes = [vp]
        L.orc_tlm_init.argtypes = [vp, _dp, _dp]
        L.orc_tlm_set_state.argtypes = [vp] + [_dp] * 6
        L.orc_tlm_step.argtypes = [vp, ctypes.c_int64]
        L.orc_tlm_get_state.argtypes = [vp] + [_dp] * 6
        L.orc_tlm_phi.argtypes = [vp, _dp, _dp]
        _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _f64(a, shape):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    assert a.shape == tuple(shape), (a.shape, shape)
    return a


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def get_threads() -> int:
    return int(lib().orc_get_threads())


def lattice():
    cx = (ctypes.c_int32 * 9)()
    cy = (ctypes.c_int32 * 9)()
    w = np.zeros(9)
    cs2 = ctypes.c_double()
    lib().orc_lattice(cx, cy, _p(w), ctypes.byref(cs2))
    return np.array(cx[:]), np.array(cy[:]), w, cs2.value


def feq(prm: Params, phi: float, mu: float) -> np.ndarray:
    out = np.zeros(9)
    lib().orc_feq(ctypes.byref(prm.c()), phi, mu, _p(out))
    return out


def source(prm: Params, S: float) -> np.ndarray:
    out = np.zeros(9)
    lib().orc_source(ctypes.byref(prm.c()), S, _p(out))
    return out


def geq(prm: Params, p: float, rho: float, ux: float, uy: float) -> np.ndarray:
    out = np.zeros(9)
    lib().orc_geq(ctypes.byref(prm.c()), p, rho, ux, uy, _p(out))
    return out


def forcing(prm: Params, tau: float, ux, uy, Fx, Fy, rx, ry) -> np.ndarray:
    out = np.zeros(9)
    lib().orc_forcing(ctypes.byref(prm.c()), tau, ux, uy, Fx, Fy, rx, ry, _p(out))
    return out


def macro(prm: Params, g9, rho, Fx, Fy, rx, ry):
    g9 = _f64(g9, (9,))
    a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    lib().orc_macro(ctypes.byref(prm.c()), _p(g9), rho, Fx, Fy, rx, ry,
                    ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
    return a.value, b.value, c.value


def gradient(prm: Params, field):
    field = _f64(field, (prm.ny, prm.nx))
    gx, gy = np.zeros_like(field), np.zeros_like(field)
    lib().orc_gradient(ctypes.byref(prm.c()), _p(field), _p(gx), _p(gy))
    return gx, gy


def divergence(prm: Params, ux, uy):
    """Discrete divergence of a velocity field, d_x u_x + d_y u_y, each
    derivative the isotropic gradient of Sec. 2.3.2 (eq. gradient) with the
    grid's periodic wrap or mirrored wall ghosts.  The equations the model
    recovers are incompressible (Sec. 2.3.2), so max |div u| measures how far
    the lattice velocity is from divergence-free."""
    gxx, _ = gradient(prm, ux)
    _, gyy = gradient(prm, uy)
    return gxx + gyy


BULK_TOL = 0.01  # a bulk cell's phase fraction lies within this of the grid's extreme


def laplace_jump(prm: Params, phi, mu, p):
    """Pressure jump between the two bulk phases, (mean of P^ over bulk-A
    cells) - (mean over bulk-B cells), with P^ = p + phi mu - psi(phi) and
    psi(phi) = beta (phi - phi_A)^2 (phi - phi_B)^2 (Sec. 2.1, eqs.
    bulk_energy, chemical_potencial): at mechanical equilibrium under the
    force -phi grad mu this is the quantity that jumps by sigma / R across a
    drop of radius R.  With the phase-A fraction s = (phi - phi_B) /
    (phi_A - phi_B), a cell is bulk A where s >= max(s) - 0.01 and bulk B
    where s <= min(s) + 0.01 (relative to the grid's extremes, since the
    bulk values themselves shift with the curvature).  Returns (jump,
    number of bulk-A cells, of bulk-B cells); the jump is 0 where either
    count is 0 or the two sets overlap (no interface)."""
    phi, mu, p = (np.asarray(a, dtype=np.float64) for a in (phi, mu, p))
    ph_hat = p + phi * mu - prm.beta * (phi - prm.phi_A) ** 2 * (phi - prm.phi_B) ** 2
    s = (phi - prm.phi_B) / (prm.phi_A - prm.phi_B)
    a, b = s >= s.max() - BULK_TOL, s <= s.min() + BULK_TOL
    na, nb = int(a.sum()), int(b.sum())
    if na == 0 or nb == 0 or np.any(a & b):
        return 0.0, na, nb
    return float(ph_hat[a].mean() - ph_hat[b].mean()), na, nb


def laplacian(prm: Params, field):
    field = _f64(field, (prm.ny, prm.nx))
    out = np.zeros_like(field)
    lib().orc_laplacian(ctypes.byref(prm.c()), _p(field), _p(out))
    return out


def chemical_potential(prm: Params, phi):
    phi = _f64(phi, (prm.ny, prm.nx))
    out = np.zeros_like(phi)
    lib().orc_chemical_potential(ctypes.byref(prm.c()), _p(phi), _p(out))
    return out


class Sim:
    """FP64 oracle simulation of one periodic or walled D2Q9 grid."""

    def __init__(self, prm: Params):
        self.prm = prm
        self._c = prm.c()
        self.h = lib().orc_create(ctypes.byref(self._c))
        self.shape = (prm.ny, prm.nx)

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().orc_destroy(h)
            self.h = None

    def init(self, phi0, ux0=None, uy0=None):
        phi0 = _f64(phi0, self.shape)
        ux0 = _f64(ux0, self.shape)
        uy0 = _f64(uy0, self.shape)
        lib().orc_init(self.h, _p(phi0), _p(ux0), _p(uy0))
        return self

    def step(self, n: int = 1):
        lib().orc_step(self.h, int(n))
        return self

    def moments(self) -> dict:
        out = {k: np.zeros(self.shape) for k in ("phi", "mu", "ux", "uy", "p", "rho", "S")}
        lib().orc_moments(self.h, *(_p(out[k]) for k in ("phi", "mu", "ux", "uy", "p", "rho", "S")))
        return out

    def get_state(self):
        f = np.zeros((9,) + self.shape)
        g = np.zeros((9,) + self.shape)
        Sp = np.zeros(self.shape)
        lib().orc_get_state(self.h, _p(f), _p(g), _p(Sp))
        return f, g, Sp

    def set_state(self, f, g, Sp):
        f = _f64(f, (9,) + self.shape)
        g = _f64(g, (9,) + self.shape)
        Sp = _f64(Sp, self.shape)
        lib().orc_set_state(self.h, _p(f), _p(g), _p(Sp))
        return self


class TLM:
    """Forward-mode tangent of the oracle (the same code over dual numbers).

    ``dtheta`` = (d kappa, d beta, d alpha, d tau_f, d nu_A, d nu_B).
    """

    def __init__(self, prm: Params, dtheta=None):
        self.prm = prm
        self._c = prm.c()
        dt = None if dtheta is None else _f64(dtheta, (6,))
        self._dt = dt
        self.h = lib().orc_tlm_create(ctypes.byref(self._c), _p(dt))
        self.shape = (prm.ny, prm.nx)

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().orc_tlm_destroy(h)
            self.h = None

    def init(self, phi0, dphi0=None):
        phi0 = _f64(phi0, self.shape)
        dphi0 = _f64(dphi0, self.shape)
        lib().orc_tlm_init(self.h, _p(phi0), _p(dphi0))
        return self

    def set_state(self, f, df, g, dg, Sp, dSp):
        sh9 = (9,) + self.shape
        args = [_f64(f, sh9), _f64(df, sh9), _f64(g, sh9), _f64(dg, sh9),
                _f64(Sp, self.shape), _f64(dSp, self.shape)]
        lib().orc_tlm_set_state(self.h, *(_p(a) for a in args))
        return self

    def step(self, n: int = 1):
        lib().orc_tlm_step(self.h, int(n))
        return self

    def get_state(self):
        sh9 = (9,) + self.shape
        out = [np.zeros(sh9), np.zeros(sh9), np.zeros(sh9), np.zeros(sh9),
               np.zeros(self.shape), np.zeros(self.shape)]
        lib().orc_tlm_get_state(self.h, *(_p(a) for a in out))
        return tuple(out)   # f, df, g, dg, Sp, dSp

    def phi(self):
        a, b = np.zeros(self.shape), np.zeros(self.shape)
        lib().orc_tlm_phi(self.h, _p(a), _p(b))
        return a, b


def kappa_beta(sigma: float, W: float, dphi: float):
    """(kappa, beta) from surface tension and interface width.

    Sec. 2.1: beta = 8 kappa / (W^2 dphi^2) (eq. beta) and
    sigma = dphi^3 sqrt(2 kappa beta) / 6 (eq. suiface_tension); substituting the
    first into the second gives sigma = (2/3) dphi^2 kappa / W.
    """
    kappa = 1.5 * sigma * W / (dphi * dphi)
    beta = 8.0 * kappa / (W * W * dphi * dphi)
    return kappa, beta


def params_for(wl, nx=None, ny=None, **over) -> Params:
    """Oracle parameters for a workload preset of ``paper_2311_10827_amd.inputs``."""
    kappa, beta = kappa_beta(wl.sigma, wl.W, abs(wl.phi_A - wl.phi_B))
    kw = dict(nx=nx or wl.nx, ny=ny or wl.ny, bc_x=wl.bc_x, bc_y=wl.bc_y, phi_A=wl.phi_A,
              phi_B=wl.phi_B, rho_A=wl.rho_A, rho_B=wl.rho_B, nu_A=wl.nu_A, nu_B=wl.nu_B,
              kappa=kappa, beta=beta, M=wl.M, alpha=wl.alpha,
              nu_form=getattr(wl, "nu_form", NU_LINEAR), collision=getattr(wl, "collision", BGK),
              mrt_f=tuple(getattr(wl, "mrt_f", (1.0, 1.0, 1.0, 1.0))),
              mrt_g=tuple(getattr(wl, "mrt_g", (1.0, 1.0))))
    kw.update(over)
    return Params(**kw)
