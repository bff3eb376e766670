"""Helpers shared by the GPU tests: the same seeded input and parameters to
the HIP path (through the C ABI) and to the FP64 oracle."""
from __future__ import annotations

import numpy as np

import oracle


def rel(a, b) -> float:
    """max|a - b| / max|b| (per field)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    s = np.abs(b).max()
    return float(np.abs(a - b).max() / (s if s > 0 else 1.0))


def gpu_sim(wl, phi0, precision=64, ux0=None, uy0=None, diag_every=0, **over):
    from paper_2311_10827_amd.sim import Sim, make_params
    p = make_params(wl, precision=precision, diag_every=diag_every, **over)
    return Sim(p, phi0, ux0, uy0)


def oracle_sim(wl, phi0, ux0=None, uy0=None, **over):
    prm = oracle.params_for(wl, **over)
    return oracle.Sim(prm).init(phi0, ux0, uy0)


def gpu_state(sim, window=None):
    return tuple(t.cpu().numpy() for t in sim.get_state(window))


def gpu_moments(sim):
    m = sim.moments()
    d = m.pop("diag")
    return {k: v.cpu().numpy() for k, v in m.items()}, d


def compare_state(gs, os_, tol):
    """Relative differences of (f, g, Sp); returns the dict and asserts tol."""
    names = ("f", "g", "Sp")
    out = {}
    for n, a, b in zip(names, gs, os_):
        out[n] = rel(a, b) if np.abs(b).max() > 0 else float(np.abs(a).max())
    assert all(v <= tol for v in out.values()), out
    return out


def compare_moments(gm, om, tol, u_floor=1e-18):
    out = {}
    for k in ("phi", "mu", "p", "rho"):
        out[k] = rel(gm[k], om[k])
    # velocity: relative to its own scale, with an absolute floor for fields
    # that sit at round-off
    s = max(np.abs(om["ux"]).max(), np.abs(om["uy"]).max())
    du = max(np.abs(gm["ux"] - om["ux"]).max(), np.abs(gm["uy"] - om["uy"]).max())
    out["u"] = du / s if s > 0 else du
    assert all(v <= tol for k, v in out.items() if k != "u"), out
    assert du <= tol * s + u_floor, out
    return out
