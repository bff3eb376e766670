"""The paper's own test cases on the GPU (Sec. 3.1, 3.2 and 3.3).

The order parameter is in {0, 1} (liquid phi = 1, vapour 0), rho_v = 1,
nu_v = 0.1, M = 0.1, alpha = 1, sigma = 0.005, all grids periodic.

* flat interface (Sec. 3.1): 32 x 128, a liquid slab between y = L_y/4 and
  3 L_y/4 (eq. flatinitial), W = 4;
* stationary droplet (Sec. 3.2): 128 x 128, R = L/4 at the centre, W = 4;
* coalescence of two drops (Sec. 3.3): 512 x 512, two drops of radius
  R_0 = L/10 with centres 0.5 L -+ (R_0 + W/2), W = 8.

The static cases relax from their tanh profiles while the total kinetic
energy E = 1/2 sum rho |u|^2 is followed down to round-off, at density ratios
10, 100, 1000 with equal kinematic viscosities, and at density ratio 1000
with dynamic viscosity ratios 10, 100, 1000.  The coalescence runs at
density ratio 1000 with kinematic viscosity ratios nu_l/nu_v of 0.1 and 0.01
(the paper's stability cases), or 1 at density ratios 10, 100, 1000.  The
paper states no step counts.

    python -m paper_2311_10827_amd.replica --case droplet --rho-ratio 1000 --steps 4000000
    python -m paper_2311_10827_amd.replica --case coalescence --rho-ratio 1000 --nu-ratio 0.01 --steps 100000
"""
from __future__ import annotations

import argparse
import sys
import time

import numpy as np

from . import inputs

SIGMA, W, M, ALPHA = 0.005, 4.0, 0.1, 1.0
RHO_V, NU_V = 1.0, 0.1


W_COALESCENCE = 8.0


def workload(case: str, rho_ratio: float, mu_ratio: float | None = None,
             nu_ratio: float | None = None) -> tuple:
    """(Workload, phi0) of one of the paper's cases.

    The liquid's kinematic viscosity: nu_v unless a ratio is given, either
    the dynamic mu_ratio = rho_l nu_l / (rho_v nu_v) or the kinematic
    nu_ratio = nu_l / nu_v."""
    if mu_ratio is not None and nu_ratio is not None:
        raise ValueError("give mu_ratio or nu_ratio, not both")
    nu_l = NU_V
    if mu_ratio is not None:
        nu_l = mu_ratio * RHO_V * NU_V / rho_ratio
    elif nu_ratio is not None:
        nu_l = nu_ratio * NU_V
    w = W
    if case == "flat":
        nx, ny = 32, 128
        phi0 = inputs.slab(nx, ny, w, phi_A=1.0, phi_B=0.0)
    elif case == "droplet":
        nx = ny = 128
        phi0 = inputs.droplet(nx, ny, 0.25 * nx, w, 0.5 * nx, 0.5 * ny, phi_A=1.0, phi_B=0.0)
    elif case == "coalescence":
        nx = ny = 512
        w = W_COALESCENCE
        phi0 = inputs.two_drops(nx, ny, 0.1 * nx, w, phi_A=1.0, phi_B=0.0)
    else:
        raise ValueError(case)
    wl = inputs.Workload(f"paper_{case}", nx, ny, phi_A=1.0, phi_B=0.0, rho_A=rho_ratio * RHO_V,
                         rho_B=RHO_V, nu_A=nu_l, nu_B=NU_V, sigma=SIGMA, W=w, M=M, alpha=ALPHA)
    return wl, phi0


def relax(case: str, rho_ratio: float, steps: int, every: int, mu_ratio: float | None = None,
          precision: int = 64, kernel_path: int = 0, log=None, nu_ratio: float | None = None,
          full: bool = False, **over):
    """Run the case and return [(step, E, max|u|, mu spread)] every `every`
    steps (E and max|u| from the library's FP64 diagnostics); with ``full``
    each record is the whole diagnostic dict instead.  ``over``: further
    lbm_params fields (a collision operator and its rates, say)."""
    from .sim import Sim, make_params
    wl, phi0 = workload(case, rho_ratio, mu_ratio, nu_ratio)
    sim = Sim(make_params(wl, precision=precision, kernel_path=kernel_path, **over), phi0)
    hist = []
    try:
        done = 0
        while done < steps:
            n = min(every, steps - done)
            sim.step(n)
            done += n
            m = sim.moments(fields=False)
            d = m["diag"]
            hist.append(dict(d) if full else (done, d["kinetic_energy"], d["max_u"], d["mu_max"] - d["mu_min"]))
            if d["n_nonfinite"]:
                raise FloatingPointError(f"non-finite state at step {done}")
            if log:
                log(f"  step {done}: E {d['kinetic_energy']:.3e}  max|u| {d['max_u']:.3e}  "
                    f"min rho {d['min_rho']:.4g}")
    finally:
        sim.close()
    return hist


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--case", choices=("flat", "droplet", "coalescence"), default="droplet")
    ap.add_argument("--rho-ratio", type=float, default=10.0)
    ap.add_argument("--mu-ratio", type=float, default=None)
    ap.add_argument("--nu-ratio", type=float, default=None)
    ap.add_argument("--steps", type=int, default=1_000_000)
    ap.add_argument("--every", type=int, default=100_000)
    ap.add_argument("--precision", type=int, choices=(32, 64), default=64)
    a = ap.parse_args(argv)
    t0 = time.time()
    hist = relax(a.case, a.rho_ratio, a.steps, a.every, a.mu_ratio, a.precision,
                 log=lambda s: print(s, flush=True), nu_ratio=a.nu_ratio)
    e = np.array([h[1] for h in hist])
    k = int(np.argmin(e))
    print(f"{a.case} rho_l/rho_v {a.rho_ratio:g} mu ratio {a.mu_ratio}: min E {e[k]:.3e} at step "
          f"{hist[k][0]} (max|u| {hist[k][2]:.3e}); final E {e[-1]:.3e}, max|u| {hist[-1][2]:.3e}, "
          f"mu spread {hist[-1][3]:.3e}; {time.time() - t0:.1f} s", flush=True)


if __name__ == "__main__":
    sys.exit(main())
