"""Seeded synthetic initial fields and workload presets.

This module holds input recipes only, none of the method's arithmetic, and
imports nothing from the rest of the package, so the HIP path and the CPU
oracle can both take their inputs from it.

Initial order-parameter profiles follow the paper's test set-ups:
  * flat interface, hyperbolic-tangent profile (Sec. 3.1, eq. flatinitial);
  * stationary droplet (Sec. 3.2, eq. case1, written there for the density;
    the same form is used here for phi);
  * two touching droplets (Sec. 3.3, the two-drop formula with d_1, d_2);
  * many separated droplets, a sum of single-drop tanh bumps, for throughput.

Cell (i, j) has centre x = i, y = j.  Seeds are
``numpy.random.default_rng(231110827 + workload_id)``.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 231110827


def rng_for(workload_id: int) -> np.random.Generator:
    return np.random.default_rng(SEED_BASE + int(workload_id))


def flat_interface(nx: int = 256, ny: int = 4, W: float = 4.0, x0: float = 128.0,
                   phi_A: float = 1.0, phi_B: float = -1.0) -> np.ndarray:
    """One flat interface normal to x at x0: phi_B for x << x0, phi_A for x >> x0."""
    x = np.arange(nx, dtype=np.float64)
    prof = 0.5 * (phi_A + phi_B) + 0.5 * (phi_A - phi_B) * np.tanh(2.0 * (x - x0) / W)
    return np.ascontiguousarray(np.broadcast_to(prof, (ny, nx)))


def slab(nx: int, ny: int, W: float, phi_A: float = 1.0, phi_B: float = -1.0) -> np.ndarray:
    """Liquid slab between y = ny/4 and 3ny/4 (Sec. 3.1, eq. flatinitial)."""
    y = np.arange(ny, dtype=np.float64)
    z1, z2 = y - 0.25 * ny, y - 0.75 * ny
    prof = phi_B + 0.5 * (phi_A - phi_B) * (np.tanh(2 * z1 / W) - np.tanh(2 * z2 / W))
    return np.ascontiguousarray(np.broadcast_to(prof[:, None], (ny, nx)))


def _periodic_delta(a: np.ndarray, c: float, L: int) -> np.ndarray:
    d = a - c
    return d - L * np.round(d / L)


def droplet(nx: int, ny: int, R: float, W: float, xc: float, yc: float,
            phi_A: float = 1.0, phi_B: float = -1.0) -> np.ndarray:
    """Circular drop of phase A, radius R, centre (xc, yc), periodic distance."""
    x = np.arange(nx, dtype=np.float64)
    y = np.arange(ny, dtype=np.float64)
    dx = _periodic_delta(x, xc, nx)[None, :]
    dy = _periodic_delta(y, yc, ny)[:, None]
    r = np.sqrt(dx * dx + dy * dy)
    return 0.5 * (phi_A + phi_B) + 0.5 * (phi_A - phi_B) * np.tanh(2.0 * (R - r) / W)


def jittered_droplet(L: int, R: float, W: float, workload_id: int = 2,
                     phi_A: float = 1.0, phi_B: float = -1.0) -> np.ndarray:
    g = rng_for(workload_id)
    jx, jy = g.uniform(-0.5, 0.5, size=2)
    return droplet(L, L, R, W, L / 2 + jx, L / 2 + jy, phi_A, phi_B)


def two_drops(nx: int, ny: int, R: float, W: float, noise: float = 0.0,
              workload_id: int = 3, phi_A: float = 1.0, phi_B: float = -1.0) -> np.ndarray:
    """Two drops whose centres sit R + W/2 either side of the domain centre."""
    x = np.arange(nx, dtype=np.float64)[None, :]
    y = np.arange(ny, dtype=np.float64)[:, None]
    x1, x2, yc = 0.5 * nx - R - 0.5 * W, 0.5 * nx + R + 0.5 * W, 0.5 * ny
    d1 = np.sqrt((x - x1) ** 2 + (y - yc) ** 2) - R
    d2 = np.sqrt((x - x2) ** 2 + (y - yc) ** 2) - R
    phi = 0.5 * (phi_A + phi_B) + 0.5 * (phi_A - phi_B) * (
        1.0 - np.tanh(2.0 * d1 / W) - np.tanh(2.0 * d2 / W))
    if noise > 0:
        phi = phi + rng_for(workload_id).uniform(-noise, noise, size=phi.shape)
    return phi


def drop_centres(L: int, n: int, rmin: float, rmax: float, W: float,
                 workload_id: int = 4, max_tries: int = 2_000_000):
    """Rejection-sampled non-overlapping drops (periodic separation >= Ri+Rj+2W)."""
    g = rng_for(workload_id)
    xs, ys, rs = [], [], []
    tries = 0
    cell = 2 * (rmax + W) + 1
    nb = max(1, int(L // cell))
    grid: dict = {}
    while len(rs) < n:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place drops")
        r = g.uniform(rmin, rmax)
        cx, cy = g.uniform(0, L, size=2)
        bx, by = int(cx / L * nb) % nb, int(cy / L * nb) % nb
        ok = True
        for ox in (-1, 0, 1):
            for oy in (-1, 0, 1):
                for k in grid.get(((bx + ox) % nb, (by + oy) % nb), ()):
                    ddx = (cx - xs[k] + L / 2) % L - L / 2
                    ddy = (cy - ys[k] + L / 2) % L - L / 2
                    if ddx * ddx + ddy * ddy < (r + rs[k] + 2 * W) ** 2:
                        ok = False
                        break
                if not ok:
                    break
            if not ok:
                break
        if ok:
            grid.setdefault((bx, by), []).append(len(rs))
            xs.append(cx); ys.append(cy); rs.append(r)
    return np.array(xs), np.array(ys), np.array(rs)


def many_drops(L: int = 16384, n: int = 2000, rmin: float = 20.0, rmax: float = 80.0,
               W: float = 4.0, workload_id: int = 4, phi_A: float = 1.0,
               phi_B: float = -1.0, window=None) -> np.ndarray:
    """phi = phi_B + (phi_A - phi_B) sum_k (1 - tanh(2 d_k / W)) / 2 over drops with d_k < 10 W.

    ``window`` = (x0, y0, w, h) returns only that periodic window of the field.
    """
    xs, ys, rs = drop_centres(L, n, rmin, rmax, W, workload_id)
    if window is None:
        x0, y0, w, h = 0, 0, L, L
    else:
        x0, y0, w, h = window
    acc = np.zeros((h, w), dtype=np.float64)
    for cx, cy, r in zip(xs, ys, rs):
        reach = r + 10 * W
        # window-relative coordinates of the drop centre's nearest periodic image
        rx = (cx - x0 + L / 2) % L - L / 2
        ry = (cy - y0 + L / 2) % L - L / 2
        for ix in {rx, rx + L, rx - L}:
            for iy in {ry, ry + L, ry - L}:
                xa, xb = int(np.floor(ix - reach)), int(np.ceil(ix + reach)) + 1
                ya, yb = int(np.floor(iy - reach)), int(np.ceil(iy + reach)) + 1
                xa, xb = max(xa, 0), min(xb, w)
                ya, yb = max(ya, 0), min(yb, h)
                if xa >= xb or ya >= yb:
                    continue
                px = np.arange(xa, xb, dtype=np.float64)[None, :] - ix
                py = np.arange(ya, yb, dtype=np.float64)[:, None] - iy
                d = np.sqrt(px * px + py * py) - r
                bump = np.where(d < 10 * W, 0.5 * (1.0 - np.tanh(2.0 * d / W)), 0.0)
                acc[ya:yb, xa:xb] += bump
    return phi_B + (phi_A - phi_B) * acc


@dataclass
class Workload:
    """Physical parameters of one synthetic workload (lattice units)."""
    name: str
    nx: int
    ny: int
    bc_x: int = 0          # 0 periodic, 1 half-way bounce-back walls
    bc_y: int = 0
    phi_A: float = 1.0
    phi_B: float = -1.0
    rho_A: float = 1.0
    rho_B: float = 1.0
    nu_A: float = 0.1
    nu_B: float = 0.1
    sigma: float = 1e-3
    W: float = 4.0
    M: float = 0.05
    alpha: float = 1.0
    nu_form: int = 0       # 0 nu, 1 1/nu, 2 ln nu linear in phi
    collision: int = 0     # 0 BGK, 1 MRT
    mrt_f: tuple = (1.0, 1.0, 1.0, 1.0)  # MRT rates of f: e, eps, q, p
    mrt_g: tuple = (1.0, 1.0)            # MRT rates of g: (rho, e, eps), q
    steps: int = 1000
    extra: dict = field(default_factory=dict)


# Flat interface: 256 x 4, walls in x, density ratio 10, nu 0.1/0.1, M 0.1, sigma 0.01, W 4.
FLAT = Workload("flat_interface_256x4", 256, 4, bc_x=1, rho_A=10.0, rho_B=1.0,
                nu_A=0.1, nu_B=0.1, sigma=0.01, W=4.0, M=0.1, steps=20000)
# Stationary droplet: 512^2, density ratio 1000, dynamic viscosity ratio 100.
DROPLET = Workload("droplet_512", 512, 512, rho_A=1000.0, rho_B=1.0, nu_A=0.01, nu_B=0.1,
                   sigma=1e-3, W=4.0, M=0.05, steps=50000,
                   extra={"radii": (32, 48, 64, 96, 128)})
# Two-drop coalescence: 4096^2, R 400, W 5, density ratio 1000, viscosity ratio 100.
COALESCENCE = Workload("coalescence_4096", 4096, 4096, rho_A=1000.0, rho_B=1.0, nu_A=0.01,
                       nu_B=0.1, sigma=1e-3, W=5.0, M=0.05, steps=10000,
                       extra={"R": 400.0, "noise": 1e-3, "crop": (1792, 1792, 512, 512)})
# Throughput: 16384^2, 2000 drops, R ~ U(20, 80), density ratio 100.
THROUGHPUT = Workload("many_drops_16384", 16384, 16384, rho_A=100.0, rho_B=1.0, nu_A=0.1,
                      nu_B=0.1, sigma=5e-4, W=4.0, M=0.05, steps=1000,
                      extra={"ndrops": 2000, "rmin": 20.0, "rmax": 80.0})
# Adjoint inverse problem: 1024^2 two drops R 100, density ratio 100.
ADJOINT = Workload("adjoint_1024", 1024, 1024, rho_A=100.0, rho_B=1.0, nu_A=0.1, nu_B=0.1,
                   sigma=1e-3, W=5.0, M=0.05, steps=2000, extra={"R": 100.0, "K": 100})

WORKLOADS = {1: FLAT, 2: DROPLET, 3: COALESCENCE, 4: THROUGHPUT, 5: ADJOINT}
