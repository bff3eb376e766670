"""Discrete phase equilibrium by Newton's method (test fixture).

Solves, on the lattice and with the same boundary rule as the method, the
discrete equilibrium of the order parameter: the chemical potential
    mu_h(phi) = 4 beta (phi - phi_A)(phi - phi_B)(phi - phi_m) - kappa L_h phi
(Sec. 2.1, eq. chemical_potencial, with the isotropic Laplacian of Sec. 2.3.2,
eq. Laplace) equals an unknown constant mu0 everywhere, with sum(phi) fixed.

Written independently of the oracle and of the HIP path: the sparse
Laplacian below is assembled here from the stencil weights (axis neighbours
weight 4/6, diagonal neighbours 1/6, centre -20/6), and boundary ghosts
mirror the adjacent cell across a wall.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def laplacian_matrix(nx: int, ny: int, wall_x: bool, wall_y: bool) -> sp.csr_matrix:
    n = nx * ny
    rows, cols, vals = [], [], []
    idx = np.arange(n).reshape(ny, nx)
    ys, xs = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    offsets = [(1, 0, 4.0), (-1, 0, 4.0), (0, 1, 4.0), (0, -1, 4.0),
               (1, 1, 1.0), (-1, 1, 1.0), (1, -1, 1.0), (-1, -1, 1.0)]
    for dx, dy, wgt in offsets:
        xx = xs + dx
        yy = ys + dy
        xx = np.clip(xx, 0, nx - 1) if wall_x else xx % nx
        yy = np.clip(yy, 0, ny - 1) if wall_y else yy % ny
        rows.append(idx.ravel())
        cols.append(idx[yy, xx].ravel())
        vals.append(np.full(n, wgt / 6.0))
    rows.append(idx.ravel())
    cols.append(idx.ravel())
    vals.append(np.full(n, -20.0 / 6.0))
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, n))


def solve(phi0: np.ndarray, kappa: float, beta: float, phi_A: float, phi_B: float,
          wall_x: bool = False, wall_y: bool = False, tol: float = 1e-15, maxit: int = 50):
    """Return (phi_star, mu0, residual history)."""
    ny, nx = phi0.shape
    L = laplacian_matrix(nx, ny, wall_x, wall_y)
    pm = 0.5 * (phi_A + phi_B)
    phi = phi0.ravel().astype(np.float64).copy()
    mass = phi.sum()

    def dpsi(p):
        return 4.0 * beta * (p - phi_A) * (p - phi_B) * (p - pm)

    def d2psi(p):
        a, b, c = p - phi_A, p - phi_B, p - pm
        return 4.0 * beta * (a * b + a * c + b * c)

    mu0 = float(np.mean(dpsi(phi) - kappa * (L @ phi)))
    hist = []
    n = phi.size
    ones = sp.csr_matrix(np.ones((1, n)))
    for _ in range(maxit):
        r = dpsi(phi) - kappa * (L @ phi) - mu0
        rm = phi.sum() - mass
        res = max(np.abs(r).max(), abs(rm) / n)
        hist.append(res)
        if res < tol:
            break
        J = sp.diags(d2psi(phi)) - kappa * L
        K = sp.bmat([[J, -sp.csr_matrix(np.ones((n, 1)))], [ones, None]], format="csc")
        d = spla.spsolve(K, -np.concatenate([r, [rm]]))
        phi += d[:n]
        mu0 += d[n]
    return phi.reshape(ny, nx), mu0, hist
