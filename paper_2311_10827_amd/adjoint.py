"""Gradient of a phi-snapshot misfit through the HIP forward and adjoint steps.

``rollout(phi0, theta, base, nsteps, K)`` runs ``nsteps`` steps from the
initial order parameter ``phi0`` and returns phi at the final step; it is a
``torch.autograd.Function`` whose backward pass calls the hand-written adjoint
kernels of the C ABI.  Memory: a raw snapshot every K steps in the forward
pass; the backward pass recomputes each segment into K snapshots with
``lbm_step_into`` (no copies) and walks it in reverse.

theta = (kappa, beta, M, tau_f, tau_gA, tau_gB): the free-energy coefficients,
the mobility and the relaxation times, passed to the library as such
(lbm_params.use_tau); the library derives the rest and returns the gradient
in this basis (lbm_adjoint_theta with LBM_THETA_TAU).
"""
from __future__ import annotations

import time

import torch

from . import _lib
from .sim import Sim

THETA_NAMES = ("kappa", "beta", "M", "tau_f", "tau_gA", "tau_gB")


def params_from_theta(base, theta):
    """A copy of the parameter block ``base`` with theta set (argument
    marshalling only)."""
    p = type(base).from_buffer_copy(base)
    p.use_sigma_W = 0
    p.use_tau = 1
    p.kappa, p.beta, p.M, p.tau_f, p.tau_gA, p.tau_gB = (float(v) for v in theta)
    return p


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, phi0, theta, base, nsteps: int, K: int, stats):
        p = params_from_theta(base, theta.detach().cpu().tolist())
        sim = Sim(p, phi0.detach())
        sim.enable_adjoint()
        ckpt = []
        t0 = time.perf_counter()
        for s in range(0, nsteps, K):
            ckpt.append(sim.snapshot())
            sim.step(min(K, nsteps - s))
        phiN = sim.moments(diag=False)["phi"]
        torch.cuda.synchronize()
        if stats is not None:
            stats["forward_s"] = time.perf_counter() - t0
        ctx.sim, ctx.ckpt, ctx.nsteps, ctx.K, ctx.stats = sim, ckpt, nsteps, K, stats
        ctx.theta = theta.detach().cpu().tolist()
        ctx.save_for_backward(phi0)
        return phiN

    @staticmethod
    def backward(ctx, grad_phiN):
        (phi0,) = ctx.saved_tensors
        sim, ckpt, nsteps, K = ctx.sim, ctx.ckpt, ctx.nsteps, ctx.K
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lam = sim.new_adjoint()
        other = sim.new_adjoint()
        # phi = sum_i f_i, so dL/df_i = dL/dphi for every i
        lam[:9] = grad_phiN.to(lam.dtype).unsqueeze(0)
        snaps = [sim.new_snapshot(zeroed=False) for _ in range(min(K, nsteps))]
        for seg, s0 in reversed(list(enumerate(range(0, nsteps, K)))):
            L = min(K, nsteps - s0)
            # recompute the segment's states and walk it backwards in one call
            if sim.adjoint_segment([ckpt[seg]] + snaps[1:L], lam, other) == 1:
                lam, other = other, lam
        dphi0 = sim.adjoint_init(ckpt[0], phi0, lam, other)
        g6 = sim.adjoint_theta(reset=True, basis=_lib.THETA_TAU)
        torch.cuda.synchronize()
        if ctx.stats is not None:
            ctx.stats["backward_s"] = time.perf_counter() - t0
        gth = torch.tensor(g6, dtype=torch.float64)
        return dphi0 * 1.0, gth, None, None, None, None


def rollout(phi0: torch.Tensor, theta: torch.Tensor, base, nsteps: int, K: int = 100, stats=None):
    """phi after ``nsteps`` steps; differentiable in phi0 and theta."""
    return _Rollout.apply(phi0, theta, base, int(nsteps), int(K), stats)


def misfit(phiN: torch.Tensor, target: torch.Tensor) -> torch.Tensor:
    """L = 1/2 sum (phi_N - phi_target)^2 (FP64 accumulation)."""
    d = phiN - target
    return 0.5 * (d * d).sum()
