"""Adjoint of the step (HIP, through the C ABI) against the oracle's
tangent-linear model and against finite differences.

Dot-product test: for the step map s_{n+1} = Phi(s_n; theta),
    <lambda_{n+1}, J v + J_theta dtheta> = <J^T lambda_{n+1}, v> + <J_theta^T lambda_{n+1}, dtheta>,
with J v from the oracle run over dual numbers (exact forward-mode
derivative of the FP64 oracle) and J^T lambda from the GPU adjoint kernels.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from harness import gpu_sim
from paper_2311_10827_amd import inputs
from paper_2311_10827_amd.adjoint import misfit, params_from_theta, rollout
from paper_2311_10827_amd.sim import Sim, make_params

pytestmark = pytest.mark.gpu

# oracle tangent order = library gradient order
THETA = ("kappa", "beta", "alpha", "tau_f", "nu_A", "nu_B")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _setup(nx, ny, bcx, bcy, steps=3, seed=0):
    wl = inputs.ADJOINT
    prm = oracle.params_for(wl, nx=nx, ny=ny, bc_x=bcx, bc_y=bcy)
    phi0 = inputs.two_drops(nx, ny, 0.25 * min(nx, ny), 4.0, noise=1e-3)
    o = oracle.Sim(prm).init(phi0).step(steps)
    f, g, Sp = o.get_state()
    gp = make_params(wl, precision=64, nx=nx, ny=ny, bc_x=bcx, bc_y=bcy, kappa=prm.kappa,
                     beta=prm.beta, M=prm.M, alpha=prm.alpha)
    return wl, prm, gp, phi0, (f, g, Sp)


def _lam_pack(f, g, Sp):
    return np.concatenate([f, g, Sp[None]], 0)


def _dot(a, b):
    return float(np.sum(a * b))


@pytest.mark.parametrize("bc", [(0, 0), (1, 0), (1, 1)])
def test_dot_product_one_step(bc):
    nx, ny = 23, 17
    wl, prm, gp, phi0, (f, g, Sp) = _setup(nx, ny, *bc)
    rng = np.random.default_rng(3)
    df = rng.standard_normal(f.shape) * 1e-3
    dg = rng.standard_normal(g.shape) * 1e-5
    dS = rng.standard_normal(Sp.shape) * 1e-6
    lam1 = rng.standard_normal((19, ny, nx))
    say(f"[gpu] adjoint dot product one step bc={bc}")
    # GPU adjoint
    sim = Sim(gp, phi0)
    sim.set_state(f, g, Sp)
    sim.enable_adjoint()
    snap = sim.snapshot()
    lin = torch.from_numpy(lam1).cuda()
    lout = sim.new_adjoint()
    sim.adjoint_step(snap, lin, lout)
    g6 = np.array(sim.adjoint_theta(reset=True))
    lam0 = lout.cpu().numpy()
    # state tangent only
    t = oracle.TLM(prm).set_state(f, df, g, dg, Sp, dS).step(1)
    _, Jf, _, Jg, _, JS = t.get_state()
    lhs = _dot(lam1, _lam_pack(Jf, Jg, JS))
    rhs = _dot(lam0, _lam_pack(df, dg, dS))
    say(f"  state: lhs {lhs:.16e} rhs {rhs:.16e}")
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1e-300)
    # each parameter alone
    scales = np.array([1e-3, 1e-4, 0.1, 0.05, 0.01, 0.01])
    for k in range(6):
        dth = np.zeros(6)
        dth[k] = scales[k]
        t = oracle.TLM(prm, dth).set_state(f, None, g, None, Sp, None).step(1)
        _, Jf, _, Jg, _, JS = t.get_state()
        lhs = _dot(lam1, _lam_pack(Jf, Jg, JS))
        say(f"  {THETA[k]}: lhs {lhs:.16e} rhs {g6[k] * scales[k]:.16e}")
        assert abs(lhs - g6[k] * scales[k]) <= 1e-11 * max(abs(lhs), 1e-300)


@pytest.mark.parametrize("bc", [(0, 0), (1, 1)])
def test_dot_product_init(bc):
    nx, ny = 21, 19
    wl, prm, gp, phi0, _ = _setup(nx, ny, *bc, steps=0)
    rng = np.random.default_rng(4)
    dphi = rng.standard_normal((ny, nx)) * 1e-3
    dth = rng.standard_normal(6) * np.array([1e-3, 1e-4, 0.1, 0.05, 0.01, 0.01])
    lam0 = rng.standard_normal((19, ny, nx))
    say(f"[gpu] adjoint dot product init bc={bc}")
    sim = Sim(gp, phi0)
    sim.enable_adjoint()
    snap = sim.snapshot()
    l0 = torch.from_numpy(lam0).cuda()
    scratch = sim.new_adjoint()
    dphi_adj = sim.adjoint_init(snap, torch.from_numpy(phi0).cuda(), l0, scratch).cpu().numpy()
    g6 = np.array(sim.adjoint_theta(reset=True))
    t = oracle.TLM(prm, dth).init(phi0, dphi)
    _, Jf, _, Jg, _, JS = t.get_state()
    lhs = _dot(lam0, _lam_pack(Jf, Jg, JS))
    rhs = _dot(dphi_adj, dphi) + _dot(g6, dth)
    say(f"  lhs {lhs:.16e} rhs {rhs:.16e}")
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1e-300)


def test_dot_product_multistep_recompute():
    nx, ny, n = 30, 26, 6
    wl, prm, gp, phi0, (f, g, Sp) = _setup(nx, ny, 1, 0, steps=2)
    rng = np.random.default_rng(5)
    df = rng.standard_normal(f.shape) * 1e-3
    dg = rng.standard_normal(g.shape) * 1e-5
    dS = rng.standard_normal(Sp.shape) * 1e-6
    dth = rng.standard_normal(6) * np.array([1e-3, 1e-4, 0.1, 0.05, 0.01, 0.01])
    lamN = rng.standard_normal((19, ny, nx))
    say("[gpu] adjoint dot product, 6 steps recomputed with step_into")
    sim = Sim(gp, phi0)
    sim.set_state(f, g, Sp)
    sim.enable_adjoint()
    states = [sim.snapshot()] + [sim.new_snapshot() for _ in range(n - 1)]
    for k in range(1, n):
        sim.step_into(states[k - 1], states[k])
    lam, other = torch.from_numpy(lamN).cuda(), sim.new_adjoint()
    for k in reversed(range(n)):
        sim.adjoint_step(states[k], lam, other)
        lam, other = other, lam
    g6 = np.array(sim.adjoint_theta(reset=True))
    t = oracle.TLM(prm, dth).set_state(f, df, g, dg, Sp, dS).step(n)
    _, Jf, _, Jg, _, JS = t.get_state()
    lhs = _dot(lamN, _lam_pack(Jf, Jg, JS))
    rhs = _dot(lam.cpu().numpy(), _lam_pack(df, dg, dS)) + _dot(g6, dth)
    say(f"  lhs {lhs:.16e} rhs {rhs:.16e}")
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1e-300)


def test_dot_product_segment_periodic():
    # lbm_adjoint_segment (recompute and reverse sweep in one call) on a
    # periodic grid, against the oracle's tangent model
    nx, ny, n = 30, 26, 6
    wl, prm, gp, phi0, (f, g, Sp) = _setup(nx, ny, 0, 0, steps=2)
    rng = np.random.default_rng(6)
    df = rng.standard_normal(f.shape) * 1e-3
    dg = rng.standard_normal(g.shape) * 1e-5
    dS = rng.standard_normal(Sp.shape) * 1e-6
    dth = rng.standard_normal(6) * np.array([1e-3, 1e-4, 0.1, 0.05, 0.01, 0.01])
    lamN = rng.standard_normal((19, ny, nx))
    say("[gpu] adjoint dot product, one 6-step segment on a periodic grid")
    sim = Sim(gp, phi0)
    sim.set_state(f, g, Sp)
    sim.enable_adjoint()
    snaps = [sim.snapshot()] + [sim.new_snapshot() for _ in range(n - 1)]
    lam, other = torch.from_numpy(lamN).cuda(), sim.new_adjoint()
    out = (lam, other)[sim.adjoint_segment(snaps, lam, other)]
    g6 = np.array(sim.adjoint_theta(reset=True))
    t = oracle.TLM(prm, dth).set_state(f, df, g, dg, Sp, dS).step(n)
    _, Jf, _, Jg, _, JS = t.get_state()
    lhs = _dot(lamN, _lam_pack(Jf, Jg, JS))
    rhs = _dot(out.cpu().numpy(), _lam_pack(df, dg, dS)) + _dot(g6, dth)
    say(f"  lhs {lhs:.16e} rhs {rhs:.16e}")
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1e-300)


@pytest.mark.parametrize("walls", [0, 1])
@pytest.mark.parametrize("collision", ["bgk", "mrt"])
@pytest.mark.parametrize("prec", [64, 32])
def test_segment_equals_single_steps(prec, collision, walls):
    # lbm_adjoint_segment against its recompute and adjoint steps made one
    # call at a time: FP64 to 1e-13 and FP32 to 1e-5 of the largest entry,
    # the parameter gradient to 1e-12 and 1e-4 of its largest entry (the same
    # kernels: equal today, but a segment may order its work differently)
    from paper_2311_10827_amd.sim import MRT
    nx, ny, n = 70, 45, 7
    over = dict(collision=MRT, mrt_f=(1.3, 1.1, 1.6, 1.4), mrt_g=(1.5, 1.7)) if collision == "mrt" else {}
    phi0 = inputs.two_drops(nx, ny, 10.0, 4.0, noise=1e-3, workload_id=5)
    say(f"[gpu] adjoint segment vs single steps, {nx}x{ny} fp{prec} {collision} walls={walls}, {n} steps")
    sim = gpu_sim(inputs.ADJOINT, phi0, prec, nx=nx, ny=ny, bc_x=walls, bc_y=walls, **over)
    sim.step(3)
    sim.enable_adjoint()
    s0 = sim.snapshot()
    lamN = torch.from_numpy(np.random.default_rng(7).standard_normal((19, ny, nx)))
    lamN = lamN.to(device=sim.device, dtype=sim.new_adjoint().dtype)
    states = [s0] + [sim.new_snapshot() for _ in range(n - 1)]
    for k in range(1, n):
        sim.step_into(states[k - 1], states[k])
    lam, other = lamN.clone(), sim.new_adjoint()
    for k in reversed(range(n)):
        sim.adjoint_step(states[k], lam, other)
        lam, other = other, lam
    ref = lam.cpu().numpy().astype(np.float64)
    g_ref = np.array(sim.adjoint_theta(reset=True))
    snaps = [s0] + [sim.new_snapshot() for _ in range(n - 1)]
    a, b = lamN.clone(), sim.new_adjoint()
    out = (a, b)[sim.adjoint_segment(snaps, a, b)].cpu().numpy().astype(np.float64)
    g_seg = np.array(sim.adjoint_theta(reset=True))
    tol, tol_th = (1e-13, 1e-12) if prec == 64 else (1e-5, 1e-4)
    assert np.isfinite(out).all()
    err = np.abs(out - ref).max() / np.abs(ref).max()
    err_th = np.abs(g_seg - g_ref).max() / np.abs(g_ref).max()
    say(f"  max |d lambda| {err:.2e}, max |d theta| {err_th:.2e} (relative to the largest entry)")
    assert err <= tol and err_th <= tol_th


@pytest.mark.parametrize("path", [1, 2])
@pytest.mark.parametrize("prec", [64, 32])
def test_step_into_equals_step_bitwise(prec, path):
    wl = inputs.ADJOINT
    phi0 = inputs.two_drops(90, 70, 14.0, 5.0, noise=1e-3)
    say(f"[gpu] step_into vs step prec={prec} kernel_path={path}")
    sim = gpu_sim(wl, phi0, prec, kernel_path=path, nx=90, ny=70)
    s0 = sim.snapshot()
    a, b = sim.new_snapshot(), sim.new_snapshot()
    sim.step_into(s0, a)
    sim.step_into(a, b)
    sim.step(2)
    c = sim.snapshot()
    assert torch.equal(b, c)
    sim.restore(s0, 0).step(2)
    d = sim.snapshot()
    assert torch.equal(d, c)


def _fd_setup():
    wl = inputs.ADJOINT
    n, R, W = 64, 8.0, 4.0
    base = make_params(wl, precision=64, nx=n, ny=n)
    from paper_2311_10827_amd.sim import derive
    d = derive(base)
    theta = np.array([d["kappa"], d["beta"], base.M, d["tau_f"], d["tau_gA"], d["tau_gB"]])
    phi0 = inputs.two_drops(n, n, R, W, noise=1e-3, workload_id=5)
    # target from hidden (sigma, M) = seeded U(0.5, 2) x nominal (W fixed)
    s1, s2 = inputs.rng_for(5).uniform(0.5, 2.0, size=2)
    th_t = theta.copy()
    th_t[0] *= s1
    th_t[1] *= s1
    th_t[2] *= s2
    return base, theta, th_t, phi0


def _loss(base, theta, phi0, target, nsteps, prec=64):
    p = params_from_theta(base, theta)
    p.precision = prec
    sim = Sim(p, phi0)
    sim.step(nsteps)
    return float(misfit(sim.moments(diag=False)["phi"], target))


def test_rollout_gradient_matches_finite_differences():
    base, theta, th_t, phi0 = _fd_setup()
    nsteps, K = 200, 50
    say("[gpu] rollout gradient vs central differences, 64x64 FP64, 200 steps")
    tgt = Sim(params_from_theta(base, th_t), phi0).step(nsteps).moments(diag=False)["phi"]
    ph = torch.from_numpy(phi0).cuda().requires_grad_(True)
    th = torch.tensor(theta, requires_grad=True)
    L = misfit(rollout(ph, th, base, nsteps, K), tgt)
    L.backward()
    gth = th.grad.numpy()
    gph = ph.grad.cpu().numpy()
    for k in range(6):
        h = 1e-6 * abs(theta[k])
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        fd = (_loss(base, tp, phi0, tgt, nsteps) - _loss(base, tm, phi0, tgt, nsteps)) / (2 * h)
        say(f"  d/d{['kappa', 'beta', 'M', 'tau_f', 'tau_gA', 'tau_gB'][k]}: adjoint {gth[k]:.10e} fd {fd:.10e}")
        assert abs(gth[k] - fd) <= 1e-4 * abs(fd) + 1e-12 * abs(float(L))
    v = np.random.default_rng(9).standard_normal(phi0.shape)
    h = 1e-6
    fd = (_loss(base, theta, phi0 + h * v, tgt, nsteps) - _loss(base, theta, phi0 - h * v, tgt, nsteps)) / (2 * h)
    ad = float(np.sum(gph * v))
    say(f"  d/dphi0 . v: adjoint {ad:.10e} fd {fd:.10e}")
    assert abs(ad - fd) <= 1e-4 * abs(fd)


def test_fp32_gradient_close_to_fp64():
    base, theta, th_t, phi0 = _fd_setup()
    nsteps, K = 200, 64
    say("[gpu] FP32 vs FP64 rollout gradient")
    tgt = Sim(params_from_theta(base, th_t), phi0).step(nsteps).moments(diag=False)["phi"]
    grads = {}
    for prec in (64, 32):
        b = make_params(inputs.ADJOINT, precision=prec, nx=64, ny=64)
        ph = torch.from_numpy(phi0).cuda().requires_grad_(True)
        th = torch.tensor(theta, requires_grad=True)
        misfit(rollout(ph, th, b, nsteps, K), tgt).backward()
        grads[prec] = (th.grad.numpy(), ph.grad.cpu().numpy())
    g64, g32 = grads[64], grads[32]
    say(f"  theta fp64 {g64[0]}\n  theta fp32 {g32[0]}")
    assert np.all(np.abs(g32[0] - g64[0]) <= 2e-3 * np.abs(g64[0]) + 1e-9 * np.abs(g64[0]).max())
    assert np.abs(g32[1] - g64[1]).max() <= 2e-3 * np.abs(g64[1]).max()


@pytest.mark.parametrize("k", range(6))
def test_dot_product_random_configuration(k):
    # one step's transpose on seeded random configurations: sizes, walls,
    # both phi conventions, densities, viscosities, alpha and a body force
    rng = np.random.default_rng(231110827 + 2000 + k)
    nx, ny = int(rng.integers(3, 30)), int(rng.integers(3, 30))
    bcx, bcy = int(rng.integers(2)), int(rng.integers(2))
    phi_B = float(rng.choice([-1.0, 0.0]))
    wl = inputs.Workload(f"adj_random_{k}", nx, ny, bc_x=bcx, bc_y=bcy, phi_A=1.0, phi_B=phi_B,
                         rho_A=float(rng.choice([1.0, 10.0, 100.0])), rho_B=1.0,
                         nu_A=float(rng.uniform(0.03, 0.2)), nu_B=float(rng.uniform(0.03, 0.2)),
                         sigma=float(rng.uniform(1e-3, 1e-2)), W=4.0,
                         M=float(rng.uniform(0.03, 0.2)), alpha=float(rng.choice([0.5, 1.0, 2.0])))
    gx, gy = (float(v) for v in rng.uniform(-1e-5, 1e-5, size=2))
    prm = oracle.params_for(wl, gx=gx, gy=gy)
    phi0 = inputs.two_drops(nx, ny, max(1.0, 0.2 * min(nx, ny)), 4.0, noise=1e-3, workload_id=2000 + k,
                            phi_A=1.0, phi_B=phi_B)
    f, g, Sp = oracle.Sim(prm).init(phi0).step(3).get_state()
    gp = make_params(wl, precision=64, kappa=prm.kappa, beta=prm.beta, gx=gx, gy=gy)
    say(f"[gpu] adjoint dot product, random case {k}: {nx}x{ny} bc=({bcx},{bcy}) phi_B={phi_B}")
    sim = Sim(gp, phi0)
    sim.set_state(f, g, Sp)
    sim.enable_adjoint()
    snap = sim.snapshot()
    lam1 = rng.standard_normal((19, ny, nx))
    lout = sim.new_adjoint()
    sim.adjoint_step(snap, torch.from_numpy(lam1).cuda(), lout)
    g6 = np.array(sim.adjoint_theta(reset=True))
    lam0 = lout.cpu().numpy()
    df = rng.standard_normal(f.shape) * 1e-3
    dg = rng.standard_normal(g.shape) * 1e-5
    dS = rng.standard_normal(Sp.shape) * 1e-6
    t = oracle.TLM(prm).set_state(f, df, g, dg, Sp, dS).step(1)
    _, Jf, _, Jg, _, JS = t.get_state()
    lhs, rhs = _dot(lam1, _lam_pack(Jf, Jg, JS)), _dot(lam0, _lam_pack(df, dg, dS))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1e-300), (lhs, rhs)
    scales = np.array([1e-3, 1e-4, 0.1, 0.05, 0.01, 0.01])
    for q in range(6):
        dth = np.zeros(6)
        dth[q] = scales[q]
        t = oracle.TLM(prm, dth).set_state(f, None, g, None, Sp, None).step(1)
        _, Jf, _, Jg, _, JS = t.get_state()
        lhs = _dot(lam1, _lam_pack(Jf, Jg, JS))
        assert abs(lhs - g6[q] * scales[q]) <= 1e-11 * max(abs(lhs), 1e-300), (THETA[q], lhs, g6[q] * scales[q])


@pytest.mark.parametrize("form", [0, 1, 2])
def test_dot_product_viscosity_forms(form):
    # one step's transpose with nu linear, inverse-linear or exponential in phi
    # (Sec. 2.3.2) at a viscosity ratio of 10, walls in x
    nx, ny = 23, 17
    wl = inputs.Workload("adj_visc", nx, ny, bc_x=1, rho_A=10.0, rho_B=1.0, nu_A=0.03, nu_B=0.2,
                         sigma=5e-3, W=4.0, M=0.05, nu_form=form)
    prm = oracle.params_for(wl)
    phi0 = inputs.two_drops(nx, ny, 4.0, 4.0, noise=1e-3, workload_id=21)
    f, g, Sp = oracle.Sim(prm).init(phi0).step(3).get_state()
    gp = make_params(wl, precision=64, kappa=prm.kappa, beta=prm.beta)
    say(f"[gpu] adjoint dot product, viscosity form {form}")
    sim = Sim(gp, phi0)
    sim.set_state(f, g, Sp)
    sim.enable_adjoint()
    snap = sim.snapshot()
    rng = np.random.default_rng(21 + form)
    lam1 = rng.standard_normal((19, ny, nx))
    lout = sim.new_adjoint()
    sim.adjoint_step(snap, torch.from_numpy(lam1).cuda(), lout)
    g6 = np.array(sim.adjoint_theta(reset=True))
    lam0 = lout.cpu().numpy()
    df = rng.standard_normal(f.shape) * 1e-3
    dg = rng.standard_normal(g.shape) * 1e-5
    dS = rng.standard_normal(Sp.shape) * 1e-6
    _, Jf, _, Jg, _, JS = oracle.TLM(prm).set_state(f, df, g, dg, Sp, dS).step(1).get_state()
    lhs, rhs = _dot(lam1, _lam_pack(Jf, Jg, JS)), _dot(lam0, _lam_pack(df, dg, dS))
    say(f"  state: lhs {lhs:.16e} rhs {rhs:.16e}")
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1e-300), (lhs, rhs)
    for q, scale in ((4, 0.01), (5, 0.01)):
        dth = np.zeros(6)
        dth[q] = scale
        _, Jf, _, Jg, _, JS = oracle.TLM(prm, dth).set_state(f, None, g, None, Sp, None).step(1).get_state()
        lhs = _dot(lam1, _lam_pack(Jf, Jg, JS))
        say(f"  {THETA[q]}: lhs {lhs:.16e} rhs {g6[q] * scale:.16e}")
        assert abs(lhs - g6[q] * scale) <= 1e-11 * max(abs(lhs), 1e-300), (THETA[q], lhs, g6[q] * scale)


@pytest.mark.parametrize("bc", [(0, 0), (1, 0), (1, 1)])
def test_dot_product_mrt(bc):
    # one step's transpose under the MRT collision (rates away from BGK's),
    # with unequal viscosities so that tau_g varies across the interface;
    # periodic and walled grids take different paths in the stencil pass
    nx, ny = 23, 17
    wl = inputs.Workload("adj_mrt", nx, ny, bc_x=bc[0], bc_y=bc[1], rho_A=10.0, rho_B=1.0, nu_A=0.03,
                         nu_B=0.2, sigma=5e-3, W=4.0, M=0.05, alpha=0.8, nu_form=2, collision=1,
                         mrt_f=(1.3, 1.1, 1.6, 1.4), mrt_g=(1.5, 1.7))
    prm = oracle.params_for(wl, gx=3e-6)
    phi0 = inputs.two_drops(nx, ny, 4.0, 4.0, noise=1e-3, workload_id=22)
    f, g, Sp = oracle.Sim(prm).init(phi0).step(3).get_state()
    gp = make_params(wl, precision=64, kappa=prm.kappa, beta=prm.beta, gx=3e-6)
    say(f"[gpu] adjoint dot product, MRT, bc={bc}")
    sim = Sim(gp, phi0)
    sim.set_state(f, g, Sp)
    sim.enable_adjoint()
    snap = sim.snapshot()
    rng = np.random.default_rng(31 + bc[0] + 2 * bc[1])
    lam1 = rng.standard_normal((19, ny, nx))
    lout = sim.new_adjoint()
    sim.adjoint_step(snap, torch.from_numpy(lam1).cuda(), lout)
    g6 = np.array(sim.adjoint_theta(reset=True))
    lam0 = lout.cpu().numpy()
    df = rng.standard_normal(f.shape) * 1e-3
    dg = rng.standard_normal(g.shape) * 1e-5
    dS = rng.standard_normal(Sp.shape) * 1e-6
    _, Jf, _, Jg, _, JS = oracle.TLM(prm).set_state(f, df, g, dg, Sp, dS).step(1).get_state()
    lhs, rhs = _dot(lam1, _lam_pack(Jf, Jg, JS)), _dot(lam0, _lam_pack(df, dg, dS))
    say(f"  state: lhs {lhs:.16e} rhs {rhs:.16e}")
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1e-300), (lhs, rhs)
    scales = np.array([1e-3, 1e-4, 0.1, 0.05, 0.01, 0.01])
    for q in range(6):
        dth = np.zeros(6)
        dth[q] = scales[q]
        _, Jf, _, Jg, _, JS = oracle.TLM(prm, dth).set_state(f, None, g, None, Sp, None).step(1).get_state()
        lhs = _dot(lam1, _lam_pack(Jf, Jg, JS))
        say(f"  {THETA[q]}: lhs {lhs:.16e} rhs {g6[q] * scales[q]:.16e}")
        assert abs(lhs - g6[q] * scales[q]) <= 1e-11 * max(abs(lhs), 1e-300), (THETA[q], lhs, g6[q] * scales[q])


def test_mrt_rollout_gradient_matches_finite_differences():
    # the checkpointed rollout under MRT, against central differences of the
    # GPU forward map (64 x 64 FP64, 200 steps)
    base, theta, th_t, phi0 = _fd_setup()
    base.collision = 1
    for k, r in enumerate((1.3, 1.1, 1.6, 1.4)):
        base.mrt_f[k] = r
    for k, r in enumerate((1.5, 1.7)):
        base.mrt_g[k] = r
    nsteps, K = 200, 50
    say("[gpu] MRT rollout gradient vs central differences, 64x64 FP64, 200 steps")
    tgt = Sim(params_from_theta(base, th_t), phi0).step(nsteps).moments(diag=False)["phi"]
    ph = torch.from_numpy(phi0).cuda().requires_grad_(True)
    th = torch.tensor(theta, requires_grad=True)
    L = misfit(rollout(ph, th, base, nsteps, K), tgt)
    L.backward()
    gth = th.grad.numpy()
    gph = ph.grad.cpu().numpy()
    for k in range(6):
        h = 1e-6 * abs(theta[k])
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        fd = (_loss(base, tp, phi0, tgt, nsteps) - _loss(base, tm, phi0, tgt, nsteps)) / (2 * h)
        say(f"  d/d{['kappa', 'beta', 'M', 'tau_f', 'tau_gA', 'tau_gB'][k]}: adjoint {gth[k]:.10e} fd {fd:.10e}")
        assert abs(gth[k] - fd) <= 1e-4 * abs(fd) + 1e-12 * abs(float(L))
    v = np.random.default_rng(10).standard_normal(phi0.shape)
    h = 1e-6
    fd = (_loss(base, theta, phi0 + h * v, tgt, nsteps) - _loss(base, theta, phi0 - h * v, tgt, nsteps)) / (2 * h)
    ad = float(np.sum(gph * v))
    say(f"  d/dphi0 . v: adjoint {ad:.10e} fd {fd:.10e}")
    assert abs(ad - fd) <= 1e-4 * abs(fd)
