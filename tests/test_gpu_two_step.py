"""Two steps per launch (kernel_path 3, FP32 on periodic grids).

k_step2 keeps the intermediate state on chip and must give the bits of two
single fused steps (kernel_path 2): checked after odd and even step counts,
on ragged, tiny and multi-strip grids, in both low-word formats and with the
MRT collision; diagnostics due on a step force single steps around it; a
snapshot taken after a pair (S in the second S plane) restores bit for bit;
the kernel timer counts steps, not launches.  Against the FP64 oracle the
path inherits the FP32 bounds through that bitwise identity, and one direct
comparison is made.
"""
import sys

import numpy as np
import pytest
import torch

from harness import gpu_moments, gpu_sim, gpu_state, oracle_sim
from paper_2311_10827_amd import _lib, inputs
from paper_2311_10827_amd.sim import MRT

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _field(nx, ny, seed=5):
    # interfaces four cells wide: resolved, so that the run stays finite
    # even where the grid is too small to hold the drops
    r = max(4.0, 0.2 * min(nx, ny))
    return inputs.two_drops(nx, ny, r, 4.0, noise=1e-3, workload_id=seed)


def _same(a, b):
    sa, sb = gpu_state(a), gpu_state(b)
    for x, y in zip(sa, sb):
        assert np.isfinite(x).all()
        assert np.array_equal(x, y)


def _pair(nx, ny, n, **over):
    wl = over.pop("wl", inputs.ADJOINT)
    phi0 = _field(nx, ny)
    a = gpu_sim(wl, phi0, 32, kernel_path=3, nx=nx, ny=ny, **over).step(n)
    b = gpu_sim(wl, phi0, 32, kernel_path=2, nx=nx, ny=ny, **over).step(n)
    return a, b


@pytest.mark.parametrize("shape", [(300, 200), (224, 128), (3, 5), (1, 70), (70, 1), (450, 9), (1000, 700)])
@pytest.mark.parametrize("n", [1, 2, 7, 40])
def test_two_step_matches_single_steps_bitwise(shape, n):
    nx, ny = shape
    say(f"[gpu] two-step vs fused {nx}x{ny}, {n} steps")
    a, b = _pair(nx, ny, n)
    assert a.step_count == b.step_count == n
    _same(a, b)


@pytest.mark.parametrize("lo_format", [_lib.LO_16, _lib.LO_32])
@pytest.mark.parametrize("collision", ["bgk", "mrt"])
def test_two_step_formats_and_collisions(lo_format, collision):
    over = dict(lo_format=lo_format)
    if collision == "mrt":
        over.update(collision=MRT, mrt_f=(1.3, 1.1, 1.6, 1.4), mrt_g=(1.5, 1.7))
    say(f"[gpu] two-step vs fused 530x300 lo_format={lo_format} {collision}")
    a, b = _pair(530, 300, 30, **over)
    _same(a, b)


def test_two_step_multi_strip_grid():
    # several rows of strips (the strip height drops to keep the launch
    # wide) and ragged last strips in x and y; compared on the device
    nx, ny = 2300, 1500
    say(f"[gpu] two-step vs fused {nx}x{ny}, 12 steps")
    a, b = _pair(nx, ny, 12, wl=inputs.COALESCENCE)
    for x, y in zip(a.get_state(), b.get_state()):
        assert bool(torch.isfinite(x).all()) and torch.equal(x, y)


def test_two_step_with_diagnostics():
    # diagnostics every 5 steps: the due steps run singly, the rest in pairs
    say("[gpu] two-step with diag_every=5, 23 steps")
    a, b = _pair(300, 200, 23, diag_every=5)
    _same(a, b)
    da, db = a.last_diag(), b.last_diag()
    assert da["step"] == db["step"] == 20
    for k in ("sum_phi", "kinetic_energy", "max_u", "min_rho", "phi_min", "phi_max"):
        assert da[k] == db[k], k


def test_two_step_snapshot_restores_after_a_pair():
    wl, nx, ny = inputs.ADJOINT, 300, 200
    phi0 = _field(nx, ny)
    a = gpu_sim(wl, phi0, 32, kernel_path=3, nx=nx, ny=ny).step(2)   # S in the second plane
    snap = a.snapshot()
    a.step(9)
    ref = gpu_state(a)
    b = gpu_sim(wl, phi0, 32, kernel_path=3, nx=nx, ny=ny)
    b.restore(snap, 2).step(9)
    for x, y in zip(gpu_state(b), ref):
        assert np.array_equal(x, y)
    c = gpu_sim(wl, phi0, 32, kernel_path=2, nx=nx, ny=ny).step(11)
    for x, y in zip(gpu_state(c), ref):
        assert np.array_equal(x, y)


def test_two_step_kernel_timer_counts_steps():
    wl, nx, ny = inputs.ADJOINT, 300, 200
    s = gpu_sim(wl, _field(nx, ny), 32, kernel_path=3, nx=nx, ny=ny)
    s.timing(True)
    s.step(7)
    ms, n = s.kernel_times()
    assert n == 7 and ms > 0


def test_two_step_against_oracle():
    # 512 x 512 crop of the coalescence workload, 1000 steps, to the FP32
    # bounds of the single-step path
    wl = inputs.COALESCENCE
    nx = ny = 512
    phi0 = inputs.two_drops(nx, ny, 80.0, 5.0, noise=1e-3)
    say("[gpu] two-step vs FP64 oracle 512x512, 1000 steps")
    g = gpu_sim(wl, phi0, 32, kernel_path=3, nx=nx, ny=ny).step(1000)
    om = oracle_sim(wl, phi0, nx=nx, ny=ny).step(1000).moments()
    gm, _ = gpu_moments(g)
    err_phi = float(np.abs(gm["phi"] - om["phi"]).max())
    du = max(float(np.abs(gm["ux"] - om["ux"]).max()), float(np.abs(gm["uy"] - om["uy"]).max()))
    say(f"[gpu]   max|dphi| {err_phi:.3e}, max|du| {du:.3e}")
    assert err_phi <= 1e-5 and du <= 1e-6

