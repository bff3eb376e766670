"""Seeded random configurations, GPU against the FP64 oracle.

Grid sizes from one cell wide to a few hundred (ragged against every tile
and strip shape), periodic or walled axes, the {-1, 1} and {0, 1}
order-parameter conventions, density ratios 1 to 100, independent
viscosities, mobilities and alpha, and a small uniform body force (Sec.
2.3.2, the G of eq. GGi), which the workload tests leave at zero.  Both step
forms; FP64 to 1e-12 relative, FP32 within the deviation-storage bounds.
"""
import sys

import numpy as np
import pytest

import oracle
from harness import compare_state, gpu_moments, gpu_sim, gpu_state, oracle_sim
from paper_2311_10827_amd import inputs

pytestmark = pytest.mark.gpu

N_CASES = 12


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _config(k):
    rng = np.random.default_rng(231110827 + 1000 + k)
    nx = int(rng.choice([1, 2, 3, 7, 17, 64, 65, 130, 257, 300]))
    ny = int(rng.choice([1, 2, 5, 9, 16, 33, 70, 129, 200]))
    phi_B = float(rng.choice([-1.0, 0.0]))
    wl = inputs.Workload(
        f"random_{k}", nx, ny, bc_x=int(rng.integers(2)), bc_y=int(rng.integers(2)), phi_A=1.0,
        phi_B=phi_B, rho_A=float(rng.choice([1.0, 10.0, 100.0])), rho_B=1.0,
        nu_A=float(rng.uniform(0.02, 0.2)), nu_B=float(rng.uniform(0.02, 0.2)),
        sigma=float(rng.uniform(1e-3, 1e-2)), W=float(rng.choice([3.0, 4.0, 5.0])),
        M=float(rng.uniform(0.02, 0.2)), alpha=float(rng.choice([0.5, 1.0, 2.0])))
    g = rng.uniform(-1e-6, 1e-6, size=2)
    R = max(0.5, 0.22 * min(nx, ny))
    phi0 = inputs.two_drops(nx, ny, R, wl.W, noise=1e-3, workload_id=1000 + k, phi_A=1.0, phi_B=phi_B)
    return wl, phi0, dict(gx=float(g[0]), gy=float(g[1]))


@pytest.mark.parametrize("path", [1, 2])
@pytest.mark.parametrize("k", range(N_CASES))
def test_random_configuration(k, path):
    wl, phi0, over = _config(k)
    say(f"[gpu] random case {k}: {wl.nx}x{wl.ny} bc=({wl.bc_x},{wl.bc_y}) phi_B={wl.phi_B} "
        f"rho_A={wl.rho_A} kernel_path={path}")
    o = oracle_sim(wl, phi0, **over)
    g64 = gpu_sim(wl, phi0, 64, kernel_path=path, **over)
    g32 = gpu_sim(wl, phi0, 32, kernel_path=path, **over)
    for n in (0, 1, 36):
        o.step(n)
        g64.step(n)
        g32.step(n)
        compare_state(gpu_state(g64), o.get_state(), 1e-12)
    om = o.moments()
    m32, d32 = gpu_moments(g32)
    assert d32["n_nonfinite"] == 0
    assert np.abs(m32["phi"] - om["phi"]).max() <= 1e-5
    assert max(np.abs(m32["ux"] - om["ux"]).max(), np.abs(m32["uy"] - om["uy"]).max()) <= 1e-6
    # max |div u|: the stencil's weights sum to 1 in absolute value per
    # derivative, so a velocity error e moves it by at most 2 e
    want = float(np.abs(oracle.divergence(o.prm, om["ux"], om["uy"])).max())
    _, d64 = gpu_moments(g64)
    assert abs(d64["max_div_u"] - want) <= 1e-9 * want + 1e-18
    assert abs(d32["max_div_u"] - want) <= 2e-6


N_VARIANT_CASES = 8


def _variant_config(k):
    # the random configurations above, with a viscosity form and a collision
    # operator drawn too (MRT rates uniform in (0.6, 1.9))
    wl, phi0, over = _config(k)
    rng = np.random.default_rng(231110827 + 3000 + k)
    wl.nu_form = int(rng.integers(3))
    wl.collision = int(rng.integers(2))
    wl.mrt_f = tuple(float(v) for v in rng.uniform(0.6, 1.9, size=4))
    wl.mrt_g = tuple(float(v) for v in rng.uniform(0.6, 1.9, size=2))
    return wl, phi0, over


@pytest.mark.parametrize("path", [1, 2])
@pytest.mark.parametrize("k", range(N_VARIANT_CASES))
def test_random_configuration_viscosity_and_collision(k, path):
    wl, phi0, over = _variant_config(k)
    say(f"[gpu] random variant {k}: {wl.nx}x{wl.ny} bc=({wl.bc_x},{wl.bc_y}) nu_form={wl.nu_form} "
        f"collision={wl.collision} kernel_path={path}")
    o = oracle_sim(wl, phi0, **over)
    g64 = gpu_sim(wl, phi0, 64, kernel_path=path, **over)
    g32 = gpu_sim(wl, phi0, 32, kernel_path=path, **over)
    for n in (0, 1, 36):
        o.step(n)
        g64.step(n)
        g32.step(n)
        compare_state(gpu_state(g64), o.get_state(), 1e-12)
    om = o.moments()
    m32, d32 = gpu_moments(g32)
    assert d32["n_nonfinite"] == 0
    assert np.abs(m32["phi"] - om["phi"]).max() <= 1e-5
    assert max(np.abs(m32["ux"] - om["ux"]).max(), np.abs(m32["uy"] - om["uy"]).max()) <= 1e-6
