"""Physics of the HIP path.

* The stationary-droplet workload (512^2, density ratio 1000, dynamic
  viscosity ratio 100, sigma 1e-3, W 4, M 0.05, 50000 steps): the Laplace
  law and the spurious velocity, in FP64 and in FP32 deviation storage.
* The paper's flat-interface case (Sec. 3.1): relaxation of the kinetic
  energy to round-off, the slow rise after it, and (at density ratio 10,
  where it completes within a minute) the final decay back to round-off.

At mechanical equilibrium under the potential-form force F = -phi grad mu
(Sec. 2.1), the quantity that jumps by sigma/R across a 2-D drop is
P^ = p + phi mu - psi(phi), psi the double-well of Sec. 2.1 (eq.
bulk_energy); the hydrodynamic p itself stays uniform.  In a 512^2 box the
slowest acoustic mode decays over ~7e4 steps (nu k^2 with nu_B = 0.1), so
a single snapshot of P^ still oscillates by O(1) around the Laplace value;
the test averages the jump over the last 10000 steps (about 15 periods of
the slowest mode, sampled every 20 steps).
"""
import sys

import numpy as np
import pytest
import torch

from harness import gpu_sim
from paper_2311_10827_amd import inputs
from paper_2311_10827_amd.sim import derive

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _laplace_run(R, prec, steps=50000, window=10000, every=20):
    wl = inputs.DROPLET
    n = wl.nx
    jx, jy = inputs.rng_for(2).uniform(-0.5, 0.5, size=2)
    xc, yc = n / 2 + jx, n / 2 + jy
    phi0 = inputs.droplet(n, n, float(R), wl.W, xc, yc)
    sim = gpu_sim(wl, phi0, prec, diag_every=1000)
    d = derive(sim.p)
    X, Y = np.meshgrid(np.arange(n, dtype=float), np.arange(n, dtype=float))
    dx = np.minimum(np.abs(X - xc), n - np.abs(X - xc))
    dy = np.minimum(np.abs(Y - yc), n - np.abs(Y - yc))
    r = np.hypot(dx, dy)
    inner = torch.from_numpy(r < R / 2).cuda()
    outer = torch.from_numpy(r > R + 4 * wl.W).cuda()
    sim.step(steps - window)
    beta = d["beta"]
    jumps, lib_jumps = [], []
    for _ in range(window // every):
        sim.step(every)
        m = sim.moments()
        ph = m["phi"]
        Ph = m["p"] + ph * m["mu"] - beta * (ph - 1.0) ** 2 * (ph + 1.0) ** 2
        jumps.append(float(Ph[inner].mean() - Ph[outer].mean()))
        lib_jumps.append(m["diag"]["laplace_dP"])
    m = sim.moments()
    diag = m.pop("diag")
    ph = m["phi"].cpu().numpy()
    umax = float(torch.sqrt(m["ux"] ** 2 + m["uy"] ** 2).max())
    po, pi = ph[r > R + 4 * wl.W].mean(), ph[r < R / 2].mean()
    reff = np.sqrt(((ph - po) / (pi - po)).sum() / np.pi)
    sim.close()
    return float(np.mean(jumps)), d["sigma"] / reff, umax, diag, float(np.mean(lib_jumps))


@pytest.mark.parametrize("R", inputs.DROPLET.extra["radii"])
def test_laplace_law_and_spurious_velocity(R):
    res = {}
    for prec in (64, 32):
        say(f"[gpu] Laplace law, 512^2 drop R={R}, prec={prec}, 50000 steps")
        jump, law, umax, diag, lib_jump = _laplace_run(R, prec)
        ratio = jump / law
        say(f"  dP^/(sigma/R_eff) = {ratio:.5f} (library's bulk-set jump: {lib_jump / law:.5f}), "
            f"max|u| = {umax:.3e}")
        assert diag["n_nonfinite"] == 0
        assert 0.95 <= ratio <= 1.03, (prec, ratio)
        assert 0.95 <= lib_jump / law <= 1.03, (prec, lib_jump / law)
        assert umax <= 1e-6, (prec, umax)
        res[prec] = jump
    # the FP32 deviation-storage step reproduces the FP64 jump
    assert abs(res[32] - res[64]) <= 1e-3 * abs(res[64])


def test_paper_flat_interface_reaches_round_off_before_its_rise():
    # Sec. 3.1: the 32 x 128 liquid slab (phi in {0, 1}) at density ratio
    # 1000 relaxes from its tanh profile to a kinetic energy at round-off
    # level within 1e6 steps (checkpoints every 1e5; the FP64 step is
    # deterministic: 4.4e-25 with max|u| 1.2e-15 at step 900000 on MI355X).
    # After that minimum a slow mode grows from round-off (the rise the
    # paper describes for its slabs): at 1e6 steps E is already above it.
    from paper_2311_10827_amd.replica import relax
    say("[gpu] paper flat interface, density ratio 1000, 1e6 steps")
    hist = relax("flat", 1000.0, 1_000_000, 100_000)
    k = min(range(len(hist)), key=lambda i: hist[i][1])
    step, E, umax, mu_spread = hist[k]
    say(f"  min E {E:.3e} at step {step}, max|u| {umax:.3e}, mu spread {mu_spread:.3e}; "
        f"E at 1e6 steps {hist[-1][1]:.3e}")
    assert E <= 1e-24
    assert umax <= 1e-14
    assert k < len(hist) - 1 and hist[-1][1] > E


def test_paper_flat_interface_rise_and_final_decay():
    # The whole history the paper describes for its slabs (Sec. 3.1): E
    # falls, rises (here to O(1e-6), from a mode that grows out of round-off),
    # and falls again to round-off.  At density ratio 10 that completes
    # within 6e6 steps (about a minute); the slabs at density ratio 100 and
    # 1000 take far longer (the recorded histories are in the design notes).
    from paper_2311_10827_amd.replica import relax
    say("[gpu] paper flat interface, density ratio 10, 6e6 steps (about a minute)")
    hist = relax("flat", 10.0, 6_000_000, 200_000, log=say)
    # (MI355X: 3.2e-19 at 2e5 steps, a peak of 5.2e-7 at 6e5, back at 8.1e-25
    # by 2.8e6 and at the round-off floor, 1e-31 to 4e-27, from 3e6 on)
    E = [h[1] for h in hist]
    peak = max(range(len(E)), key=lambda i: E[i])
    say(f"  E {E[0]:.3e} at step {hist[0][0]}, peak {E[peak]:.3e} at step {hist[peak][0]}, "
        f"final {E[-1]:.3e} (max|u| {hist[-1][2]:.3e})")
    assert E[0] <= 1e-15                                  # fallen from the start
    assert peak > 0 and E[peak] >= 1e4 * E[0]            # the rise
    late = hist[len(hist) // 2:]                          # the last 3e6 steps
    assert max(h[1] for h in late) <= 1e-25 and max(h[2] for h in late) <= 1e-14  # back at round-off


def test_paper_flat_interface_relaxes_to_round_off_under_mrt():
    # The same slab with the MRT collision (free rates away from BGK's): the
    # discrete equilibrium is still a fixed point, so the kinetic energy
    # still falls to round-off.
    from paper_2311_10827_amd.replica import relax
    say("[gpu] paper flat interface, MRT, density ratio 1000, 1e6 steps")
    hist = relax("flat", 1000.0, 1_000_000, 100_000, collision=1, mrt_f=(1.3, 1.1, 1.6, 1.4),
                 mrt_g=(1.5, 1.7))
    k = min(range(len(hist)), key=lambda i: hist[i][1])
    step, E, umax, mu_spread = hist[k]
    say(f"  min E {E:.3e} at step {step}, max|u| {umax:.3e}, mu spread {mu_spread:.3e}")
    assert E <= 1e-24
    assert umax <= 1e-14

