"""Host-side set-up of the paper's static test cases (Sec. 3.1, 3.2)."""
import numpy as np
import pytest

from paper_2311_10827_amd import replica


@pytest.mark.parametrize("case,shape", [("flat", (128, 32)), ("droplet", (128, 128))])
def test_case_geometry(case, shape):
    wl, phi0 = replica.workload(case, 10.0)
    assert phi0.shape == shape == (wl.ny, wl.nx)
    assert wl.bc_x == wl.bc_y == 0
    # phi in {0, 1}: liquid 1, vapour 0, interfaces at phi = 1/2
    assert (wl.phi_A, wl.phi_B) == (1.0, 0.0)
    assert phi0.max() <= 1.0 and phi0.min() >= 0.0
    if case == "flat":
        col = phi0[:, 0]
        assert np.all(phi0 == col[:, None])              # uniform along x
        assert col[64] > 0.999 and col[0] < 1e-3         # liquid in the middle half
        assert abs(col[32] - 0.5) < 1e-12 and abs(col[96] - 0.5) < 1e-12
    else:
        assert phi0[64, 64] > 0.999 and phi0[0, 0] < 1e-12
        assert abs(phi0[64, 96] - 0.5) < 1e-12          # R = L/4 from the centre


def test_case_parameters():
    wl, _ = replica.workload("droplet", 1000.0)
    assert (wl.rho_A, wl.rho_B, wl.nu_A, wl.nu_B) == (1000.0, 1.0, 0.1, 0.1)
    assert (wl.sigma, wl.W, wl.M, wl.alpha) == (0.005, 4.0, 0.1, 1.0)
    # dynamic viscosity ratio: rho_l nu_l / (rho_v nu_v)
    for mu in (10.0, 100.0, 1000.0):
        wl, _ = replica.workload("flat", 1000.0, mu)
        assert wl.rho_A * wl.nu_A / (wl.rho_B * wl.nu_B) == pytest.approx(mu, rel=1e-15)
    with pytest.raises(ValueError):
        replica.workload("coalescence", 10.0)
