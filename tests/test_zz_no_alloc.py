"""lbm_step_noalloc: the step for callers that cannot allocate, with its
diagnostic reductions in the library's per-GPU scratch, against lbm_step on
twin contexts, bit for bit (same kernels, same reduction order): three calls
in a row on different contexts, each on a smaller grid than the one before,
so that each reuses the scratch the one before left behind."""
import sys

import numpy as np
import pytest

from harness import gpu_sim, gpu_state
from paper_2311_10827_amd import _lib, inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


# (nx, ny, precision, kernel_path, diag_every): the fused step, then the
# two-kernel step on a smaller grid, then two steps per launch on a smaller
# one still (diagnostics every 5 steps: steps 1-4 run as two launches of two
# steps each)
CALLS = [(300, 200, 64, 2, 2), (130, 70, 32, 1, 2), (120, 64, 32, 3, 5)]


def test_step_noalloc_matches_step():
    wl = inputs.COALESCENCE
    for nx, ny, prec, path, every in CALLS:
        say(f"[gpu] lbm_step_noalloc vs lbm_step: {nx}x{ny} fp{prec} kernel_path={path}")
        phi0 = inputs.two_drops(nx, ny, 0.15 * nx, 5.0, noise=1e-3, workload_id=3)
        ref = gpu_sim(wl, phi0, prec, diag_every=every, nx=nx, ny=ny, kernel_path=path)
        new = gpu_sim(wl, phi0, prec, diag_every=every, nx=nx, ny=ny, kernel_path=path)
        ref.step(7)
        new.step_noalloc(7)
        for a, b in zip(gpu_state(ref), gpu_state(new)):
            assert np.array_equal(a, b)
        da, db = ref.last_diag(), new.last_diag()
        assert da["ok"] and db["ok"] and da["step"] == db["step"] == 6 // every * every
        assert da == db
        assert new.step_count == ref.step_count == 7
        ref.close()
        new.close()


def test_step_noalloc_rejects_a_grid_beyond_its_scratch():
    # 4096^2 in the two-kernel form: 65536 tiles of diagnostic partials
    # (5.9 MB) do not fit the 4 MiB scratch; the call is refused and no step
    # is taken.  Without diagnostics no scratch is needed and it steps.
    wl = inputs.COALESCENCE
    say("[gpu] lbm_step_noalloc size limit: 4096^2 fp32 two-kernel")
    phi0 = inputs.two_drops(4096, 4096, 400.0, 5.0, workload_id=3)
    g = gpu_sim(wl, phi0, 32, diag_every=1, kernel_path=1)
    with pytest.raises(_lib.LbmError) as e:
        g.step_noalloc(1)
    assert e.value.code == _lib.LBM_EINVAL and "scratch" in str(e.value)
    assert g.step_count == 0
    g.close()
    g = gpu_sim(wl, phi0, 32, diag_every=0, kernel_path=1)
    g.step_noalloc(1)
    assert g.step_count == 1
    g.close()
