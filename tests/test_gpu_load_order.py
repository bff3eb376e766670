"""The binding in a fresh process that loads the HIP library before anything
imports torch: the step must still run (torch's HIP runtime and the
library's must be one)."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CODE = """
import sys
sys.path.insert(0, {root!r})
from paper_2311_10827_amd import _lib
_lib.load()
from paper_2311_10827_amd import inputs
from paper_2311_10827_amd.sim import Sim, make_params
s = Sim(make_params(inputs.FLAT, precision=64), inputs.flat_interface())
s.step(3)
print("steps", s.step_count, flush=True)
"""


def test_library_loaded_before_torch():
    r = subprocess.run([sys.executable, "-c", CODE.format(root=ROOT)], capture_output=True, text=True,
                       timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "steps 3" in r.stdout
