"""MI355X-native hot path of the well-balanced phase-field lattice Boltzmann
model (Ju et al., arXiv 2311.10827): HIP kernels behind the C ABI of
``include/lbmwb.h`` and a thin PyTorch-side binding.

Submodules load lazily: ``inputs`` (seeded initial fields) needs neither
torch nor the HIP library.
"""
import importlib

__all__ = ["Sim", "make_params", "derive", "stream_copy", "inputs"]


def __getattr__(name):
    if name in ("Sim", "make_params", "derive", "stream_copy"):
        return getattr(importlib.import_module(__name__ + ".sim"), name)
    if name in ("inputs", "sim", "adjoint"):
        return importlib.import_module(__name__ + "." + name)
    raise AttributeError(name)
