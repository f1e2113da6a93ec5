"""MI355X-native FDTD-Esirkepov PIC step with the small-k_z correction
stencils of Godfrey & Vay (arXiv:1401.0838).

The compute path is libpic.so (hand-written HIP for gfx950) behind the C ABI
of include/pic_api.h; `_lib` is its ctypes binding and `sim.Simulation` the
torch-memory front end.  `fit` holds the growth-rate fit used on the energy
traces.
"""
from . import _lib  # noqa: F401

__all__ = ["_lib", "sim", "fit"]
