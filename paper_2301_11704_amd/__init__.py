"""MI355X-native hot path of the Jacobian-free variational method for
connecting orbits (Ashtari & Schneider, arXiv:2301.11704) on the
Kuramoto-Sivashinsky equation.

The computation runs in hand-written HIP kernels for gfx950 behind the C ABI
of include/ksc.h (libksc.so, built in-tree by ``paper_2301_11704_amd.build``).
This package is the thin Python binding: ``Problem`` (ABI calls on torch
tensors), ``KSCurveJ2`` (autograd), ``descend_to`` (descent driver with an
FP64 finish).  Importing it does not require a GPU; calling into the library
does, and raises if libksc.so has not been built.
"""
from ._lib import (  # noqa: F401
    KSC_FLAG_INCREASED,
    KSC_FLAG_NONFINITE,
    KSC_LAUNCH_AUTO,
    KSC_LAUNCH_PERSISTENT,
    KSC_LAUNCH_PLAIN,
    KscError,
    LIB_PATH,
)
from .problem import CurveDesc, Problem, n_modes  # noqa: F401
from .autograd import KSCurveJ2, curve_J2  # noqa: F401
