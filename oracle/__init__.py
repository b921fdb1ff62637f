"""FP64 CPU oracle for the Jacobian-free variational method on the
Kuramoto-Sivashinsky equation (Ashtari & Schneider, arXiv:2301.11704).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The GPU library never
imports it, and it shares no code with the library: it is a plain, slow,
obviously-correct NumPy transcription of the definitions, kept independent so
that agreement between the two means something.

Parity status of each function is stated in its docstring; the pins live in
``tests/test_oracle_*.py``.  Functions with no independent pin say
"parity unpinned".
"""
from .ks import (  # noqa: F401
    Curve,
    n_modes,
    to_physical,
    to_spectral,
    dft_to_physical,
    dft_to_spectral,
    vector_field,
    residual,
    J2,
    J_arc,
    jvp,
    adjoint,
    grad,
    step,
    inner,
    rational_Dt,
    odd_to_full,
    full_to_odd,
    J2_odd,
    J_arc_odd,
    grad_odd,
    step_odd,
    implicit_s_operator,
    step_implicit_s,
    solve_implicit_s,
    precondition_implicit_s,
    step_implicit_s_odd,
    descend_implicit_s_momentum,
    from_physical_curve,
    to_physical_curve,
)
from .etdrk4 import etdrk4_coeffs, etdrk4_integrate  # noqa: F401
