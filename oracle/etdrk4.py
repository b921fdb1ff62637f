"""FP64 time integrator for the dealiased semi-discrete KS equation
du_hat/dt = A_k u_hat + N(u_hat), used to build integral curves (curves with a
discrete residual that vanishes as the s-grid is refined) and trajectory
endpoints for the batched workload.

Test infrastructure only (see the package docstring).

Scheme: the fourth-order exponential time-differencing Runge-Kutta method of
Cox & Matthews (J. Comput. Phys. 176, 2002), with the phi-function
coefficients evaluated by a contour average around each h A_k as proposed by
Kassam & Trefethen (SIAM J. Sci. Comput. 26, 2005) to avoid cancellation for
small |h A_k|.  Written from those papers' formulas.

Parity: pinned against the exact linear solution (small amplitude) and against
an independent classical RK4 run with a much smaller step.
"""
from __future__ import annotations

import numpy as np

from .ks import Curve, to_physical, to_spectral


def _nonlinear(c: Curve, Uh: np.ndarray) -> np.ndarray:
    """-u u_x of eq. KSE, dealiased: -1/2 d_x (u^2) formed in physical space."""
    u = to_physical(Uh[None, :], c.n_x)[0]
    return -0.5j * c.q * to_spectral(u * u, c.K)


def etdrk4_coeffs(A: np.ndarray, h: float, n_contour: int = 64):
    """Exponentials and phi-combinations of the Cox-Matthews scheme for the
    diagonal linear symbol A and step h."""
    z = h * np.asarray(A, dtype=np.float64)
    E = np.exp(z)
    E2 = np.exp(z / 2)
    roots = np.exp(1j * np.pi * (np.arange(1, n_contour + 1) - 0.5) / n_contour)
    Z = z[:, None] + roots[None, :]
    Q = h * np.mean((np.exp(Z / 2) - 1.0) / Z, axis=1).real
    f1 = h * np.mean((-4.0 - Z + np.exp(Z) * (4.0 - 3.0 * Z + Z ** 2)) / Z ** 3, axis=1).real
    f2 = h * np.mean((2.0 + Z + np.exp(Z) * (-2.0 + Z)) / Z ** 3, axis=1).real
    f3 = h * np.mean((-4.0 - 3.0 * Z - Z ** 2 + np.exp(Z) * (4.0 - Z)) / Z ** 3, axis=1).real
    return E, E2, Q, f1, f2, f3


def etdrk4_integrate(c: Curve, u0: np.ndarray, h: float, n_steps: int,
                     sample_every: int = 1) -> np.ndarray:
    """Integrate from coefficients u0 [K+1] for n_steps of size h.

    Returns the samples [n_steps // sample_every + 1, K+1] (the first is u0).
    """
    E, E2, Q, f1, f2, f3 = etdrk4_coeffs(c.A, h)
    v = np.array(u0, dtype=np.complex128)
    v[0] = v[0].real
    out = [v.copy()]
    for n in range(1, n_steps + 1):
        Nv = _nonlinear(c, v)
        a = E2 * v + Q * Nv
        Na = _nonlinear(c, a)
        b = E2 * v + Q * Na
        Nb = _nonlinear(c, b)
        cc = E2 * a + Q * (2.0 * Nb - Nv)
        Nc = _nonlinear(c, cc)
        v = E * v + Nv * f1 + 2.0 * (Na + Nb) * f2 + Nc * f3
        if n % sample_every == 0:
            out.append(v.copy())
    return np.array(out)
