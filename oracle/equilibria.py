"""Equilibria of the Kuramoto-Sivashinsky equation and their linear stability,
for the end states of the paper's L = 22 connections (Sec. V.D: E0..E3,
Fig. KSE_FPs, Table I).

Test infrastructure only (part of the oracle; see the package docstring).

An equilibrium is a state with f(u) = 0 (eq. KSE, nu = 1), f the dealiased
vector field of ``ks.vector_field``.  E1, E2 and E3 are inversion symmetric
about x = 0 (the paper says so for all three), so they are found by Newton's
method in that subspace, where u_hat_k = i b_k and f maps b to i g(b) with a
real g.  The linear stability of the equilibrium is the spectrum of the
Jacobian of f on the paper's state space, the fields of zero spatial mean
(real coordinates Re u_hat_k, Im u_hat_k for k = 1..K; the mean is conserved
and left out, as in Sec. V.D); Table I lists its eigenvalues with positive
real part.  f is quadratic, so a central difference with any step is its exact
derivative; the Jacobians below use step 1 (no truncation error).

Parity: pinned by Table I (every printed unstable eigenvalue of E1, E2, E3 to
its four decimals), by the zero eigenvalue of the translation mode, by the
discrete symmetries the paper states (E2 under x -> x + L/2, E3 under
x -> x + L/3) and by |f| at the solution.
"""
from __future__ import annotations

import numpy as np

from .ks import Curve, full_to_odd, odd_to_full, vector_field


def _state_curve(n_x: int, L: float) -> Curve:
    # a three-row curve only carries the grid and the Fourier symbols here
    return Curve(3, n_x, L)


def f_odd(c: Curve, b: np.ndarray) -> np.ndarray:
    """g(b) with f(u) = i g(b) for u_hat_k = i b_k (k = 1..K)."""
    F = vector_field(c, odd_to_full(np.asarray(b, dtype=np.float64)[None, :]))[0]
    return F[1:].imag.copy()


def jacobian_odd(c: Curve, b: np.ndarray) -> np.ndarray:
    """dg/db, K x K (exact central differences of the quadratic g)."""
    K = c.K
    J = np.zeros((K, K))
    for j in range(K):
        e = np.zeros(K)
        e[j] = 1.0
        J[:, j] = (f_odd(c, b + e) - f_odd(c, b - e)) / 2.0
    return J


def newton_odd(c: Curve, b0: np.ndarray, tol: float = 1e-13, max_iter: int = 60):
    """Newton's method with step halving on |g| for g(b) = 0; returns
    (b, |g(b)|)."""
    b = np.array(b0, dtype=np.float64)
    res = np.linalg.norm(f_odd(c, b))
    for _ in range(max_iter):
        if res < tol:
            break
        db = np.linalg.solve(jacobian_odd(c, b), -f_odd(c, b))
        lam = 1.0
        while True:
            bn = b + lam * db
            rn = np.linalg.norm(f_odd(c, bn))
            if rn < res or lam < 1e-6:
                break
            lam *= 0.5
        b, res = bn, rn
    return b, res


def _pack(U: np.ndarray) -> np.ndarray:
    return np.concatenate([U[1:].real, U[1:].imag])


def _unpack(x: np.ndarray, K: int) -> np.ndarray:
    U = np.zeros(K + 1, dtype=np.complex128)
    U[1:] = x[:K] + 1j * x[K:]
    return U


def jacobian_full(c: Curve, U: np.ndarray) -> np.ndarray:
    """Jacobian of f on the zero-mean fields in the real coordinates
    (Re u_hat_1..K, Im u_hat_1..K): 2K x 2K, exact central differences.
    U must have zero mean."""
    K = c.K
    U = np.asarray(U, dtype=np.complex128)
    if U[0] != 0:
        raise ValueError("the state space here is the zero-mean fields")
    x0 = _pack(U)
    n = 2 * K
    J = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        fp = vector_field(c, _unpack(x0 + e, K)[None, :])[0]
        fm = vector_field(c, _unpack(x0 - e, K)[None, :])[0]
        J[:, j] = (_pack(fp) - _pack(fm)) / 2.0
    return J


def stability(c: Curve, U: np.ndarray) -> np.ndarray:
    """Eigenvalues of the linearized flow at the state U, largest real part
    first."""
    ev = np.linalg.eigvals(jacobian_full(c, U))
    return ev[np.argsort(-ev.real)]


def equilibrium(n_x: int, L: float, b0: np.ndarray):
    """The inversion-symmetric equilibrium that Newton reaches from b0:
    (U_hat [K+1] complex, |f|)."""
    c = _state_curve(n_x, L)
    b, res = newton_odd(c, b0)
    return odd_to_full(b[None, :])[0], res


__all__ = ["f_odd", "jacobian_odd", "newton_odd", "jacobian_full", "stability", "equilibrium",
           "full_to_odd"]
