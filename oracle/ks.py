"""FP64 NumPy oracle: cost J^2, its adjoint gradient and the descent step for a
discretized Kuramoto-Sivashinsky connecting curve.

Test infrastructure only (see the package docstring).

Notation follows the paper (Ashtari & Schneider, arXiv:2301.11704):
  * u(x, s) is the connecting curve, x in [0, L) periodic, s in R (Sec. II).
  * r = f(u) - du/ds is the residual (Sec. II, eq. residual_definition); for KS
    with nu = 1, r = -u_s - u u_x - u_xx - u_xxxx (Sec. V.A, eq. KSE_residual).
  * J^2 = int int r r dx ds (Sec. II, eq. cost_function_general).
  * L^dagger(u; r) = r_s + u r_x - r_xx - r_xxxx (Sec. V.A; Appendix A) and the
    descent flow du/dtau = -L^dagger(u; r) (eq. KSE_G).
  * Fourier modes in x with x_n = n L / N (Sec. V.C.1).

Discretization choices where the paper leaves room (each is a stated reading):
  * The state holds the Fourier coefficients u_hat_k, k = 0..K, of every s-row,
    K = floor((N_x - 1) / 3) (2/3-rule dealiasing; mode 0 real; negative modes
    by Hermitian symmetry).  Physical fields live on N_x points.
  * s is reached through a uniform computational coordinate sigma_j = j/(N_s-1).
    The rational map is the paper's s = s0 + S cot(theta) (Sec. IV,
    eq. Rational_domain) with theta = pi (1 - sigma), so row 0 is s = -inf and
    row N_s-1 is s = +inf (the paper numbers the other way round).  The metric
    g = d sigma / d s = sin^2(theta) / (pi S) is the diagonal factor of the
    paper's differentiation matrix (eq. rational_diff_matrix).  The finite map
    s = T sigma has g = 1/T.
  * d/ds of a row quantity q is g_j (q_{j+1} - q_{j-1}) / (2 dsigma)
    (ds = "stencil"), or the paper's rational Chebyshev differentiation matrix
    D_t applied along s (ds = "spectral", rational map only; Sec. IV,
    eq. rational_diff_matrix).
  * int ds is the trapezoid rule in sigma with weights w_j = dsigma / g_j over
    the interior rows; r and G vanish on the two end rows (Sec. V.C.1).
"""
from __future__ import annotations

import numpy as np


def n_modes(n_x: int) -> int:
    """Number of kept Fourier modes K+1, K = floor((N_x - 1)/3) (2/3 rule)."""
    return (n_x - 1) // 3 + 1


class Curve:
    """Grid, metric and Fourier symbols of one curve.

    Parity: ``A`` is pinned by the E0 row of Table I (the unstable eigenvalues
    of u = 0 are A_k for the modes with A_k > 0); ``g`` by the metric test
    against the analytic derivative of tanh and against the paper's D_t.
    """

    def __init__(self, n_s: int, n_x: int, L: float, map: str = "rational",
                 scale: float = 40.0, s0: float = 0.0, ds: str = "stencil"):
        if n_s < 3:
            raise ValueError("need at least 3 rows")
        if ds not in ("stencil", "spectral"):
            raise ValueError(ds)
        if ds == "spectral" and map != "rational":
            raise ValueError("the spectral d/ds is the rational Chebyshev one (rational map)")
        self.ds = ds
        self.n_s, self.n_x, self.L = int(n_s), int(n_x), float(L)
        self.map, self.scale, self.s0 = map, float(scale), float(s0)
        self.K = (self.n_x - 1) // 3
        k = np.arange(self.K + 1, dtype=np.float64)
        # wavenumbers of the Fourier modes exp(i 2 pi k x / L) (Sec. V.C.1)
        self.q = 2.0 * np.pi * k / self.L
        # Fourier symbol of -d_xx - d_xxxx (eq. KSE with nu = 1): (iq)^2 -> -q^2, (iq)^4 -> q^4
        self.A = self.q ** 2 - self.q ** 4
        # weight of mode k in int_0^L a b dx = L sum_{|k|<=K} a_k conj(b_k)
        self.c = np.full(self.K + 1, 2.0)
        self.c[0] = 1.0
        self.sigma = np.arange(self.n_s, dtype=np.float64) / (self.n_s - 1)
        self.dsigma = 1.0 / (self.n_s - 1)
        if map == "rational":
            theta = np.pi * (1.0 - self.sigma)
            with np.errstate(divide="ignore"):
                self.s = self.s0 + self.scale * np.cos(theta) / np.sin(theta)
            self.s[0], self.s[-1] = -np.inf, np.inf
            self.g = np.sin(theta) ** 2 / (np.pi * self.scale)
            self.g[0] = self.g[-1] = 0.0
        elif map == "finite":
            self.s = self.scale * self.sigma
            self.g = np.full(self.n_s, 1.0 / self.scale)
        else:
            raise ValueError(map)
        self.w = np.zeros(self.n_s)
        self.w[1:-1] = self.dsigma / self.g[1:-1]
        if ds == "spectral":
            # the paper's D_t numbers its points from s = +inf; rows here run
            # from s = -inf, so both indices are reversed
            self.D = rational_Dt(self.n_s - 2, self.scale)[::-1, ::-1].copy()

    @property
    def shape(self):
        return (self.n_s, self.K + 1)


# ----------------------------------------------------------------------------
# Fourier transforms between the K+1 kept modes and the N_x-point grid
# (Sec. V.C.1: u(x_n) = sum_j u_hat_j exp(2 pi i j x_n / L), x_n = n L / N).
# ----------------------------------------------------------------------------

def to_physical(Uh: np.ndarray, n_x: int) -> np.ndarray:
    """u_n = sum_{|k|<=K} u_hat_k e^{2 pi i k n / N}, row-wise, via numpy's irfft.

    Parity: pinned against the brute-force sum ``dft_to_physical``.
    """
    Uh = np.atleast_2d(Uh)
    X = np.zeros(Uh.shape[:-1] + (n_x // 2 + 1,), dtype=np.complex128)
    X[..., :Uh.shape[-1]] = Uh
    X[..., 0] = X[..., 0].real
    return np.fft.irfft(X, n=n_x, axis=-1) * n_x


def to_spectral(u: np.ndarray, K: int) -> np.ndarray:
    """u_hat_k = (1/N) sum_n u_n e^{-2 pi i k n / N} for k = 0..K, via numpy's rfft.

    Parity: pinned against ``dft_to_spectral``.
    """
    n_x = u.shape[-1]
    return np.fft.rfft(u, axis=-1)[..., :K + 1] / n_x


def dft_to_physical(Uh: np.ndarray, n_x: int) -> np.ndarray:
    """Brute-force O(N K) version of ``to_physical`` (independent check)."""
    Uh = np.atleast_2d(Uh)
    K = Uh.shape[-1] - 1
    n = np.arange(n_x)
    out = np.zeros(Uh.shape[:-1] + (n_x,))
    for k in range(0, K + 1):
        e = np.exp(2j * np.pi * k * n / n_x)
        if k == 0:
            out += Uh[..., 0:1].real * np.ones(n_x)
        else:
            # u_k e^{ikx} + conj(u_k) e^{-ikx} = 2 Re(u_k e^{ikx})
            out += 2.0 * (Uh[..., k:k + 1] * e).real
    return out


def dft_to_spectral(u: np.ndarray, K: int) -> np.ndarray:
    """Brute-force O(N K) version of ``to_spectral`` (independent check)."""
    n_x = u.shape[-1]
    n = np.arange(n_x)
    out = np.zeros(u.shape[:-1] + (K + 1,), dtype=np.complex128)
    for k in range(K + 1):
        out[..., k] = (u * np.exp(-2j * np.pi * k * n / n_x)).sum(axis=-1) / n_x
    return out


def _clean(c: Curve, U: np.ndarray) -> np.ndarray:
    U = np.array(U, dtype=np.complex128, copy=True)
    if U.shape != c.shape:
        raise ValueError(f"state shape {U.shape} != {c.shape}")
    U[:, 0] = U[:, 0].real  # mode 0 of a real field is real
    return U


def _dx(c: Curve, Uh: np.ndarray) -> np.ndarray:
    """Spectral x-derivative: Hadamard product with (2 pi i k / L) (Sec. V.C.1)."""
    return 1j * c.q * Uh


def _dxx(c: Curve, Uh: np.ndarray) -> np.ndarray:
    """Second x-derivative: multiplier (i q)^2 = -q^2."""
    return -(c.q ** 2) * Uh


def _dxxxx(c: Curve, Uh: np.ndarray) -> np.ndarray:
    """Fourth x-derivative: multiplier (i q)^4 = q^4."""
    return (c.q ** 4) * Uh


def _ds(c: Curve, Q: np.ndarray) -> np.ndarray:
    """d/ds on interior rows: g_j (q_{j+1} - q_{j-1}) / (2 dsigma), or D_t q for
    the spectral variant; zero on end rows."""
    out = np.zeros_like(Q)
    if c.ds == "spectral":
        out[1:-1] = (c.D @ Q)[1:-1]
        return out
    out[1:-1] = c.g[1:-1, None] * (Q[2:] - Q[:-2]) / (2.0 * c.dsigma)
    return out


def _ds_adjoint(c: Curve, R: np.ndarray) -> np.ndarray:
    """The s-part of L^dagger: the adjoint of -d/ds in the inner product <p, q>
    (weights w_j on the interior rows) applied to r, zero on the end rows.

    Stencil: this is +g_j (r_{j+1} - r_{j-1}) / (2 dsigma), the paper's r_s (the
    discrete and the continuous adjoint coincide for the central difference
    with trapezoid weights).  Spectral: -(1/w_i) sum_j D_t[j, i] w_j r_j, the
    exact discrete adjoint of -D_t; it agrees with D_t r up to the quadrature
    error of the trapezoid rule.
    """
    if c.ds == "stencil":
        return _ds(c, R)
    out = np.zeros_like(R)
    out[1:-1] = -(c.D.T @ (c.w[:, None] * R))[1:-1] / c.w[1:-1, None]
    return out


# ----------------------------------------------------------------------------
# The KS vector field, the residual and the cost.
# ----------------------------------------------------------------------------

def vector_field(c: Curve, Uh: np.ndarray) -> np.ndarray:
    """f(u) = -u u_x - u_xx - u_xxxx (eq. KSE, nu = 1) for each row, dealiased.

    The product u u_x is formed in physical space (Sec. V.C.1) and truncated to
    k <= K.  Parity: pinned by the single-mode closed form of f.
    """
    u = to_physical(Uh, c.n_x)
    ux = to_physical(_dx(c, Uh), c.n_x)
    nonlin = -to_spectral(u * ux, c.K)
    return nonlin - _dxx(c, Uh) - _dxxxx(c, Uh)


def residual(c: Curve, U: np.ndarray) -> np.ndarray:
    """r = f(u) - du/ds (eq. residual_definition / KSE_residual) on interior rows;
    r = 0 on the two end rows (Sec. V.C.1).

    Parity: pinned by the integral-curve test (J -> 0 at order 2 in dsigma on a
    sampled KS trajectory) and by a closed-form separable curve.
    """
    U = _clean(c, U)
    R = vector_field(c, U) - _ds(c, U)
    R[0] = 0.0
    R[-1] = 0.0
    return R


def inner(c: Curve, P: np.ndarray, Q: np.ndarray) -> float:
    """<p, q> = int int p q dx ds (Sec. III): trapezoid in sigma with weights
    w_j = dsigma / g_j, Parseval in x (L sum_k c_k Re(p_k conj(q_k)))."""
    row = (c.c[None, :] * (P * np.conj(Q)).real).sum(axis=1) * c.L
    return float((c.w * row).sum())


def J2(c: Curve, U: np.ndarray) -> float:
    """J^2 = <r, r> (eq. cost_function_general).  Parity: pinned by the
    integral-curve test and the separable closed form."""
    R = residual(c, U)
    return inner(c, R, R)


def _row_norm(c: Curve, Q: np.ndarray) -> np.ndarray:
    """|q| = sqrt(int_0^L q q dx) per row (the norm under eq. J_arc)."""
    return np.sqrt(c.L * (c.c[None, :] * np.abs(Q) ** 2).sum(axis=1))


def J_arc(c: Curve, U: np.ndarray) -> float:
    """Arc-length weighted cost (eq. J_arc):
        int |r| |u_s| ds / int |u_s| ds.
    With ds = dsigma / g and u_s = g u_sigma the metric cancels; both integrals
    are taken with the trapezoid rule over the interior rows.

    Parity: pinned against the integral itself, evaluated by adaptive
    quadrature in s for closed-form curves on the rational map (first-order
    convergence: the end rows' share of the denominator is left out, and a
    Richardson step converges at second order) and with the spectral d/ds
    (convergence faster than any power of N_s); weighting the rows by g or
    1/g, or dropping or inverting w in the spectral branch, fails those pins.
    """
    U = _clean(c, U)
    R = residual(c, U)
    if c.ds == "spectral":
        # |u_s| ds = |D_t u|_j w_j on the interior rows
        Us = _ds(c, U)
        a = _row_norm(c, R)[1:-1]
        b = _row_norm(c, Us)[1:-1] * c.w[1:-1]
        den = b.sum()
        return float((a * b).sum() / den) if den > 0 else float("nan")
    Dsig = np.zeros_like(U)
    Dsig[1:-1] = (U[2:] - U[:-2]) / (2.0 * c.dsigma)
    a = _row_norm(c, R)[1:-1]
    b = _row_norm(c, Dsig)[1:-1]
    den = b.sum()
    return float((a * b).sum() / den) if den > 0 else float("nan")


# ----------------------------------------------------------------------------
# Directional derivative, its adjoint, the gradient and the descent step.
# ----------------------------------------------------------------------------

def jvp(c: Curve, U: np.ndarray, V: np.ndarray) -> np.ndarray:
    """Directional derivative of r along v (Appendix A, eq.
    KSE_directional_derivative): -v_s - (u v)_x - v_xx - v_xxxx, zero on end rows.

    Parity: pinned by central differences of ``residual`` (r is quadratic in u,
    so the central difference is exact up to rounding).
    """
    U = _clean(c, U)
    V = np.array(V, dtype=np.complex128)
    V[:, 0] = V[:, 0].real
    u = to_physical(U, c.n_x)
    v = to_physical(V, c.n_x)
    uv = to_spectral(u * v, c.K)
    out = -_ds(c, V) - _dx(c, uv) - _dxx(c, V) - _dxxxx(c, V)
    out[0] = 0.0
    out[-1] = 0.0
    return out


def adjoint(c: Curve, U: np.ndarray, R: np.ndarray | None = None) -> np.ndarray:
    """L^dagger(u; r) = r_s + u r_x - r_xx - r_xxxx (Sec. V.A; Appendix A), with r
    zero on the end rows and the result zeroed there (G keeps the endpoints).

    Parity: pinned by the adjoint identity <L(u;v), r> = <v, L^dagger(u;r)>
    against ``jvp`` and by Richardson-extrapolated finite differences of J^2.
    """
    U = _clean(c, U)
    if R is None:
        R = residual(c, U)
    u = to_physical(U, c.n_x)
    rx = to_physical(_dx(c, R), c.n_x)
    out = _ds_adjoint(c, R) + to_spectral(u * rx, c.K) - _dxx(c, R) - _dxxxx(c, R)
    out[0] = 0.0
    out[-1] = 0.0
    return out


def grad(c: Curve, U: np.ndarray) -> np.ndarray:
    """Euclidean gradient of J^2 with respect to the real and imaginary parts of
    the stored coefficients, returned as a complex array
        G.real = dJ^2 / d Re u_hat_{jk},  G.imag = dJ^2 / d Im u_hat_{jk}.
    dJ^2 = 2 <r, L(u; du)> = 2 <L^dagger r, du> (eq. rate_of_J_with_adjoint), so
    G_{jk} = 2 w_j L c_k L^dagger_{jk}; zero on the end rows and for Im of mode 0.

    Parity: pinned by Richardson-extrapolated central differences of ``J2``
    (exact up to rounding because J^2 is a quartic polynomial of the state).
    """
    Ad = adjoint(c, U)
    G = 2.0 * c.w[:, None] * c.L * c.c[None, :] * Ad
    G[:, 0] = G[:, 0].real
    return G


def step(c: Curve, U: np.ndarray, dtau: float) -> np.ndarray:
    """One semi-implicit forward-Euler step of du/dtau = -L^dagger(u; r)
    (eq. KSE_G; Sec. V.C.3).  The part of G that is linear in u and diagonal in
    Fourier space, -A_k^2 u_hat, is taken implicitly; everything else explicitly:
        u_hat <- u_hat - dtau L^dagger / (1 + dtau A_k^2)   (interior rows).

    Parity: pinned by monotone decrease of J^2, by the first-order rate
    dJ^2/dtau = -2 ||L^dagger r||^2 and by the single-mode closed form.
    """
    U = _clean(c, U)
    Ad = adjoint(c, U)
    out = U - dtau * Ad / (1.0 + dtau * c.A[None, :] ** 2)
    out[0] = U[0]
    out[-1] = U[-1]
    out[:, 0] = out[:, 0].real
    return out


# ----------------------------------------------------------------------------
# Conversions between the physical-grid curve and the spectral state.
# ----------------------------------------------------------------------------

def from_physical_curve(c: Curve, u: np.ndarray) -> np.ndarray:
    """[n_s, N_x] physical samples -> [n_s, K+1] coefficients (truncated)."""
    return to_spectral(np.asarray(u, dtype=np.float64), c.K)


def to_physical_curve(c: Curve, U: np.ndarray) -> np.ndarray:
    """[n_s, K+1] coefficients -> [n_s, N_x] physical samples."""
    return to_physical(_clean(c, U), c.n_x)


# ----------------------------------------------------------------------------
# The paper's spectral differentiation matrix along s (reference operator).
# ----------------------------------------------------------------------------

def rational_Dt(M: int, S: float) -> np.ndarray:
    """D_t of eq. rational_diff_matrix on the M+2 rational Chebyshev points
    s_j = s0 + S cot(j pi / (M+1)) (eq. t_grid; j = 0 is s = +inf).

    Used by the metric test and as the spectral d/ds of ``Curve(ds="spectral")``.
    """
    n = M + 2
    cb = np.ones(n)
    cb[0] = cb[-1] = 2.0
    idx = np.arange(n)
    h = np.pi / (M + 1)
    # angles k j h reduced exactly modulo 2 pi (integer arithmetic) before sin/cos
    ph = (np.outer(idx, idx) % (2 * (M + 1))) * h
    sin_jk = np.sin(ph)                     # [j, k]: sin(k j h)
    cos_mk = np.cos(ph)                     # [m, k]: cos(m k h)
    # D[j, m] = sum_k (k / (cbar_m cbar_k)) cos(m k h) sin(k j h), as one matrix product
    D = (sin_jk * (idx / cb)[None, :]) @ cos_mk.T / cb[None, :]
    D *= (2.0 / (S * (M + 1))) * np.sin(idx * h)[:, None] ** 2
    return D

# ----------------------------------------------------------------------------
# The inversion-symmetric subspace (Sec. V.B: the residual commutes with the
# inversion sigma, so the descent flow eq. KSE_G preserves curves that are
# inversion symmetric about x = 0; the paper's searches run there, Sec. V.D).
# For such a curve u(-x, s) = -u(x, s): every u_hat_k is purely imaginary and
# the mean is zero, u_hat_k = i b_k, k = 1..K.  The state of this subspace holds
# b (K reals per row); the functions below are the full method restricted to it.
# ----------------------------------------------------------------------------

def odd_to_full(B: np.ndarray) -> np.ndarray:
    """[n_s, K] reals b_k -> [n_s, K+1] coefficients u_hat_k = i b_k, u_hat_0 = 0."""
    B = np.asarray(B, dtype=np.float64)
    U = np.zeros((B.shape[0], B.shape[1] + 1), dtype=np.complex128)
    U[:, 1:] = 1j * B
    return U


def full_to_odd(U: np.ndarray) -> np.ndarray:
    """[n_s, K+1] coefficients -> b_k = Im u_hat_k, k = 1..K."""
    return np.asarray(U)[:, 1:].imag.astype(np.float64)


def J2_odd(c: Curve, B: np.ndarray) -> float:
    """J^2 of the inversion-symmetric curve b."""
    return J2(c, odd_to_full(B))


def J_arc_odd(c: Curve, B: np.ndarray) -> float:
    """J_arc of the inversion-symmetric curve b."""
    return J_arc(c, odd_to_full(B))


def grad_odd(c: Curve, B: np.ndarray) -> np.ndarray:
    """dJ^2/db_k: the imaginary part of the full Euclidean gradient (its real
    part and mode 0 vanish on the subspace)."""
    return full_to_odd(grad(c, odd_to_full(B)))


def step_odd(c: Curve, B: np.ndarray, dtau: float) -> np.ndarray:
    """One semi-implicit step of eq. KSE_G, which stays in the subspace."""
    return full_to_odd(step(c, odd_to_full(B), dtau))


# ----------------------------------------------------------------------------
# A descent step with the s-part of the linear operator implicit as well (an
# extension of the semi-implicit scheme of Sec. V.C.3; not in the paper).
# ----------------------------------------------------------------------------

def implicit_s_operator(c: Curve, k: int) -> np.ndarray:
    """The part of L^dagger(u; r(u)) that is linear in the interior rows of
    mode k, as an (n_s - 2) x (n_s - 2) matrix B_k acting on those rows:

        B_k = A_k^2 I - D m D,

    D the central difference of ``_ds`` on the interior rows (reading the
    neighbour rows) and m the mask that zeroes the end rows of the residual
    before the second d/ds.  The residual's linear part is A u - u_s and the
    adjoint's is r_s + A r, so the cross terms A u_s cancel and what remains
    is A^2 u - (m u_s)_s; couplings of an interior row to the fixed end rows
    are constants, not part of B_k.  Stencil d/ds only.

    Parity: pinned by the Jacobian of ``adjoint`` at u = 0 (central
    differences, exact for the polynomial map up to rounding).
    """
    if c.ds != "stencil":
        raise ValueError("the banded operator is the central-difference one")
    n = c.n_s
    ni = n - 2
    beta = np.zeros(n)
    beta[1:-1] = c.g[1:-1] / (2.0 * c.dsigma)   # d/ds at row j: beta_j (q_{j+1} - q_{j-1})
    # first derivative on the interior rows, as a map from all rows
    Dfull = np.zeros((n, n))
    for j in range(1, n - 1):
        Dfull[j, j + 1] = beta[j]
        Dfull[j, j - 1] = -beta[j]
    DmD = Dfull @ Dfull          # rows and columns of the end rows of the inner D are zero
    B = c.A[k] ** 2 * np.eye(ni) - DmD[1:-1, 1:-1]
    return B


def step_implicit_s(c: Curve, U: np.ndarray, dtau: float) -> np.ndarray:
    """One linearly implicit Euler step of du/dtau = -L^dagger(u; r) in which
    the whole linear part B_k of ``implicit_s_operator`` is implicit (the
    paper's step makes only A_k^2 implicit):

        (I + dtau B_k) delta_k = -dtau L^dagger_k,   u_hat <- u_hat + delta

    on the interior rows of every mode k; end rows unchanged, Im of mode 0
    zero.  B_k is self-adjoint and positive semi-definite in the weighted
    inner product, so -delta is a descent direction for J^2 at any dtau > 0,
    and fixed points are those of the paper's flow.

    Parity: pinned through ``implicit_s_operator``; the step itself by its
    first-order agreement with ``step`` as dtau -> 0 and by monotone decrease
    of J^2.
    """
    U = _clean(c, U)
    return U + solve_implicit_s(c, adjoint(c, U), dtau)


def solve_implicit_s(c: Curve, Ad: np.ndarray, dtau: float) -> np.ndarray:
    """The increment of ``step_implicit_s`` for the adjoint field Ad:
    (I + dtau B_k) delta_k = -dtau Ad_k on the interior rows of every mode k;
    zero on the end rows and for Im of mode 0."""
    delta = np.zeros_like(Ad, dtype=np.complex128)
    ni = c.n_s - 2
    if ni <= 0:
        return delta
    for k in range(c.K + 1):
        M = np.eye(ni) + dtau * implicit_s_operator(c, k)
        delta[1:-1, k] = np.linalg.solve(M, -dtau * Ad[1:-1, k])
    delta[:, 0] = delta[:, 0].real
    return delta


def precondition_implicit_s(c: Curve, G: np.ndarray, dtau: float) -> np.ndarray:
    """The implicit-in-s increment for a given Euclidean gradient G (the
    layout of ``grad``): ``solve_implicit_s`` of L^dagger = G / (2 w_j L c_k)
    on the interior rows.  As a map of the stored real and imaginary parts it
    is -H0 G with H0 = dtau (I + dtau B)^{-1} (2 w L c)^{-1}: B is
    self-adjoint and positive semi-definite in the w-weighted inner product,
    so H0 is symmetric positive definite in the plain Euclidean one (the
    initial inverse Hessian of a quasi-Newton method over the state, whose
    gradient is G).

    Parity: pinned by the symmetry and positivity of H0 in the Euclidean
    inner product (tests/test_oracle_implicit_s.py) and, through
    ``step_implicit_s``, by the Jacobian pin of ``implicit_s_operator``.
    """
    Ad = np.zeros_like(G, dtype=np.complex128)
    if c.n_s > 2:
        Ad[1:-1] = G[1:-1] / (2.0 * c.w[1:-1, None] * c.L * c.c[None, :])
    return solve_implicit_s(c, Ad, dtau)


def step_implicit_s_odd(c: Curve, B: np.ndarray, dtau: float) -> np.ndarray:
    """``step_implicit_s`` of the inversion-symmetric curve b (B_k is real and
    acts per mode, so the step stays in the subspace)."""
    return full_to_odd(step_implicit_s(c, odd_to_full(B), dtau))


def descend_implicit_s_momentum(c: Curve, U: np.ndarray, n: int, dtau: float, beta: float,
                                storage=None) -> np.ndarray:
    """n implicit-in-s steps with heavy-ball momentum (Polyak's two-step
    iteration; an acceleration beyond the paper's scheme):

        u_{i+1} = step_implicit_s(u_i) + beta (u_i - u_{i-1}),  u_{-1} = u_0,

    the momentum term on the interior rows only (end rows fixed, Im of mode 0
    zero), and dropped for a step whose input cost rose against the previous
    input's, J^2(u_i) > J^2(u_{i-1}) (1 + 1e-12) (an adaptive restart).
    storage = np.float32 rounds each new state to FP32 (what an FP32 state
    holds between steps).

    Parity: with beta = 0 it is n steps of ``step_implicit_s``; the momentum
    term and the restart are the definitions above.
    """
    prev = _clean(c, U)
    cur = prev.copy()
    J_prev = np.nan
    for _ in range(n):
        J_cur = J2(c, cur)
        nxt = step_implicit_s(c, cur, dtau)
        if not (np.isfinite(J_prev) and J_cur > J_prev * (1.0 + 1e-12)):
            nxt[1:-1] += beta * (cur[1:-1] - prev[1:-1])
        nxt[:, 0] = nxt[:, 0].real
        if storage is not None and np.dtype(storage) == np.float32:
            nxt = nxt.astype(np.complex64).astype(np.complex128)
        prev, cur, J_prev = cur, nxt, J_cur
    return cur
