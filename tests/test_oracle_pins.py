"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics
(closed forms, brute force, exact identities, printed values).  CPU only."""
import os

import numpy as np
import pytest

import ksinputs
import oracle
from oracle import Curve

HERE = os.path.dirname(os.path.abspath(__file__))


def _rand_state(c, rng, amp=1.0, kmax=None):
    kmax = c.K if kmax is None else kmax
    U = np.zeros(c.shape, dtype=np.complex128)
    k = np.arange(1, kmax + 1)
    U[:, 1:kmax + 1] = amp * (rng.standard_normal((c.n_s, kmax))
                              + 1j * rng.standard_normal((c.n_s, kmax))) / k ** 2
    U[:, 0] = amp * 0.1 * rng.standard_normal(c.n_s)
    return U


def _rand_interior(c, rng, kmax=None):
    V = _rand_state(c, rng, kmax=kmax)
    V[0] = 0
    V[-1] = 0
    return V


# ---------------------------------------------------------------- Table I ---

def test_table1_E0_row_pins_linear_operator():
    """Unstable eigenvalues of u = 0 at L = 22 are the positive A_k = q^2 - q^4,
    each double (Table I, E0 row).  Pins nu = 1, the sign of both linear terms
    and the L scaling of q."""
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "table1_E0_eigenvalues.txt"))
            if l.strip() and not l.startswith("#")]
    printed = sorted(float(r[1]) for r in rows)
    mult = [int(r[2]) for r in rows]
    c = Curve(8, 64, 22.0)
    pos = sorted(a for a in c.A if a > 0)
    assert len(pos) == len(printed)
    assert all(m == 2 for m in mult)  # +k and -k modes share A_k
    for a, p in zip(pos, printed):
        assert abs(a - p) < 0.5e-4, (a, p)


# ----------------------------------------------------------- transforms ---

@pytest.mark.parametrize("n_x", [8, 16, 32, 64])
def test_transforms_match_brute_force(n_x):
    rng = np.random.default_rng(1)
    K = (n_x - 1) // 3
    Uh = rng.standard_normal((5, K + 1)) + 1j * rng.standard_normal((5, K + 1))
    Uh[:, 0] = Uh[:, 0].real
    u1 = oracle.to_physical(Uh, n_x)
    u2 = oracle.dft_to_physical(Uh, n_x)
    assert np.allclose(u1, u2, atol=1e-12, rtol=0)
    x = rng.standard_normal((5, n_x))
    assert np.allclose(oracle.to_spectral(x, K), oracle.dft_to_spectral(x, K), atol=1e-13, rtol=0)
    # round trip on band-limited data
    assert np.allclose(oracle.to_spectral(u1, K), Uh, atol=1e-12, rtol=0)


def test_products_are_alias_free():
    """A product of two |k|<=K fields truncated to |k|<=K is the same on the
    N_x grid and on a 2N_x grid (the 2/3 rule: N_x > 3K)."""
    rng = np.random.default_rng(2)
    for n_x in (32, 64, 128):
        K = (n_x - 1) // 3
        a = rng.standard_normal((3, K + 1)) + 1j * rng.standard_normal((3, K + 1))
        b = rng.standard_normal((3, K + 1)) + 1j * rng.standard_normal((3, K + 1))
        a[:, 0] = a[:, 0].real
        b[:, 0] = b[:, 0].real
        p1 = oracle.to_spectral(oracle.to_physical(a, n_x) * oracle.to_physical(b, n_x), K)
        p2 = oracle.to_spectral(oracle.to_physical(a, 2 * n_x) * oracle.to_physical(b, 2 * n_x), K)
        assert np.allclose(p1, p2, atol=1e-12, rtol=0)


# ---------------------------------------------------- vector field / KS ---

def _two_mode_field(L, x, a, b):
    """u = a sin(q1 x) + b cos(q2 x) and its x-derivatives in closed form."""
    q1, q2 = 2 * np.pi / L, 4 * np.pi / L
    u = a * np.sin(q1 * x) + b * np.cos(q2 * x)
    ux = a * q1 * np.cos(q1 * x) - b * q2 * np.sin(q2 * x)
    uxx = -a * q1 ** 2 * np.sin(q1 * x) - b * q2 ** 2 * np.cos(q2 * x)
    uxxxx = a * q1 ** 4 * np.sin(q1 * x) + b * q2 ** 4 * np.cos(q2 * x)
    return u, ux, uxx, uxxxx


def _two_mode_coeffs(K, a, b):
    Uh = np.zeros(K + 1, dtype=np.complex128)
    Uh[1] = -0.5j * a   # a sin(q1 x) = a (e^{iq1x} - e^{-iq1x}) / (2i)
    Uh[2] = 0.5 * b     # b cos(q2 x)
    return Uh


@pytest.mark.parametrize("L", [22.0, 39.0])
def test_vector_field_closed_form(L):
    """f(u) = -u u_x - u_xx - u_xxxx (eq. KSE) evaluated pointwise from the
    closed-form derivatives of a two-mode field."""
    n_x = 32
    c = Curve(3, n_x, L)
    x = np.arange(n_x) * L / n_x
    a, b = 0.7, -1.3
    u, ux, uxx, uxxxx = _two_mode_field(L, x, a, b)
    expect = -u * ux - uxx - uxxxx
    Uh = _two_mode_coeffs(c.K, a, b)[None, :]
    got = oracle.to_physical(oracle.vector_field(c, Uh), n_x)[0]
    assert np.allclose(got, expect, atol=1e-12, rtol=0)


@pytest.mark.parametrize("map_,scale", [("finite", 7.0), ("rational", 40.0)])
def test_residual_separable_closed_form(map_, scale):
    """u(x, sigma) = alpha(sigma) sin(q1 x) + beta(sigma) cos(q2 x) with alpha, beta
    quadratic in sigma: the central difference is exact, so r_j(x) has a closed
    form (eq. KSE_residual) with u_s = g alpha'(sigma) sin + g beta'(sigma) cos."""
    L, n_x, n_s = 22.0, 32, 9
    c = Curve(n_s, n_x, L, map_, scale)
    x = np.arange(n_x) * L / n_x
    sig = c.sigma
    al = 0.3 + 1.1 * sig - 0.8 * sig ** 2
    be = -0.5 + 0.2 * sig + 0.9 * sig ** 2
    dal = 1.1 - 1.6 * sig
    dbe = 0.2 + 1.8 * sig
    U = np.array([_two_mode_coeffs(c.K, al[j], be[j]) for j in range(n_s)])
    R = oracle.residual(c, U)
    q1, q2 = 2 * np.pi / L, 4 * np.pi / L
    for j in range(n_s):
        got = oracle.to_physical(R[j:j + 1], n_x)[0]
        if j in (0, n_s - 1):
            assert np.all(got == 0)
            continue
        u, ux, uxx, uxxxx = _two_mode_field(L, x, al[j], be[j])
        us = c.g[j] * (dal[j] * np.sin(q1 * x) + dbe[j] * np.cos(q2 * x))
        expect = -us - u * ux - uxx - uxxxx
        assert np.allclose(got, expect, atol=1e-11, rtol=0)


def test_J2_equals_physical_space_quadrature():
    """J^2 (eq. cost_function_general) equals sum_j w_j * (L/N) sum_n r_j(x_n)^2,
    the rectangle rule in x that is exact for the band-limited r^2; w_j = dsigma/g_j."""
    rng = np.random.default_rng(3)
    c = Curve(12, 32, 22.0)
    U = _rand_state(c, rng)
    R = oracle.residual(c, U)
    r = oracle.dft_to_physical(R, c.n_x)
    dsig = 1.0 / (c.n_s - 1)
    theta = np.pi * (1 - np.arange(c.n_s) * dsig)
    gg = np.sin(theta) ** 2 / (np.pi * 40.0)
    expect = sum(dsig / gg[j] * (c.L / c.n_x) * (r[j] ** 2).sum() for j in range(1, c.n_s - 1))
    assert abs(oracle.J2(c, U) - expect) <= 1e-12 * expect


def test_J_arc_closed_form():
    """Linear blend u = sigma B (finite map): u_sigma = B on every row, so
    J_arc (eq. J_arc) is the plain mean over interior rows of |r_j|, with |r_j|
    from the closed-form residual of a two-mode B."""
    L, n_x, n_s, T = 22.0, 32, 11, 5.0
    c = Curve(n_s, n_x, L, "finite", T)
    x = np.arange(n_x) * L / n_x
    a, b = 0.4, 0.25
    U = np.array([_two_mode_coeffs(c.K, s * a, s * b) for s in c.sigma])
    norms = []
    for j in range(1, n_s - 1):
        s = c.sigma[j]
        u, ux, uxx, uxxxx = _two_mode_field(L, x, s * a, s * b)
        B, *_ = _two_mode_field(L, x, a, b)
        r = -B / T - u * ux - uxx - uxxxx
        norms.append(np.sqrt((r ** 2).sum() * L / n_x))
    assert abs(oracle.J_arc(c, U) - np.mean(norms)) < 1e-12 * np.mean(norms)


# ------------------------------------------------------ derivatives ---

def test_jvp_is_exact_derivative_of_residual():
    """r is quadratic in u, so the central difference of r along v is exact."""
    rng = np.random.default_rng(4)
    c = Curve(10, 16, 22.0)
    U = _rand_state(c, rng)
    V = _rand_interior(c, rng)
    eps = 1e-3
    fd = (oracle.residual(c, U + eps * V) - oracle.residual(c, U - eps * V)) / (2 * eps)
    jv = oracle.jvp(c, U, V)
    assert np.abs(fd - jv).max() <= 1e-9 * np.abs(jv).max()


@pytest.mark.parametrize("map_", ["rational", "finite"])
def test_adjoint_identity(map_):
    """<L(u; v), r> = <v, L^dagger(u; r)> for r, v vanishing on the end rows
    (eq. adjoint_definition; Appendix A)."""
    rng = np.random.default_rng(5)
    c = Curve(14, 32, 39.0, map_, 40.0 if map_ == "rational" else 3.0)
    U = _rand_state(c, rng)
    V = _rand_interior(c, rng)
    R = _rand_interior(c, rng)
    lhs = oracle.inner(c, oracle.jvp(c, U, V), R)
    rhs = oracle.inner(c, V, oracle.adjoint(c, U, R))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)


@pytest.mark.parametrize("map_", ["rational", "finite"])
def test_gradient_matches_richardson_fd(map_):
    """J^2 is a quartic polynomial of the state, so Richardson-extrapolated
    central differences are exact up to rounding; check every free coordinate
    (interior rows; the end rows are pinned and carry no gradient)."""
    rng = np.random.default_rng(6)
    c = Curve(6, 8, 22.0, map_, 40.0 if map_ == "rational" else 2.0)
    U = _rand_state(c, rng, amp=0.5)
    G = oracle.grad(c, U)
    scale = np.abs(G).max()
    eps = 1e-3
    for j in range(1, c.n_s - 1):
        for k in range(c.K + 1):
            for part in (1.0, 1j):
                if k == 0 and part == 1j:
                    continue
                E = np.zeros(c.shape, dtype=np.complex128)
                E[j, k] = part

                def cd(h):
                    return (oracle.J2(c, U + h * E) - oracle.J2(c, U - h * E)) / (2 * h)
                fd = (4 * cd(eps / 2) - cd(eps)) / 3
                got = G[j, k].real if part == 1.0 else G[j, k].imag
                assert abs(fd - got) <= 1e-9 * scale, (j, k, part, fd, got)


def test_gradient_vanishes_on_pinned_rows_and_imag_mode0():
    rng = np.random.default_rng(7)
    c = Curve(8, 16, 22.0)
    G = oracle.grad(c, _rand_state(c, rng))
    assert np.all(G[0] == 0) and np.all(G[-1] == 0)
    assert np.all(G[:, 0].imag == 0)


# --------------------------------------------------------- symmetries ---

def test_translation_and_inversion_symmetry():
    """gamma(alpha) and sigma of eqs. translation/reflection commute with r, so J^2
    is invariant and the gradient is equivariant."""
    rng = np.random.default_rng(8)
    c = Curve(10, 32, 22.0)
    U = _rand_state(c, rng)
    J0 = oracle.J2(c, U)
    G0 = oracle.grad(c, U)
    alpha = 0.137
    ph = np.exp(1j * c.q * alpha * c.L)          # u(x + alpha L)
    Ut = U * ph
    assert abs(oracle.J2(c, Ut) - J0) <= 1e-12 * J0
    assert np.allclose(oracle.grad(c, Ut), G0 * ph, atol=1e-10 * np.abs(G0).max())
    Ui = -np.conj(U)                              # -u(-x)
    assert abs(oracle.J2(c, Ui) - J0) <= 1e-12 * J0
    assert np.allclose(oracle.grad(c, Ui), -np.conj(G0), atol=1e-10 * np.abs(G0).max())


# ------------------------------------------------------------ descent ---

def test_step_rate_identity():
    """d J^2 / d tau = 2 <L^dagger r, G> with G = -L^dagger r / (1 + dtau A^2)
    (first order in dtau; eqs. rate_of_J_with_adjoint and KSE_G)."""
    spec = ksinputs.config_specs(0)[0]
    c = Curve(spec.n_s, spec.n_x, spec.L)
    _, _, U = ksinputs.make_curve(spec, c.K + 1)
    J0 = oracle.J2(c, U)
    Ad = oracle.adjoint(c, U)
    for dtau in (1e-6, 1e-7):
        U1 = oracle.step(c, U, dtau)
        rate = (oracle.J2(c, U1) - J0) / dtau
        pred = -2 * oracle.inner(c, Ad, Ad / (1 + dtau * c.A[None, :] ** 2))
        assert abs(rate / pred - 1) < 20 * dtau * 1e3 + 1e-6


def test_step_single_mode_closed_form():
    """Tiny amplitude, constant in s: away from the end rows r = A_k u and
    L^dagger r = A_k^2 u, so one step multiplies the mode by 1/(1 + dtau A_k^2)."""
    c = Curve(20, 32, 22.0, "finite", 5.0)
    k = 5
    eps = 1e-9
    U = np.zeros(c.shape, dtype=np.complex128)
    U[:, k] = eps * (0.3 - 0.4j)
    dtau = 0.01
    U1 = oracle.step(c, U, dtau)
    expect = U[5:-5, k] / (1 + dtau * c.A[k] ** 2)
    assert np.allclose(U1[5:-5, k], expect, rtol=1e-7, atol=0)
    R = oracle.residual(c, U)
    assert np.allclose(R[5:-5, k], c.A[k] * U[5:-5, k], rtol=1e-7, atol=0)


def test_descent_is_monotone_on_workload0():
    """2000 steps at dtau = 1e-3 decrease J^2 monotonically (eq. monotonic decrease)."""
    spec = ksinputs.config_specs(0)[0]
    c = Curve(spec.n_s, spec.n_x, spec.L)
    _, _, U = ksinputs.make_curve(spec, c.K + 1)
    prev = oracle.J2(c, U)
    first = prev
    for n in range(2000):
        U = oracle.step(c, U, 1e-3)
        if n % 50 == 49:
            cur = oracle.J2(c, U)
            assert cur < prev
            prev = cur
    assert prev < 0.7 * first


# ------------------------------------------------ metric and s-grid ---

def test_metric_against_analytic_derivative_and_paper_Dt():
    """The metric g = sin^2(theta)/(pi S) with theta = pi (1 - sigma): g times the
    central difference in sigma converges at second order to d/ds of a smooth
    function with constant asymptotes, and the paper's spectral D_t
    (eq. rational_diff_matrix, its index running the other way) agrees with
    the analytic derivative to spectral accuracy."""
    S, Sp = 10.0, 7.0

    def f(s):
        return np.tanh(s / Sp)

    def df(s):
        return 1.0 / (Sp * np.cosh(s / Sp) ** 2)

    errs = []
    for n_s in (33, 65, 129, 257):
        c = Curve(n_s, 8, 22.0, "rational", S)
        fs = np.where(np.isinf(c.s), np.sign(c.s), f(np.where(np.isinf(c.s), 0, c.s)))
        d = c.g[1:-1] * (fs[2:] - fs[:-2]) / (2 * c.dsigma)
        errs.append(np.abs(d - df(c.s[1:-1])).max())
        # paper's D_t on the same points, numbered from s = +inf
        M = n_s - 2
        D = rational_Dt = oracle.rational_Dt(M, S)
        fp = fs[::-1]
        dp = (D @ fp)[::-1]
        if n_s >= 65:
            assert np.abs(dp[1:-1] - df(c.s[1:-1])).max() < 1e-8
        assert rational_Dt.shape == (n_s, n_s)
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders > 1.8), orders


# ---------------------------------------------------------- integrator ---

def test_etdrk4_small_amplitude_is_linear_exponential():
    c = Curve(3, 32, 22.0)
    u0 = np.zeros(c.K + 1, dtype=np.complex128)
    u0[1:6] = 1e-13 * (1 + 0.5j) / np.arange(1, 6)
    h, n = 0.05, 40
    traj = oracle.etdrk4_integrate(c, u0, h, n)
    exact = u0 * np.exp(c.A * h * n)
    assert np.allclose(traj[-1][1:6], exact[1:6], rtol=1e-9, atol=0)
    assert np.abs(traj[-1][6:]).max() < 1e-24  # O(amplitude^2) nonlinear leakage only


def test_etdrk4_matches_classical_rk4():
    """Independent check at O(1) amplitude: classical RK4 with a 10x smaller step
    (stable because |h A_K| stays small at N_x = 16)."""
    c = Curve(3, 16, 22.0)
    rng = np.random.default_rng(9)
    u0 = np.zeros(c.K + 1, dtype=np.complex128)
    u0[1:] = (rng.standard_normal(c.K) + 1j * rng.standard_normal(c.K)) / np.arange(1, c.K + 1) ** 2

    def rhs(v):
        return oracle.vector_field(c, v[None, :])[0]

    T = 2.0
    traj = oracle.etdrk4_integrate(c, u0, 0.01, 200)
    v = u0.copy()
    h = 0.001
    for _ in range(2000):
        k1 = rhs(v)
        k2 = rhs(v + 0.5 * h * k1)
        k3 = rhs(v + 0.5 * h * k2)
        k4 = rhs(v + h * k3)
        v = v + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    assert T == 200 * 0.01
    assert np.abs(traj[-1] - v).max() < 1e-8 * np.abs(v).max()


def test_integral_curve_residual_converges_at_second_order():
    """A curve sampled from a KS trajectory (finite map s = T sigma) has a discrete
    residual that vanishes at second order in dsigma: J -> 0 (Sec. II: r = 0
    along an integral curve)."""
    L, n_x, T = 39.0, 64, 2.0
    c0 = Curve(3, n_x, L)
    rng = np.random.default_rng(10)
    u0 = np.zeros(c0.K + 1, dtype=np.complex128)
    u0[1:7] = (rng.standard_normal(6) - 1j * rng.standard_normal(6)) / (2 * np.arange(1, 7) ** 2)
    fine = 512
    traj = oracle.etdrk4_integrate(c0, u0, T / fine, fine)   # samples at t = T m / 512
    Js = []
    for n_s in (17, 33, 65, 129):
        c = Curve(n_s, n_x, L, "finite", T)
        stride = fine // (n_s - 1)
        U = traj[::stride]
        assert U.shape[0] == n_s
        Js.append(np.sqrt(oracle.J2(c, U)))
    ratios = np.array(Js[:-1]) / np.array(Js[1:])
    assert np.all(np.abs(ratios - 4.0) < 0.25), (Js, ratios)


# ---------------------------------------------------- inversion-symmetric subspace


def _odd_curve(seed, n_s, n_x, L, map_="rational", scale=40.0):
    c = oracle.Curve(n_s, n_x, L, map_, scale)
    rng = np.random.default_rng(seed)
    k = np.arange(1, c.K + 1)
    B = rng.standard_normal((n_s, c.K)) * 0.4 / k[None, :]
    return c, B


def test_odd_state_is_the_sine_series():
    """b_k = Im u_hat_k means u(x) = -2 sum_k b_k sin(q_k x): explicit sine sums
    on the grid (no FFT) against the spectral-to-physical map."""
    c, B = _odd_curve(31, 5, 32, 22.0)
    x = np.arange(c.n_x) * c.L / c.n_x
    k = np.arange(1, c.K + 1)
    u_sines = -2.0 * (B[:, :, None] * np.sin(2 * np.pi * k[None, :, None] * x[None, None, :] / c.L)).sum(1)
    assert np.abs(oracle.to_physical(oracle.odd_to_full(B), c.n_x) - u_sines).max() <= 1e-13
    assert np.array_equal(oracle.full_to_odd(oracle.odd_to_full(B)), B)


@pytest.mark.parametrize("map_,scale", [("rational", 40.0), ("finite", 5.0)])
def test_inversion_symmetric_subspace_is_invariant(map_, scale):
    """The residual, the gradient and the step of an inversion-symmetric curve
    stay in the subspace (purely imaginary coefficients, zero mean), Sec. V.B."""
    c, B = _odd_curve(32, 24, 64, 39.0, map_, scale)
    U = oracle.odd_to_full(B)
    r = oracle.residual(c, U)
    assert np.abs(r.real).max() <= 1e-12 * np.abs(r).max()
    G = oracle.grad(c, U)
    assert np.abs(G.real).max() <= 1e-12 * np.abs(G).max()
    assert np.abs(G[:, 0]).max() <= 1e-12 * np.abs(G).max()
    U1 = oracle.step(c, U, 1e-3)
    assert np.abs(U1.real).max() <= 1e-12 * np.abs(U1).max()


def test_odd_gradient_is_the_derivative_in_b():
    """J^2 restricted to the subspace is a quartic polynomial in b, so a
    Richardson-extrapolated central difference along a direction in b is exact
    up to rounding; it must equal <dJ^2/db, V>."""
    c, B = _odd_curve(33, 20, 32, 22.0, "finite", 4.0)
    rng = np.random.default_rng(34)
    V = rng.standard_normal(B.shape) / np.arange(1, c.K + 1)[None, :]
    V[0] = 0
    V[-1] = 0
    G = oracle.grad_odd(c, B)

    def fd(h):
        return (oracle.J2_odd(c, B + h * V) - oracle.J2_odd(c, B - h * V)) / (2 * h)

    rich = (4 * fd(1e-3) - fd(2e-3)) / 3
    dot = float(np.sum(G * V))
    assert abs(rich - dot) <= 1e-9 * abs(dot)


# ------------------------------------------- spectral d/ds (paper's D_t) ---

def _decaying_curve(s, n_x):
    """A smooth curve u(x, s) that decays to u = 0 at both ends, with its exact
    s-derivative: u_hat_1 = 0.3 sech(s/4), u_hat_2 = -0.2 i sech(s/4) tanh(s/4)."""
    K1 = oracle.n_modes(n_x)
    sech, th = 1.0 / np.cosh(s / 4.0), np.tanh(s / 4.0)
    U = np.zeros((len(s), K1), dtype=np.complex128)
    dU = np.zeros_like(U)
    U[:, 1] = 0.3 * sech
    dU[:, 1] = -0.3 * th * sech / 4.0
    U[:, 2] = -0.2j * sech * th
    dU[:, 2] = -0.2j * (sech ** 3 - th ** 2 * sech) / 4.0
    return U, dU


def test_spectral_ds_residual_converges_spectrally():
    """With the paper's D_t along s (eq. rational_diff_matrix) the discrete
    residual of a smooth curve matches f(u) - u_s at the collocation points with
    an error that falls faster than any power of N_s; the central difference
    converges at second order.  A wrong sign, orientation or scale of D_t would
    leave an O(|u_s|) = O(5e-2) error."""
    errs = {"spectral": [], "stencil": []}
    for n_s in (33, 65, 129):
        for ds in errs:
            c = Curve(n_s, 16, 22.0, "rational", 8.0, ds=ds)
            s = np.where(np.isinf(c.s), 0.0, c.s)
            U, dU = _decaying_curve(s, c.n_x)
            U[0] = U[-1] = 0.0  # the asymptotic states (u = 0)
            R = oracle.residual(c, U)
            exact = oracle.vector_field(c, U) - dU
            errs[ds].append(np.abs(R[1:-1] - exact[1:-1]).max())
    sp, st = errs["spectral"], errs["stencil"]
    assert sp[0] < 1e-5 and sp[2] < 1e-10, sp
    assert sp[0] / sp[1] > 100 and sp[1] / sp[2] > 100, sp
    orders = np.log2(np.array(st[:-1]) / np.array(st[1:]))
    assert np.all((orders > 1.8) & (orders < 2.2)), st


def test_spectral_adjoint_identity_and_gradient():
    """<L(u; v), r> = <v, L^dagger(u; r)> with the spectral d/ds (its s-part is
    the weighted transpose of D_t), and the gradient equals Richardson central
    differences of the quartic J^2 in every free coordinate."""
    rng = np.random.default_rng(15)
    c = Curve(14, 16, 22.0, "rational", 6.0, ds="spectral")
    U = _rand_state(c, rng)
    V = _rand_interior(c, rng)
    R = _rand_interior(c, rng)
    lhs = oracle.inner(c, oracle.jvp(c, U, V), R)
    rhs = oracle.inner(c, V, oracle.adjoint(c, U, R))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)
    c = Curve(7, 8, 22.0, "rational", 6.0, ds="spectral")
    U = _rand_state(c, rng, amp=0.5)
    G = oracle.grad(c, U)
    scale = np.abs(G).max()
    eps = 1e-3
    for j in range(1, c.n_s - 1):
        for k in range(c.K + 1):
            for part in (1.0, 1j):
                if k == 0 and part == 1j:
                    continue
                E = np.zeros(c.shape, dtype=np.complex128)
                E[j, k] = part

                def cd(h):
                    return (oracle.J2(c, U + h * E) - oracle.J2(c, U - h * E)) / (2 * h)
                fd = (4 * cd(eps / 2) - cd(eps)) / 3
                got = G[j, k].real if part == 1.0 else G[j, k].imag
                assert abs(fd - got) <= 1e-9 * scale, (j, k, part, fd, got)
    assert np.all(G[0] == 0) and np.all(G[-1] == 0)


def test_spectral_step_rate_and_transpose_matches_paper_adjoint():
    """The step decreases J^2 at the rate 2 <L^dagger r, G>; and the discrete
    adjoint's s-part, -(1/w) D_t^T (w r), agrees with the paper's r_s = D_t r up
    to the trapezoid rule's error, which vanishes spectrally for a smooth r
    that decays at both ends."""
    rng = np.random.default_rng(16)
    c = Curve(40, 16, 22.0, "rational", 8.0, ds="spectral")
    U = _rand_state(c, rng, amp=0.2, kmax=3)
    J0 = oracle.J2(c, U)
    Ad = oracle.adjoint(c, U)
    for dtau in (1e-6, 1e-7):
        U1 = oracle.step(c, U, dtau)
        rate = (oracle.J2(c, U1) - J0) / dtau
        pred = -2 * oracle.inner(c, Ad, Ad / (1 + dtau * c.A[None, :] ** 2))
        assert abs(rate / pred - 1) < 1e-3
    from oracle.ks import _ds, _ds_adjoint
    errs = []
    for n_s in (33, 65, 129):
        c = Curve(n_s, 16, 22.0, "rational", 8.0, ds="spectral")
        s = np.where(np.isinf(c.s), 0.0, c.s)
        Rr, _ = _decaying_curve(s, c.n_x)
        Rr[0] = Rr[-1] = 0.0
        errs.append(np.abs(_ds_adjoint(c, Rr) - _ds(c, Rr))[1:-1].max())
    assert errs[-1] < 1e-8 and errs[0] / errs[1] > 30, errs


# ------------------------------------------------------------- J_arc pins ---

def _resid_norm_two_mode(L, A, dA, B, dB):
    """|r| = sqrt(int_0^L r^2 dx) of u = A cos(q1 x) + B sin(q2 x) with
    u_s = dA cos(q1 x) + dB sin(q2 x), r = -u_s - u u_x - u_xx - u_xxxx
    (eq. KSE_residual), and |u_s|, from pointwise values on 64 points (the
    rectangle rule is exact for these band-limited fields)."""
    n = 64
    x = np.arange(n) * L / n
    q1, q2 = 2 * np.pi / L, 4 * np.pi / L
    c1, s2 = np.cos(q1 * x), np.sin(q2 * x)
    u = A * c1 + B * s2
    ux = -A * q1 * np.sin(q1 * x) + B * q2 * np.cos(q2 * x)
    uxx = -A * q1 ** 2 * c1 - B * q2 ** 2 * s2
    uxxxx = A * q1 ** 4 * c1 + B * q2 ** 4 * s2
    us = dA * c1 + dB * s2
    r = -us - u * ux - uxx - uxxxx
    return np.sqrt((r ** 2).sum() * L / n), np.sqrt((us ** 2).sum() * L / n)


def _J_arc_integral(L, curve_of_s, metric_power=0):
    """int |r| |u_s| ds / int |u_s| ds over s in (-inf, inf) (eq. J_arc),
    evaluated in s by adaptive quadrature; curve_of_s(s) -> (A, dA/ds, B, dB/ds).
    metric_power != 0 weights both integrands by (du/ds magnitude)^metric_power
    extra - a deliberately wrong weighting, to show the pin tells them apart."""
    from scipy.integrate import quad

    def parts(s):
        rn, usn = _resid_norm_two_mode(L, *curve_of_s(s))
        return rn, usn

    num = quad(lambda s: np.prod(parts(s)) * parts(s)[1] ** metric_power, -np.inf, np.inf,
               limit=400, epsabs=0, epsrel=1e-13)[0]
    den = quad(lambda s: parts(s)[1] ** (1 + metric_power), -np.inf, np.inf,
               limit=400, epsabs=0, epsrel=1e-13)[0]
    return num / den


def test_J_arc_rational_map_converges_to_the_integral_in_s():
    """eq. J_arc on the rational map, where the metric g = d sigma / ds is not
    constant: a curve from u = 0 to u = 0 (an equilibrium at both ends, so r
    vanishes there) with coefficients quadratic in sigma; the oracle's J_arc
    must converge to int |r||u_s| ds / int |u_s| ds evaluated by adaptive
    quadrature in s itself, with u_s = g u_sigma.  The sums run over the
    interior rows, whose central differences exist; the end rows' share of
    the denominator (|u_s| ds = |u_sigma| dsigma stays finite at s = +-inf)
    is left out, so the convergence is first order, and one Richardson step
    (2 J(2N) - J(N)) must then converge at second order.  Weighting the rows
    by g or 1/g (a dropped or inverted metric) converges to another number,
    which the same test would reject."""
    L, S = 22.0, 7.0
    a, b = 0.9, -1.4

    def curve_of_s(s):
        th = np.pi / 2 - np.arctan(s / S)          # s = S cot(theta)
        sig = 1.0 - th / np.pi
        g = np.sin(th) ** 2 / (np.pi * S)          # d sigma / ds
        A, dA = a * sig * (1 - sig), a * (1 - 2 * sig) * g
        B, dB = b * sig * (1 - sig), b * (1 - 2 * sig) * g
        return A, dA, B, dB

    exact = _J_arc_integral(L, curve_of_s)
    vals = []
    for n_s in (65, 129, 257, 513):
        c = Curve(n_s, 32, L, "rational", S)
        sig = c.sigma
        U = np.zeros((n_s, c.K + 1), dtype=np.complex128)
        U[:, 1] = 0.5 * a * sig * (1 - sig)           # A cos(q1 x): u_hat_1 = A / 2
        U[:, 2] = -0.5j * b * sig * (1 - sig)         # B sin(q2 x): u_hat_2 = -i B / 2
        vals.append(oracle.J_arc(c, U))
    errs = np.abs(np.array(vals) - exact) / exact
    orders = np.log2(errs[:-1] / errs[1:])
    assert np.all((orders > 0.95) & (orders < 1.05)), (errs, orders)
    rich = np.abs(2 * np.array(vals[1:]) - np.array(vals[:-1]) - exact) / exact
    assert rich[-1] < 1e-5, rich
    assert np.all(np.log2(rich[:-1] / rich[1:]) > 1.8), rich
    # the weighting matters on this curve: the same integrals with the rows
    # weighted by |u_s| once more differ from eq. J_arc by far more than the
    # discretization error above
    assert abs(_J_arc_integral(L, curve_of_s, metric_power=1) - exact) > 1e-2 * exact


def test_J_arc_spectral_ds_converges_to_the_integral_in_s():
    """eq. J_arc with the paper's D_t along s (eq. rational_diff_matrix): on the
    decaying closed-form curve the oracle's J_arc converges faster than any
    power of N_s to the same integral in s evaluated by adaptive quadrature."""
    L, S = 22.0, 8.0

    def curve_of_s(s):
        e = np.exp(-np.abs(s) / 4.0)
        sech, th = 2.0 * e / (1.0 + e * e), np.tanh(s / 4.0)  # no overflow as |s| grows
        # u = 0.6 sech cos(q1 x) + 0.4 sech tanh sin(q2 x): the coefficients
        # u_hat_1 = 0.3 sech, u_hat_2 = -0.2 i sech tanh of _decaying_curve
        A, dA = 0.6 * sech, -0.6 * th * sech / 4.0
        B, dB = 0.4 * sech * th, 0.4 * (sech ** 3 - th ** 2 * sech) / 4.0
        return A, dA, B, dB

    exact = _J_arc_integral(L, curve_of_s)
    errs = []
    for n_s in (33, 65, 129):
        c = Curve(n_s, 16, L, "rational", S, ds="spectral")
        s = np.where(np.isinf(c.s), 0.0, c.s)
        U, _ = _decaying_curve(s, c.n_x)
        U[0] = U[-1] = 0.0
        errs.append(abs(oracle.J_arc(c, U) - exact) / exact)
    assert errs[-1] < 1e-9, errs
    assert errs[0] / errs[1] > 30 and errs[1] / errs[2] > 30, errs
