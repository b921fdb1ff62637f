"""Pins of the oracle's implicit-in-s descent step (the linear part of the
adjoint flow taken implicitly along s as well as in x).  CPU only."""
import numpy as np
import pytest

import ksinputs
import oracle
from oracle import Curve


def _adjoint_jacobian(c, k, part):
    """Jacobian of L^dagger(u; r(u)) at u = 0 with respect to the interior rows
    of mode k (real or imaginary part), read off in the same mode and part.
    L^dagger is a cubic polynomial of u, so the Richardson combination of two
    central differences is exact up to rounding."""
    ni = c.n_s - 2
    J = np.zeros((ni, ni))
    unit = 1.0 if part == "re" else 1j
    for col in range(ni):
        def d(h):
            U = np.zeros(c.shape, dtype=np.complex128)
            U[1 + col, k] = h * unit
            Ap = oracle.adjoint(c, U)
            U[1 + col, k] = -h * unit
            Am = oracle.adjoint(c, U)
            return (Ap - Am) / (2 * h)
        D = (4 * d(0.5) - d(1.0)) / 3
        out = D[1:-1, k]
        J[:, col] = out.real if part == "re" else out.imag
        # the linearization at u = 0 does not couple modes
        other = np.delete(D[1:-1], k, axis=1)
        assert np.abs(other).max() < 1e-9 * max(1.0, np.abs(out).max())
    return J


@pytest.mark.parametrize("map_,scale,n_s", [("rational", 40.0, 11), ("finite", 3.0, 12),
                                            ("rational", 7.0, 4)])
@pytest.mark.parametrize("k,part", [(0, "re"), (3, "re"), (3, "im")])
def test_operator_is_the_linear_part_of_the_adjoint(map_, scale, n_s, k, part):
    """B_k = A_k^2 - D m D is exactly the linearization of L^dagger at u = 0 on
    the interior rows: a sign, a dropped mask or a wrong metric factor in the
    banded operator fails here."""
    c = Curve(n_s, 16, 22.0, map_, scale)
    B = oracle.implicit_s_operator(c, k)
    J = _adjoint_jacobian(c, k, part)
    assert np.allclose(B, J, rtol=0, atol=1e-9 * np.abs(J).max())


def test_operator_couples_rows_two_apart_and_is_weighted_symmetric():
    """The central difference applied twice reaches rows j - 2 and j + 2 only,
    and B_k is self-adjoint and positive semi-definite in the inner product
    with weights w_j = dsigma / g_j."""
    c = Curve(15, 16, 22.0, "rational", 30.0)
    B = oracle.implicit_s_operator(c, 2)
    ni = c.n_s - 2
    for i in range(ni):
        for j in range(ni):
            if abs(i - j) not in (0, 2):
                assert B[i, j] == 0.0
    W = np.diag(c.w[1:-1])
    S = W @ B
    assert np.allclose(S, S.T, rtol=0, atol=1e-12 * np.abs(S).max())
    assert np.linalg.eigvalsh(0.5 * (S + S.T)).min() > -1e-9 * np.abs(S).max()


def _config0_curve():
    spec = ksinputs.config_specs(0)[0]
    c = Curve(spec.n_s, spec.n_x, spec.L)
    _, _, U = ksinputs.make_curve(spec, c.K + 1)
    return c, U


def test_step_agrees_with_the_paper_step_to_first_order():
    """Both steps follow du/dtau = -L^dagger: they differ at O(dtau^2)."""
    c, U = _config0_curve()
    diffs = []
    for dtau in (1e-4, 5e-5, 2.5e-5):
        d = oracle.step_implicit_s(c, U, dtau) - oracle.step(c, U, dtau)
        diffs.append(np.abs(d).max())
    r1, r2 = diffs[0] / diffs[1], diffs[1] / diffs[2]
    assert 3.5 < r1 < 4.5 and 3.5 < r2 < 4.5, diffs


def test_step_descends_beyond_the_explicit_stability_bound():
    """On a finite-map curve whose s-stiffness limits the paper's step, a dtau
    40 times larger still decreases J^2 monotonically, where the paper's step
    grows without bound."""
    # a short finite-map curve (the kind of the 64-curve batch) keeps it quick
    c = Curve(129, 32, 66.0, "finite", 5.0)
    rng = np.random.default_rng(3)
    s = np.linspace(0.0, 1.0, c.n_s)[:, None]
    k = np.arange(c.K + 1)[None, :]
    U = (np.exp(-0.3 * k) * (np.cos(2 * np.pi * s * (1 + k % 3)) + 0.5j * np.sin(np.pi * s * k))
         + 0.01 * (rng.standard_normal(c.shape) + 1j * rng.standard_normal(c.shape)))
    U[:, 0] = 0.0
    beta = c.g[1] / (2 * c.dsigma)
    dtau_explicit = 0.5 / (4 * beta ** 2)   # the s-part's own explicit bound, halved
    dtau = 40 * dtau_explicit
    J = [oracle.J2(c, U)]
    V = U.copy()
    for _ in range(30):
        V = oracle.step_implicit_s(c, V, dtau)
        J.append(oracle.J2(c, V))
    assert all(b < a for a, b in zip(J, J[1:])), J
    W = U.copy()
    with np.errstate(all="ignore"):
        for _ in range(30):
            W = oracle.step(c, W, dtau)
        Jw = oracle.J2(c, W)
    assert not np.isfinite(Jw) or Jw > J[0]


def test_step_keeps_the_inversion_symmetric_subspace():
    c = Curve(20, 32, 22.0, "rational", 20.0)
    rng = np.random.default_rng(5)
    Bv = 0.3 * rng.standard_normal((c.n_s, c.K)) / np.arange(1, c.K + 1) ** 2
    U = oracle.odd_to_full(Bv)
    U1 = oracle.step_implicit_s(c, U, 0.05)
    # the real parts stay at the rounding level of the transforms
    assert np.abs(U1.real).max() < 1e-15 * np.abs(U1.imag).max()
    assert np.allclose(oracle.step_implicit_s_odd(c, Bv, 0.05), U1[:, 1:].imag, rtol=0, atol=0)


def test_step_keeps_end_rows_and_zero_imaginary_mode0():
    c, U = _config0_curve()
    U1 = oracle.step_implicit_s(c, U, 0.1)
    assert np.array_equal(U1[0], U[0]) and np.array_equal(U1[-1], U[-1])
    assert np.all(U1[:, 0].imag == 0)


def test_momentum_descent_reduces_to_implicit_steps_and_accelerates():
    """Heavy-ball momentum on the implicit-in-s step: with beta = 0 it is the
    plain sequence of steps; with beta > 0 the first step equals the plain
    one (the iteration starts from rest) and the end rows and Im of mode 0 are
    untouched; on workload 0's curve it lowers J^2 faster than the plain steps
    over the same number of steps."""
    import ksinputs
    spec = ksinputs.config_specs(0)[0]
    c = oracle.Curve(spec.n_s, spec.n_x, spec.L, spec.map, spec.scale)
    _, _, U = ksinputs.make_curve(spec, c.K + 1)
    U[:, 0] = U[:, 0].real
    plain = U.copy()
    for _ in range(3):
        plain = oracle.step_implicit_s(c, plain, 0.01)
    assert np.array_equal(oracle.descend_implicit_s_momentum(c, U, 3, 0.01, 0.0), plain)
    one = oracle.descend_implicit_s_momentum(c, U, 1, 0.01, 0.9)
    assert np.array_equal(one, oracle.step_implicit_s(c, U, 0.01))
    m = oracle.descend_implicit_s_momentum(c, U, 40, 0.01, 0.9)
    assert np.array_equal(m[0], U[0]) and np.array_equal(m[-1], U[-1])
    assert np.all(m[:, 0].imag == 0)
    p40 = U.copy()
    for _ in range(40):
        p40 = oracle.step_implicit_s(c, p40, 0.01)
    assert oracle.J2(c, m) < oracle.J2(c, p40)


def test_precondition_is_symmetric_positive_definite_in_the_euclidean_product():
    """The implicit-in-s preconditioner G -> -H0 G (``precondition_implicit_s``)
    as a map of the stored real and imaginary parts: <a, H0 b> = <H0 a, b> and
    <a, H0 a> > 0 for seeded gradient-shaped a, b (zero on the end rows and
    for Im of mode 0), on both maps; on the rational map a constant weight
    in place of w_j breaks the symmetry.  Applied to the gradient it is the
    increment of the implicit-in-s step."""
    import ksinputs
    rng = np.random.default_rng(7)
    for map_, scale in (("rational", 30.0), ("finite", 5.0)):
        c = oracle.Curve(33, 16, 22.0, map_, scale)
        K1 = c.K + 1

        def vec():
            v = rng.standard_normal((c.n_s, K1)) + 1j * rng.standard_normal((c.n_s, K1))
            v[0] = v[-1] = 0
            v[:, 0] = v[:, 0].real
            return v

        def dot(x, y):
            return float(np.sum(x.real * y.real + x.imag * y.imag))

        for dtau in (0.01, 1.0):
            a, b = vec(), vec()
            Ha = -oracle.precondition_implicit_s(c, a, dtau)
            Hb = -oracle.precondition_implicit_s(c, b, dtau)
            assert abs(dot(a, Hb) - dot(Ha, b)) <= 1e-12 * abs(dot(a, Hb)), (dot(a, Hb), dot(Ha, b))
            assert dot(a, Ha) > 0 and dot(b, Hb) > 0
            # the same map without the metric weight is not symmetric
            w_saved = c.w.copy()
            c.w = np.ones_like(c.w) * c.w.mean()
            Hb_bad = -oracle.precondition_implicit_s(c, b, dtau)
            Ha_bad = -oracle.precondition_implicit_s(c, a, dtau)
            c.w = w_saved
            if map_ == "rational":
                assert abs(dot(a, Hb_bad) - dot(Ha_bad, b)) > 1e-6 * abs(dot(a, Hb_bad))
        spec = ksinputs.CurveSpec(33, 16, 22.0, 4, 1.0, 4, 0.2, True, (131, 0), map_, scale)
        _, _, U = ksinputs.make_curve(spec, K1)
        U[:, 0] = U[:, 0].real
        step = oracle.step_implicit_s(c, U, 0.1)
        inc = oracle.precondition_implicit_s(c, oracle.grad(c, U), 0.1)
        assert np.abs(U + inc - step).max() <= 1e-13 * np.abs(step).max()
