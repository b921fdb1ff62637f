"""Pins of the oracle's equilibria of KS at L = 22 (Sec. V.D, Table I): the
stored E1, E2, E3 (tests/golden/L22_equilibria.npz, written by
make_L22_equilibria.py from the oracle alone) are zeros of the vector field
whose unstable eigenvalues are the ones Table I prints.  CPU only."""
import os

import numpy as np
import pytest

import oracle
from oracle.equilibria import equilibrium, f_odd, stability

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = os.path.join(HERE, "golden")


def _table1():
    rows = {}
    with open(os.path.join(GOLD, "table1_E123_eigenvalues.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            name, re_, im_ = line.split()
            rows.setdefault(name, []).append(complex(float(re_), float(im_)))
    return rows


def _stored():
    d = np.load(os.path.join(GOLD, "L22_equilibria.npz"))
    return int(d["n_x"]), float(d["L"]), {k: d[k] for k in ("E1", "E2", "E3")}


@pytest.mark.parametrize("name", ["E1", "E2", "E3"])
def test_stored_equilibria_match_table1(name):
    n_x, L, eqs = _stored()
    c = oracle.Curve(3, n_x, L)
    U = eqs[name]
    # a zero of the vector field
    F = oracle.vector_field(c, U[None, :])[0]
    assert np.abs(F).max() < 1e-12
    ev = stability(c, U)
    unstable = [e for e in ev if e.real > 1e-6]
    want = _table1()[name]
    # each printed value (and its conjugate) appears, to the printed 4 decimals
    expect = []
    for w in want:
        expect.append(w)
        if w.imag != 0:
            expect.append(w.conjugate())
    assert len(unstable) == len(expect), (name, unstable)
    for w in expect:
        assert min(abs(e - w) for e in unstable) < 6e-5, (name, w, unstable)
    # exactly one zero eigenvalue (translation), every other one decaying
    small = [e for e in ev if abs(e) < 1e-6]
    assert len(small) == 1, small
    rest = [e for e in ev if abs(e) >= 1e-6 and e.real <= 1e-6]
    assert all(e.real < -1e-6 for e in rest)


def test_equilibria_symmetries_and_newton():
    """E2 is invariant under x -> x + L/2 (only even wavenumbers), E3 under
    x -> x + L/3 (only multiples of 3); E1 has both odd and even ones.  The
    stored states are fixed points of the Newton iteration."""
    n_x, L, eqs = _stored()
    k = np.arange(n_x // 3 + 1)
    b2, b3, b1 = (np.abs(eqs[n][1:].imag) for n in ("E2", "E3", "E1"))
    assert np.all(b2[(k[1:] % 2) == 1] < 1e-13) and b2.max() > 0.1
    assert np.all(b3[(k[1:] % 3) != 0] < 1e-13) and b3.max() > 0.1
    assert b1[0] > 0.1 and b1[1] > 0.01
    c = oracle.Curve(3, n_x, L)
    for name, U in eqs.items():
        assert np.all(U.real == 0)  # inversion symmetric about x = 0
        U2, res = equilibrium(n_x, L, U[1:].imag)
        assert res < 1e-12 and np.abs(U2 - U).max() < 1e-12
        assert np.linalg.norm(f_odd(c, U[1:].imag)) < 1e-12


def test_initial_curve_and_spectral_descent_from_E1_to_E2():
    """The initial curve of eq. KSE_initial_curve (a = 0) between the stored
    E1 and E2 on the paper's grid (N_x = 64, M = 550, S = 55) has the
    equilibria as its end rows and stays in the inversion-symmetric subspace;
    with the spectral d/ds the semi-implicit step at the paper's dtau = 0.01
    decreases J^2 monotonically (the paper reports this step as stable)."""
    import ksinputs
    spec, U = ksinputs.l22_connection_curve("E1", "E2")
    assert spec.n_s == 552 and spec.n_x == 64 and spec.scale == 55.0
    E1, E2 = ksinputs.l22_equilibrium("E1"), ksinputs.l22_equilibrium("E2")
    assert np.array_equal(U[0], E1) and np.array_equal(U[-1], E2)
    assert np.all(U.real == 0)
    c = oracle.Curve(spec.n_s, spec.n_x, spec.L, "rational", spec.scale, ds="spectral")
    J = [oracle.J2(c, U)]
    for _ in range(60):
        U = oracle.step(c, U, 0.01)
        J.append(oracle.J2(c, U))
    assert np.all(np.diff(J) < 0) and J[-1] < 0.6 * J[0]
    assert np.abs(U.real).max() < 1e-12  # the descent keeps the subspace


def test_table2_phase_variants_are_distinct_runs():
    """The Table II initial curves: every one is inversion symmetric, and the
    second curve of a row is a different run, not the first one moved by a
    common translation.  For row 7 the destination's other copy would not be:
    shifting E2 and E3 + L/6 both by L/2 gives E2 and E3 (E2 repeats after
    L/2 and E3 after L/3), so the row varies its source instead."""
    import ksinputs
    made = ksinputs.table2_connections()
    labels = [m[0] for m in made]
    assert len(made) == 14 and "row7:E2+L/4->E3" in labels and "row7:E2->E3+L/6" not in labels
    for _, _, U in made:
        assert np.abs(U.real).max() < 1e-12 and np.all(U[:, 0] == 0)
    k = np.arange(22)

    def shift(U, frac):
        return U * np.exp(2j * np.pi * k * frac)

    E2, E3 = ksinputs.l22_equilibrium("E2"), ksinputs.l22_equilibrium("E3")
    E3b = ksinputs.l22_equilibrium("E3+L/6")
    assert np.allclose(shift(E2, 0.5), E2, atol=1e-10)
    assert np.allclose(shift(E3b, 0.5), E3, atol=1e-10)
    # while E2 + L/4 -> E3 is no common translation of E2 -> E3
    E2b = ksinputs.l22_equilibrium("E2+L/4")
    for frac in np.arange(12) / 12:
        assert not (np.allclose(shift(E2b, frac), E2, atol=1e-6)
                    and np.allclose(shift(E3, frac), E3, atol=1e-6))
