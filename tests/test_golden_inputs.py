"""The stored workload-4 trajectory pieces (tests/golden/c4_trajectories.npz)
are what their oracle-only script computes, and each is an integral curve of
KS under the finite map s = T sigma: the oracle's J of the samples falls at
second order in dsigma (Sec. II: the residual vanishes along a trajectory).
CPU only."""
import importlib.util
import os

import numpy as np
import pytest

import oracle

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _script():
    spec = importlib.util.spec_from_file_location(
        "make_c4_trajectories", os.path.join(GOLD, "make_c4_trajectories.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("i", [0, 63])
def test_stored_trajectories_regenerate_bit_exactly(i):
    mod = _script()
    stored = np.load(os.path.join(GOLD, "c4_trajectories.npz"))
    assert stored["traj"].shape == (64, 129, 43)
    assert (float(stored["L"]), int(stored["n_x"]), float(stored["T"])) == (mod.L, mod.N_X, mod.T)
    assert np.array_equal(mod.trajectory(i).astype(np.complex64), stored["traj"][i])


def test_stored_trajectories_are_integral_curves():
    stored = np.load(os.path.join(GOLD, "c4_trajectories.npz"))
    L, n_x, T = float(stored["L"]), int(stored["n_x"]), float(stored["T"])
    for i in (5, 40):
        traj = stored["traj"][i].astype(np.complex128)
        Js = []
        for n_s in (33, 65, 129):
            c = oracle.Curve(n_s, n_x, L, "finite", T)
            Js.append(np.sqrt(oracle.J2(c, traj[::128 // (n_s - 1)])))
        ratios = np.array(Js[:-1]) / np.array(Js[1:])
        assert np.all(np.abs(ratios - 4.0) < 0.4), (i, Js, ratios)
