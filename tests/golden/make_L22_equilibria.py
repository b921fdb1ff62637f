"""Write tests/golden/L22_equilibria.npz: the inversion-symmetric equilibria
E1, E2, E3 of KS at L = 22 on N_x = 64 points (the discretization of the
paper's Sec. V.D runs), found by the oracle's Newton solver.

Only oracle/ is called.  The starting guesses are rough sine coefficients
b_1..b_6 (u_hat_k = i b_k) that Newton's method carries to each solution;
which equilibrium a guess reaches is checked by Table I's eigenvalues in
tests/test_oracle_equilibria.py.  Usage (from the repository root):
    python tests/golden/make_L22_equilibria.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.equilibria import equilibrium  # noqa: E402

N_X, L = 64, 22.0
K = (N_X - 1) // 3
GUESSES = {
    "E1": [0.4, 0.1, 0.2, 0.2, 0.06, 0.02],
    "E2": [0.0, 0.56, 0.0, 0.35, 0.0, 0.06],
    "E3": [0.0, 0.0, 1.24, 0.0, 0.0, 0.22],
}


def main():
    out = {"n_x": np.int64(N_X), "L": np.float64(L)}
    for name, g in GUESSES.items():
        b0 = np.zeros(K)
        b0[:len(g)] = g
        U, res = equilibrium(N_X, L, b0)
        assert res < 1e-12, (name, res)
        out[name] = U
        print(name, "|f| = %.2e" % res)
    np.savez(os.path.join(HERE, "L22_equilibria.npz"), **out)


if __name__ == "__main__":
    main()
