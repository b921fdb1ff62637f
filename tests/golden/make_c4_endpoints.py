"""Write c4_endpoints.npz: the endpoint pairs of the 64-curve batched workload
(L = 66, N_x = 128, finite map T = 20).

For each curve i, a smooth random state (modes k <= 6, amplitude N(0,1)/k^2,
seed (4, i)) is integrated for 20 time units to shed its transient; that state
is the endpoint A_i and B_i = Phi_20(A_i) is the state 20 time units later on
the same trajectory, so a connecting curve from A_i to B_i with J = 0 exists.
Calls only the FP64 oracle's ETDRK4 integrator; values are stored in FP64.
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import ksinputs  # noqa: E402
import oracle  # noqa: E402


def main(n_curves=64, h=0.01):
    L, n_x, T = 66.0, 128, 20.0
    c = oracle.Curve(3, n_x, L)
    K1 = c.K + 1
    A = np.zeros((n_curves, K1), dtype=np.complex128)
    B = np.zeros((n_curves, K1), dtype=np.complex128)
    n = int(round(T / h))
    for i in range(n_curves):
        rng = np.random.default_rng(np.random.SeedSequence([4, i]))
        u0 = ksinputs.smooth_coeffs(rng, 6, 1.0, K1)
        a = oracle.etdrk4_integrate(c, u0, h, n, sample_every=n)[-1]
        b = oracle.etdrk4_integrate(c, a, h, n, sample_every=n)[-1]
        A[i], B[i] = a, b
    np.savez(os.path.join(HERE, "c4_endpoints.npz"), A=A, B=B, L=L, n_x=n_x, T=T, h=h)


if __name__ == "__main__":
    main()
