"""Write c4_trajectories.npz: the KS trajectory pieces behind the 64-curve
batched workload (L = 66, N_x = 128, finite map s = T sigma, T = 20).

For each curve i a smooth random state (modes k <= 6, amplitude N(0,1)/k^2,
seed (4, i)) is integrated for 20 time units to shed its transient; that
state is the endpoint u_- = A_i.  The trajectory from A_i is then sampled at
t_m = T m / 128, m = 0..128, so u_+ = B_i = Phi_T(A_i) is its last sample and
the sampled trajectory is an integral curve of KS from A_i to B_i: a
connecting curve with J = 0 exists in the continuum, and a discrete zero of
the cost lies next to the samples on any fine s-grid.  Calls only the FP64
oracle's ETDRK4 integrator (fourth order, step 20/128/16 ~ 0.0098); the
samples are stored in FP32 (they seed an initial curve, not a reference).
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import ksinputs  # noqa: E402
import oracle  # noqa: E402


L, N_X, T = 66.0, 128, 20.0


def trajectory(i, n_samples=128, substeps=16, spinup_h=0.01):
    """The FP64 trajectory piece of curve i, [n_samples + 1, K + 1]."""
    c = oracle.Curve(3, N_X, L)
    rng = np.random.default_rng(np.random.SeedSequence([4, i]))
    u0 = ksinputs.smooth_coeffs(rng, 6, 1.0, c.K + 1)
    a = oracle.etdrk4_integrate(c, u0, spinup_h, int(round(T / spinup_h)),
                                sample_every=int(round(T / spinup_h)))[-1]
    h = T / n_samples / substeps
    return oracle.etdrk4_integrate(c, a, h, n_samples * substeps, sample_every=substeps)


def main(n_curves=64, n_samples=128, substeps=16):
    traj = np.stack([trajectory(i, n_samples, substeps).astype(np.complex64)
                     for i in range(n_curves)])
    np.savez_compressed(os.path.join(HERE, "c4_trajectories.npz"), traj=traj, L=L, n_x=N_X, T=T,
                        h=T / n_samples / substeps)


if __name__ == "__main__":
    main()
