"""The batched L-BFGS of paper_2301_11704_amd/lbfgs.py on the CPU, with a
model built from the FP64 oracle (gradient, cost and the implicit-in-s
preconditioner of ``oracle.precondition_implicit_s``).  No GPU."""
import numpy as np
import torch

import ksinputs
import oracle
from helpers import OracleOps
from paper_2301_11704_amd.lbfgs import BatchLBFGS


def _batch(n_curves=2, n_s=33, n_x=16):
    specs = [ksinputs.CurveSpec(n_s, n_x, 22.0, 4, 1.0, 4, 0.3, True, (140, i), "finite", 5.0)
             for i in range(n_curves)]
    curves = [oracle.Curve(s.n_s, s.n_x, s.L, s.map, s.scale) for s in specs]
    Us = []
    for s, c in zip(specs, curves):
        _, _, U = ksinputs.make_curve(s, c.K + 1)
        U[:, 0] = U[:, 0].real
        Us.append(U)
    return curves, Us


def test_first_iteration_is_the_implicit_in_s_step():
    curves, Us = _batch()
    ops = OracleOps(curves, 0.05)
    opt = BatchLBFGS(ops, m=5)
    opt.start(ops.flat(Us))
    opt.iterate(torch.ones(2, dtype=torch.bool))
    for i, (c, U) in enumerate(zip(curves, Us)):
        ref = oracle.step_implicit_s(c, U, 0.05)
        got = ops.unflat(opt.x, i)
        assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


def test_monotone_and_faster_than_the_implicit_in_s_steps():
    """J^2 never rises on any curve, an inactive curve does not move, and 40
    iterations take J^2 lower than 40 implicit-in-s steps of the same dtau."""
    curves, Us = _batch(3)
    ops = OracleOps(curves, 0.05)
    opt = BatchLBFGS(ops, m=6)
    x0 = ops.flat(Us)
    opt.start(x0)
    active = torch.tensor([True, True, False])
    prev = opt.J2.clone()
    for _ in range(40):
        J2 = opt.iterate(active)
        assert torch.all(J2 <= prev * (1 + 1e-12))
        prev = J2.clone()
    o, n = ops.offsets[2], ops.sizes[2]
    assert torch.equal(opt.x[o:o + n], x0[o:o + n])
    for i in range(2):
        U = Us[i].copy()
        for _ in range(40):
            U = oracle.step_implicit_s(curves[i], U, 0.05)
        assert float(J2[i]) < oracle.J2(curves[i], U), (float(J2[i]), oracle.J2(curves[i], U))
