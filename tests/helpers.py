"""Shared helpers of the parity tests: seeded curves, oracle evaluation and the
parity metrics.  The gradient metric compares L2 gradients (Euclidean
gradient divided by 2 w_j L c_k) in the norm weighted by 1/(1 + A_k^2) per
mode, since FP64 implementations that differ only in transform rounding
already disagree in the unweighted norm at the large-A_k modes."""
from __future__ import annotations

import numpy as np
import torch

import ksinputs
import oracle


def oracle_curve(spec: ksinputs.CurveSpec) -> oracle.Curve:
    return oracle.Curve(spec.n_s, spec.n_x, spec.L, spec.map, spec.scale, spec.s0)


def seeded_state(spec: ksinputs.CurveSpec, dtype) -> np.ndarray:
    """The seeded curve rounded to the run precision (both sides consume it)."""
    K1 = oracle.n_modes(spec.n_x)
    _, _, U = ksinputs.make_curve(spec, K1)
    U[:, 0] = U[:, 0].real
    return ksinputs.round_to(U, dtype)


def l2_gradient(c: oracle.Curve, G: np.ndarray) -> np.ndarray:
    """Euclidean gradient -> L2 gradient (L^dagger r) on interior rows."""
    w = c.w[1:-1, None] * c.L * c.c[None, :]
    return G[1:-1] / (2.0 * w)


def precond_rel_err(c: oracle.Curve, G_test: np.ndarray, G_ref: np.ndarray) -> float:
    Pi = 1.0 / (1.0 + c.A ** 2)
    a = l2_gradient(c, G_test) * Pi[None, :]
    b = l2_gradient(c, G_ref) * Pi[None, :]
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def directional_rel_err(c: oracle.Curve, G_test: np.ndarray, G_ref: np.ndarray, seeds) -> float:
    """max over seeded smooth directions V of the error of the directional
    derivative <G, V> relative to its condition, sum |G_ref| |V| (the size of the
    terms the dot product adds up; a plain |<G_ref, V>| can cancel to a few
    percent of that and then measures cancellation, not the gradient)."""
    worst = 0.0
    for s in seeds:
        V = ksinputs.random_direction(s, c.n_s, c.K + 1)
        dref = float(np.sum(G_ref.real * V.real + G_ref.imag * V.imag))
        dtest = float(np.sum(G_test.real * V.real + G_test.imag * V.imag))
        mag = float(np.sum(np.abs(G_ref.real * V.real) + np.abs(G_ref.imag * V.imag)))
        worst = max(worst, abs(dtest - dref) / mag)
    return worst


def elementwise_rel_err(c: oracle.Curve, G_test: np.ndarray, G_ref: np.ndarray) -> float:
    """max over rows j and modes k of |Pi_k (L2 gradient_test - L2 gradient_ref)_{jk}|
    relative to max |Pi_k L2 gradient_ref|, Pi_k = 1/(1 + A_k^2): every element of
    the gradient, in the same mode weighting as precond_rel_err."""
    Pi = 1.0 / (1.0 + c.A ** 2)
    a = l2_gradient(c, G_test) * Pi[None, :]
    b = l2_gradient(c, G_ref) * Pi[None, :]
    return float(np.abs(a - b).max() / np.abs(b).max())


def oracle_descent(c: oracle.Curve, U: np.ndarray, n: int, dtau: float, storage=None,
                   trace_every: int = 0):
    """n steps of oracle.step from U.  With storage = np.float32 the state is
    rounded to FP32 after every step (what an FP32 state holds between steps;
    each step is still computed in FP64).  With trace_every > 0 also returns
    the cost of the state entering every step i with (i + 1) % trace_every == 0
    (the last step of each captured group, whose cost ksc_descend traces)."""
    X = U.copy()
    tr = []
    for i in range(n):
        if trace_every and (i + 1) % trace_every == 0:
            tr.append(oracle.J2(c, X))
        X = oracle.step(c, X, dtau)
        if storage is not None:
            X = ksinputs.round_to(X, storage)
    return (X, tr) if trace_every else X


class OracleOps:
    """The model of paper_2301_11704_amd.lbfgs.BatchLBFGS from the FP64 oracle
    (gradient, cost, implicit-in-s preconditioner) over flat FP64 torch CPU
    vectors in the library's state layout (curve after curve,
    row-major, re/im interleaved)."""

    def __init__(self, curves, dtau):
        self.curves = curves
        self.dtau = dtau
        self.shapes = [(c.n_s, c.K + 1) for c in curves]
        self.sizes = [2 * n * k for n, k in self.shapes]
        self.offsets = np.concatenate([[0], np.cumsum(self.sizes)[:-1]]).astype(int)
        self.nc = len(curves)

    def unflat(self, x, i):
        o, n = self.offsets[i], self.sizes[i]
        v = x[o:o + n].numpy().reshape(*self.shapes[i], 2)
        return v[..., 0] + 1j * v[..., 1]

    def flat(self, arrs):
        return torch.from_numpy(np.concatenate(
            [np.stack([a.real, a.imag], axis=-1).ravel() for a in arrs]))

    def grad(self, x):
        Us = [self.unflat(x, i) for i in range(self.nc)]
        G = self.flat([oracle.grad(c, U) for c, U in zip(self.curves, Us)])
        return G, torch.tensor([oracle.J2(c, U) for c, U in zip(self.curves, Us)],
                               dtype=torch.float64)

    def J2(self, x):
        return torch.tensor([oracle.J2(c, self.unflat(x, i)) for i, c in enumerate(self.curves)],
                            dtype=torch.float64)

    def precond(self, g):
        return -self.flat([oracle.precondition_implicit_s(c, self.unflat(g, i), self.dtau)
                           for i, c in enumerate(self.curves)])

    def dot(self, a, b):
        return torch.tensor([float(torch.dot(a[o:o + n], b[o:o + n]))
                             for o, n in zip(self.offsets, self.sizes)], dtype=torch.float64)

    def scale(self, v, a):
        out = torch.empty_like(v)
        for i, (o, n) in enumerate(zip(self.offsets, self.sizes)):
            out[o:o + n] = v[o:o + n] * float(a[i])
        return out

    def axpy(self, v, a, x):
        return v + self.scale(x, a)
