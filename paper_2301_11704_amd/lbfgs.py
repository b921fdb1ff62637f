"""Batched limited-memory BFGS over the curves of a problem.

An acceleration of the final approach to a connecting orbit, beyond the
paper's gradient flow (the flow's fixed points are kept; the path in tau is
not): each curve of the batch is minimized independently, with

  * the Euclidean gradient of J^2 from the fused adjoint kernel (eval_grad),
  * the implicit-in-s increment as the initial inverse Hessian H0
    (ksc_precondition: -H0 G, H0 symmetric positive definite in the
    Euclidean inner product of the stored real and imaginary parts), so a
    first iteration from an empty memory is the implicit-in-s step; after
    each update H0 is scaled per curve by gamma = s.y / (y.H0 y), the
    usual scaling of the initial matrix (Nocedal & Wright eq. 7.20 with H0
    in place of the identity),
  * the two-loop recursion over the last m pairs (s, y) (Nocedal & Wright,
    Numerical Optimization, Alg. 7.4), and
  * a backtracking line search to the Armijo condition per curve, starting
    from the unit step.

All vectors live on the device; the per-curve dot products and scalings are
plain tensor operations over the state layout.  `ops` supplies the model:
``grad(x) -> (G, J2)``, ``J2(x)``, ``precond(g) -> H0 g``, ``dot(a, b) ->
per-curve values``, ``scale(v, a) -> v scaled per curve`` and ``axpy(v, a,
x) -> v + a x per curve``; TorchOps wraps a Problem.  An iteration waits on
the device once in the common case (the line search's first trial).
"""
from __future__ import annotations

import torch


class TorchOps:
    """The L-BFGS model of a Problem whose scheme is "implicit_s" (the
    preconditioner is its solve); the state dtype should be FP64."""

    def __init__(self, prob, dtau: float):
        self.prob = prob
        self.dtau = float(dtau)
        nc = prob.n_curves
        probe = prob.new_state()
        sizes = [prob.view(probe, c).numel() for c in range(nc)]
        del probe
        self.uniform = len(set(sizes)) == 1 and sum(sizes) == prob.numel
        dev = prob.device
        if not self.uniform:
            # curve index of every scalar of the state (curves are contiguous)
            idx = torch.full((prob.numel,), -1, dtype=torch.long, device=dev)
            for c in range(nc):
                n = sizes[c]
                idx[prob.offsets[c]:prob.offsets[c] + n] = c
            self.cidx = idx
            self.valid = idx >= 0
        self.nc = nc
        self._buf = torch.empty(prob.numel, dtype=prob.dtype, device=dev)

    def grad(self, x):
        G, J2 = self.prob.eval_grad(x)
        return G, J2

    def J2(self, x):
        return self.prob.eval_J(x)

    def precond(self, g):
        return torch.neg(self.prob.precondition(g, self._buf, self.dtau))

    def dot(self, a, b):
        if self.uniform:
            return torch.linalg.vecdot(a.view(self.nc, -1), b.view(self.nc, -1)).to(torch.float64)
        out = torch.zeros(self.nc, dtype=torch.float64, device=a.device)
        p = (a * b).to(torch.float64)
        return out.index_add_(0, self.cidx.clamp(min=0), torch.where(self.valid, p, 0.0))

    def scale(self, v, a):
        a = a.to(v.dtype)
        if self.uniform:
            return (v.view(self.nc, -1) * a[:, None]).view(-1)
        return v * torch.where(self.valid, a[self.cidx.clamp(min=0)], 0.0)

    def axpy(self, v, a, x):
        if self.uniform:
            return torch.addcmul(v.view(self.nc, -1), x.view(self.nc, -1),
                                 a.to(v.dtype)[:, None]).view(-1)
        return v + self.scale(x, a)


class BatchLBFGS:
    """L-BFGS iterations on every active curve of a batch (see the module
    docstring).  State, gradient and history are vectors in the state
    layout; per-curve quantities are FP64 vectors of n_curves entries."""

    def __init__(self, ops, m: int = 8, c1: float = 1e-4, max_backtrack: int = 12):
        if m < 1:
            raise ValueError("m must be >= 1")
        self.ops = ops
        self.m = int(m)
        self.c1 = float(c1)
        self.max_backtrack = int(max_backtrack)
        self.S, self.Y, self.rho = [], [], []
        self.x = self.g = self.J2 = self.gamma = None

    def start(self, x):
        """Begin at x (copied): gradient, cost, empty memory."""
        self.x = x.clone()
        self.g, self.J2 = self.ops.grad(self.x)
        self.g = self.g.clone()
        self.J2 = self.J2.clone()
        self.S, self.Y, self.rho = [], [], []
        self.gamma = torch.ones_like(self.J2)

    def _forget(self, mask):
        """Drop the memory (and the H0 scaling) of the curves in mask."""
        for i in range(len(self.rho)):
            self.rho[i] = torch.where(mask, torch.zeros_like(self.rho[i]), self.rho[i])
        self.gamma = torch.where(mask, torch.ones_like(self.gamma), self.gamma)

    def direction(self):
        """-H g by the two-loop recursion (Nocedal & Wright Alg. 7.4)."""
        ops = self.ops
        q = self.g.clone()
        alpha = []
        for s, y, rho in zip(reversed(self.S), reversed(self.Y), reversed(self.rho)):
            a = rho * ops.dot(s, q)
            q = ops.axpy(q, -a, y)
            alpha.append(a)
        r = ops.scale(ops.precond(q), self.gamma)
        for (s, y, rho), a in zip(zip(self.S, self.Y, self.rho), reversed(alpha)):
            b = rho * ops.dot(y, r)
            r = ops.axpy(r, a - b, s)
        return -r

    def iterate(self, active):
        """One iteration on the curves where `active` (bool tensor) holds;
        the others stay where they are.  Returns the per-curve J2."""
        ops = self.ops
        act = active.to(torch.bool)
        d = self.direction()
        gd = ops.dot(self.g, d)
        J2 = self.J2
        step = act.to(torch.float64)
        Jt = ops.J2(ops.axpy(self.x, step, d))
        ok = ~act | (Jt <= J2 + self.c1 * step * gd)
        # a curve whose direction is not a descent direction (rounding, or a
        # memory that no longer fits) restarts from the preconditioned step
        bad = act & ~(gd < 0)
        flags = torch.stack([bad.any(), ok.all()]).cpu()  # the one wait
        if bool(flags[0]):
            self._forget(bad)
            d0 = -ops.precond(self.g)
            sel = bad.to(d.dtype)
            d = ops.axpy(ops.scale(d, 1 - sel), sel, d0)
            gd = ops.dot(self.g, d)
            Jt = ops.J2(ops.axpy(self.x, step, d))
            ok = ~act | (Jt <= J2 + self.c1 * step * gd)
            flags[1] = ok.all().cpu()
        for _ in range(self.max_backtrack):
            if bool(flags[1]):
                break
            step = torch.where(ok, step, 0.5 * step)
            Jt = ops.J2(ops.axpy(self.x, step, d))
            ok = ~act | (Jt <= J2 + self.c1 * step * gd)
            flags[1] = ok.all().cpu()
        if not bool(flags[1]):
            # no acceptable step along d: stay, and forget the memory
            failed = ~ok
            step = torch.where(failed, torch.zeros_like(step), step)
            self._forget(failed)
        x_new = ops.axpy(self.x, step, d)
        g_new, J2_new = ops.grad(x_new)
        s = x_new - self.x
        y = g_new - self.g
        sy = ops.dot(s, y)
        yy = ops.dot(y, y)
        # keep the pair only where it carries curvature (s.y > 0 well above
        # rounding); elsewhere its weight is 0 and the pair is inert
        keep = (step > 0) & (sy > 1e-12 * torch.sqrt(ops.dot(s, s) * yy))
        rho = torch.where(keep, 1.0 / torch.where(keep, sy, torch.ones_like(sy)),
                          torch.zeros_like(sy))
        Hy = ops.precond(y)
        yHy = ops.dot(y, Hy)
        ok_g = keep & (yHy > 0)
        self.gamma = torch.where(ok_g, sy / torch.where(ok_g, yHy, torch.ones_like(yHy)),
                                 self.gamma)
        self._push(s, y, rho)
        self.x, self.g = x_new, g_new.clone()
        self.J2 = torch.where(act, J2_new, J2)
        return self.J2

    def _push(self, s, y, rho):
        """Store the pair (s, y) with weight rho (a curve whose rho is 0
        ignores the pair: both loops of the recursion skip it)."""
        self.S.append(s)
        self.Y.append(y)
        self.rho.append(rho)
        if len(self.S) > self.m:
            self.S.pop(0)
            self.Y.pop(0)
            self.rho.pop(0)

    def run(self, n: int, active, every: int = 1):
        """n iterations; the J2 of every `every`-th iteration, [n // every, n_curves]."""
        rows = []
        for i in range(int(n)):
            J2 = self.iterate(active)
            if (i + 1) % every == 0:
                rows.append(J2.clone())
        if rows:
            return torch.stack(rows)
        return torch.zeros((0, self.ops.nc), dtype=torch.float64, device=self.x.device)
