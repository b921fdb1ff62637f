"""Descent driver: integrate du/dtau = -L^dagger(u; r) (eq. KSE_G) with the
semi-implicit Euler step until every curve reaches a target J, the paper's
monitor J_arc (eq. J_arc) falls below its threshold, or a step budget runs out.

Policy (all decisions on the host, every `every` steps, from the J2 trace the
library writes while the steps run as captured HIP graphs):
  * FP32 phase until J < switch_J or J stops decreasing for `stall_records`
    consecutive records (the FP32 rounding floor); then the state is promoted
    to FP64 and the same kernels continue in FP64.
  * A record in which J of a curve rose by more than rise_tol (relative) or
    became non-finite rolls the whole batch back to the last accepted state
    and halves dtau; smaller rises count as a stall (rounding noise).
  * Curves that reached the target are frozen (the library's active mask), so
    the batch keeps running for the others.
  * Checkpoints (.npz) hold the state, dtype, tau, step count, dtau, the
    active mask and the history; resuming continues bitwise identically
    because the kernels are deterministic.

The driver talks to a backend object (``GpuBackend`` here); any object with
the same methods can stand in for it, which is how the failure handling is
tested on the CPU.
"""
from __future__ import annotations

import json
from dataclasses import dataclass, field

import numpy as np


@dataclass
class DescentLog:
    steps: int = 0
    tau: float = 0.0
    dtau: float = 0.0
    dtype: str = "f32"
    J_history: list = field(default_factory=list)  # (step, [J per curve])
    Jarc_history: list = field(default_factory=list)  # (step, [J_arc per curve]) with a J_arc target
    events: list = field(default_factory=list)     # (step, text)
    converged: np.ndarray | None = None


class GpuBackend:
    """Backend over the HIP library (Problem) for one dtype."""

    def __init__(self, problem, state):
        self.prob = problem
        self.state = state
        import torch
        self._torch = torch
        self.scratch = torch.empty_like(state)
        self.active = torch.ones(problem.n_curves, dtype=torch.uint8, device=state.device)
        self._lbfgs = None
        self._lbfgs_key = None

    @property
    def dtype(self) -> str:
        return "f64" if self.state.dtype == self._torch.float64 else "f32"

    def n_curves(self) -> int:
        return self.prob.n_curves

    def run(self, n_steps: int, dtau: float, every: int) -> np.ndarray:
        tr = self.prob.descend(self.state, n_steps, dtau, every=every, scratch=self.scratch,
                               active=self.active)
        return tr.cpu().numpy()

    def run_lbfgs(self, n_iter: int, dtau: float, every: int, m: int) -> np.ndarray:
        """n_iter batched L-BFGS iterations (lbfgs.py) on the active curves
        from the current state, H0 = the implicit-in-s solve at dtau; the
        memory carries over between calls while the state is the one the
        last call left.  Returns the J2 of every `every`-th iteration."""
        from .lbfgs import BatchLBFGS, TorchOps
        torch = self._torch
        key = (float(dtau), int(m))
        if self._lbfgs is None or self._lbfgs_key != key or \
                not torch.equal(self._lbfgs.x, self.state):
            self._lbfgs = BatchLBFGS(TorchOps(self.prob, dtau), m=m)
            self._lbfgs.start(self.state)
            self._lbfgs_key = key
        tr = self._lbfgs.run(n_iter, self.active.bool(), every)
        self.state.copy_(self._lbfgs.x)
        return tr.cpu().numpy()

    def J2(self) -> np.ndarray:
        return self.prob.eval_J(self.state).cpu().numpy()

    def J_arc(self) -> np.ndarray:
        return self.prob.eval_J(self.state, arc=True)[1].cpu().numpy()

    def set_active(self, mask: np.ndarray) -> None:
        self.active.copy_(self._torch.from_numpy(mask.astype(np.uint8)))

    def snapshot(self) -> np.ndarray:
        return self.state.detach().cpu().numpy().copy()

    def restore(self, arr: np.ndarray) -> None:
        self.state.copy_(self._torch.from_numpy(arr).to(self.state.dtype))

    def promote(self) -> "GpuBackend":
        """The same curves continued in FP64."""
        from .problem import Problem
        p64 = Problem(self.prob.curves, dtype=self._torch.float64, device=self.state.device,
                      space=self.prob.space, ds=self.prob.ds)
        p64.set_scheme(self.prob.scheme)
        p64.set_momentum(self.prob.momentum)
        b = GpuBackend(p64, self.state.double())
        b.active.copy_(self.active)
        return b

    def flags(self) -> np.ndarray:
        return self.prob.query_flags()

    def set_momentum(self, beta: float) -> None:
        self.prob.set_momentum(beta)


def save_checkpoint(path: str, backend, log: DescentLog, active: np.ndarray) -> None:
    np.savez(path, state=backend.snapshot(), dtype=log.dtype, steps=log.steps, tau=log.tau,
             dtau=log.dtau, active=active.astype(np.uint8),
             history=json.dumps([(s, list(map(float, j))) for s, j in log.J_history]),
             events=json.dumps(log.events))


def load_checkpoint(path: str):
    d = np.load(path, allow_pickle=False)
    log = DescentLog(steps=int(d["steps"]), tau=float(d["tau"]), dtau=float(d["dtau"]),
                     dtype=str(d["dtype"]))
    log.J_history = [(s, np.array(j)) for s, j in json.loads(str(d["history"]))]
    log.events = [tuple(e) for e in json.loads(str(d["events"]))]
    return d["state"], d["active"].astype(bool), log


def descend_to(backend, dtau: float, J_target: float = 1e-8, max_steps: int = 10**6,
               every: int = 100, chunk: int | None = None, switch_J: float = 1e-8,
               stall_records: int = 10, fp64_finish: bool = True, Jarc_target: float | None = None,
               min_dtau: float = 1e-9, rise_tol: float = 1e-3, checkpoint: str | None = None,
               checkpoint_every: int | None = None, resume: bool = False, log: DescentLog | None = None,
               progress=None, momentum: float = 0.0, lbfgs: int = 0, lbfgs_chunk: int = 500):
    """Run the descent; returns (backend, DescentLog).  The returned backend may
    be a promoted (FP64) one holding the final state.  progress(log, J) is
    called after every accepted chunk with the per-curve J.  momentum > 0
    (implicit-in-s scheme) turns on the library's heavy-ball momentum from
    the second FP64 chunk on, for the slow final approach; the FP32 phase, far
    from the minimum, runs the plain steps.  A chunk whose cost rose with the
    momentum on is redone with plain steps at the same dtau, and the momentum
    resumes after it; a rise without momentum halves dtau.  lbfgs = m > 0
    (implicit-in-s scheme) runs that late phase as batched L-BFGS iterations
    instead (memory m, lbfgs_chunk iterations per chunk, H0 the implicit-in-s
    solve at dtau; an iteration counts as a step and tau does not advance)."""
    every = max(1, int(every))
    chunk = int(chunk or every)
    chunk = max(every, (chunk // every) * every)
    nc = backend.n_curves()
    active = np.ones(nc, dtype=bool)
    if log is None:
        log = DescentLog(dtau=dtau, dtype=backend.dtype)
    if resume and checkpoint:
        arr, active, log = load_checkpoint(checkpoint)
        if log.dtype == "f64" and backend.dtype != "f64":
            backend = backend.promote()
        backend.restore(arr)
        dtau = log.dtau
    backend.set_active(active)
    last_good = backend.snapshot()
    J_prev = np.sqrt(np.maximum(backend.J2(), 0.0))
    best = J_prev.copy()
    stall = np.zeros(nc, dtype=int)
    log.converged = J_prev < J_target
    since_ckpt = 0
    momentum_on = False
    switched_at = log.steps if log.dtype == "f64" else 1 << 62
    while log.steps < max_steps:
        late = backend.dtype == "f64" and log.steps > switched_at
        if lbfgs > 0 and late:
            n = max(1, min(int(lbfgs_chunk), max_steps - log.steps))
            tr = backend.run_lbfgs(n, dtau, n, lbfgs)
        else:
            n = min(chunk, max_steps - log.steps)
            n = max(every, (n // every) * every)
            tr = backend.run(n, dtau, every)
        J2 = backend.J2()
        Jn = np.sqrt(np.abs(J2))
        # a rise beyond rounding noise (rise_tol, relative) or a non-finite cost;
        # with momentum the cost is not monotone (the library restarts the
        # momentum of a curve at each rise), so only a rise by half is rejected
        tol = max(rise_tol, 0.5) if momentum_on else rise_tol
        rose = (~np.isfinite(J2)) | (np.isfinite(J_prev) & (Jn > J_prev * (1 + tol)) & active)
        trace_bad = ~np.all(np.isfinite(tr[:, active]), axis=0) if tr.size else np.zeros(active.sum(), bool)
        if np.any(rose & active) or np.any(trace_bad):
            backend.restore(last_good)
            if momentum_on:
                # the heavy ball overshot: redo the chunk with plain steps at
                # the same dtau (the momentum comes back after it)
                backend.set_momentum(0.0)
                momentum_on = False
                log.events.append((log.steps, "J rose with momentum; rollback, plain chunk"))
                continue
            dtau *= 0.5
            log.events.append((log.steps, f"J rose or non-finite; rollback, dtau -> {dtau:.3g}"))
            if dtau < min_dtau:
                log.events.append((log.steps, "dtau below minimum; stopping"))
                break
            continue
        lbfgs_chunk_done = lbfgs > 0 and late
        log.steps += n
        if not lbfgs_chunk_done:
            log.tau += n * dtau
        log.dtau = dtau
        log.J_history.append((log.steps, Jn.copy()))
        Ja = None
        if Jarc_target is not None:
            Ja = backend.J_arc()
            log.Jarc_history.append((log.steps, Ja.copy()))
        if progress is not None:
            progress(log, Jn)
        if momentum > 0 and lbfgs <= 0 and not momentum_on and backend.dtype == "f64" and \
                log.steps > switched_at:
            # momentum from the second FP64 chunk on: the first plain FP64
            # chunk removes the FP32 rounding noise, whose fast initial decrease
            # would otherwise throw the heavy ball out of the basin
            backend.set_momentum(momentum)
            momentum_on = True
            log.events.append((log.steps, f"momentum {momentum} on"))
        improved = Jn < best * (1 - 1e-7)
        stall = np.where(improved, 0, stall + 1)
        best = np.minimum(best, Jn)
        J_prev = Jn
        last_good = backend.snapshot()
        done = Jn < J_target
        if Ja is not None:
            done = done | (Ja < Jarc_target)
        newly = done & active
        if np.any(newly):
            log.events.append((log.steps, f"converged: {np.flatnonzero(newly).tolist()}"))
        active = active & ~done
        log.converged = done | log.converged
        backend.set_active(active)
        if not np.any(active):
            break
        if fp64_finish and backend.dtype == "f32":
            need = active & ((Jn < switch_J) | (stall >= stall_records))
            if np.any(need):
                backend = backend.promote()
                backend.set_active(active)
                log.dtype = "f64"
                log.events.append((log.steps, "switched to FP64"))
                switched_at = log.steps
                last_good = backend.snapshot()
                stall[:] = 0
        since_ckpt += n
        if checkpoint and checkpoint_every and since_ckpt >= checkpoint_every:
            save_checkpoint(checkpoint, backend, log, active)
            since_ckpt = 0
    if checkpoint:
        save_checkpoint(checkpoint, backend, log, active)
    return backend, log


def main(argv=None):
    """Descend the batched workload-4 curves (stored KS-trajectory pieces,
    L = 66, N_x = 128) to a target J, FP32 first and FP64 to finish, printing
    one progress line per chunk.  With --connection, descend instead the
    initial curves of eq. KSE_initial_curve (a = 0) between stored L = 22
    equilibria, e.g. E1-E2 (the paper's first run: N_x = 64, N_s = 552,
    S = 55, dtau = 0.01, spectral d/ds, stop at J_arc < 1e-12)."""
    import argparse
    import sys
    import time

    import torch

    ap = argparse.ArgumentParser(prog="python -m paper_2301_11704_amd.driver")
    ap.add_argument("--curves", type=int, default=64)
    ap.add_argument("--n-s", type=int, default=1024)
    ap.add_argument("--dtau", type=float, default=5e-4)
    ap.add_argument("--target", type=float, default=1e-8, help="stop when J = sqrt(J2) < target")
    ap.add_argument("--switch", type=float, default=1e-6, help="J below which FP64 takes over")
    ap.add_argument("--stall-records", type=int, default=10)
    ap.add_argument("--max-steps", type=int, default=4_000_000)
    ap.add_argument("--every", type=int, default=500)
    ap.add_argument("--chunk", type=int, default=50_000)
    ap.add_argument("--checkpoint", default=None)
    ap.add_argument("--checkpoint-every", type=int, default=None, help="steps between checkpoints")
    ap.add_argument("--resume", action="store_true")
    ap.add_argument("--connection", default=None,
                    help="comma-separated SRC-DST pairs of L = 22 equilibria, e.g. E1-E2,E1-E2+L/4")
    ap.add_argument("--table2", action="store_true",
                    help="the connections of the paper's Table II with their M and S, both "
                         "relative phases where they differ (implies the --connection defaults)")
    ap.add_argument("--ds", default=None, choices=["stencil", "spectral"],
                    help="d/ds (default: spectral with --connection, else stencil)")
    ap.add_argument("--S", type=float, default=55.0, help="rational map scale (--connection)")
    ap.add_argument("--space", default=None, choices=["full", "odd"],
                    help="state space (default: odd, the inversion-symmetric subspace the paper "
                         "searches, with --connection / --table2; else full)")
    ap.add_argument("--dtype", default=None, choices=["f32", "f64"],
                    help="start precision (default: f64 with --connection, else f32)")
    ap.add_argument("--jarc-target", type=float, default=None,
                    help="also stop a curve when J_arc falls below this (--connection: 1e-12)")
    ap.add_argument("--scheme", default="paper", choices=["paper", "implicit_s"],
                    help="descent step: the paper's (A_k^2 implicit) or implicit_s (the whole "
                         "linear part, d/ds included, implicit: larger stable dtau)")
    ap.add_argument("--lbfgs", type=int, default=0, metavar="M",
                    help="batched L-BFGS with memory M (H0 the implicit-in-s solve) from the "
                         "second FP64 chunk on instead of further steps (0: off)")
    ap.add_argument("--lbfgs-chunk", type=int, default=500,
                    help="L-BFGS iterations between the driver's decisions")
    ap.add_argument("--momentum", type=float, default=0.0,
                    help="heavy-ball momentum beta of the implicit_s descent from the FP64 switch "
                         "on (0: off; include/ksc.h ksc_set_momentum)")
    ap.add_argument("--history", default=None,
                    help="write the J and J_arc records (per chunk) and the events to this JSON file")
    args = ap.parse_args(argv)

    import ksinputs
    from . import CurveDesc, Problem

    labels = None
    if args.table2:
        made = ksinputs.table2_connections()
        labels = [m[0] for m in made]
        specs, Us = [m[1] for m in made], [m[2] for m in made]
        args.connection = "table2"
    elif args.connection:
        pairs = [p.split("-", 1) for p in args.connection.split(",")]
        n_s = args.n_s if args.n_s != 1024 else 552
        made = [ksinputs.l22_connection_curve(a, b, n_s, args.S) for a, b in pairs]
        specs, Us = [m[0] for m in made], [m[1] for m in made]
        labels = [p for p in args.connection.split(",")]
    space = args.space or ("odd" if args.connection else "full")
    if args.connection:
        ds = args.ds or "spectral"
        dt = torch.float64 if (args.dtype or "f64") == "f64" else torch.float32
        if args.dtau == 5e-4:
            args.dtau = 0.01
        if args.jarc_target is None:
            args.jarc_target = 1e-12
        if args.target == 1e-8:
            args.target = 0.0
    else:
        specs, Us = ksinputs.config4_curves(args.curves, args.n_s)
        ds = args.ds or "stencil"
        dt = torch.float64 if args.dtype == "f64" else torch.float32
    prob = Problem([CurveDesc(s.n_s, s.n_x, s.L, s.map, s.scale, s.s0) for s in specs],
                   dtype=dt, ds=ds, space=space)
    if space == "odd":
        if any(np.abs(U.real).max() > 0 for U in Us):
            raise ValueError("the odd subspace needs inversion-symmetric curves (u_hat_k = i b_k)")
        Us = [np.ascontiguousarray(U[:, 1:].imag) for U in Us]
    if args.lbfgs > 0 and args.scheme != "implicit_s":
        raise ValueError("--lbfgs takes its initial inverse Hessian from --scheme implicit_s")
    prob.set_scheme(args.scheme)
    prob.tune(None)
    X = prob.new_state()
    for c, U in enumerate(Us):
        prob.upload(X, c, U)
    b = GpuBackend(prob, X)
    t0 = time.time()
    J0 = np.sqrt(b.J2())
    print(f"start: {len(specs)} curves ({ds} d/ds, {space} space, {args.scheme} step"
          + (f", momentum {args.momentum}" if args.momentum else "") + "), "
          f"J max {J0.max():.3e} "
          f"min {J0.min():.3e}"
          + (f", J_arc {np.array2string(b.J_arc(), precision=3)}" if args.jarc_target else ""),
          flush=True)

    def report(log, J):
        arc = ""
        if log.Jarc_history and log.Jarc_history[-1][0] == log.steps:
            arc = " J_arc " + np.array2string(log.Jarc_history[-1][1], precision=3)
        print(f"step {log.steps:9d} tau {log.tau:10.3f} {log.dtype} dtau {log.dtau:.2e} "
              f"J max {np.max(J):.3e} min {np.min(J):.3e} below target {int(np.sum(J < args.target))}"
              f"{arc} wall {time.time() - t0:7.1f}s", flush=True)

    b2, log = descend_to(b, dtau=args.dtau, J_target=args.target, max_steps=args.max_steps,
                         every=args.every, chunk=args.chunk, switch_J=args.switch,
                         stall_records=args.stall_records, checkpoint=args.checkpoint,
                         checkpoint_every=args.checkpoint_every, resume=args.resume,
                         progress=report, Jarc_target=args.jarc_target, momentum=args.momentum,
                         lbfgs=args.lbfgs, lbfgs_chunk=args.lbfgs_chunk)
    J = np.sqrt(np.abs(b2.J2()))
    ok = J < args.target
    if args.jarc_target is not None:
        Ja = b2.J_arc()
        ok = ok | (Ja < args.jarc_target)
        print(f"J_arc {np.array2string(Ja, precision=3)}", flush=True)
        if labels:
            first = {}
            for st, a in log.Jarc_history:
                for i in np.flatnonzero(a < args.jarc_target):
                    first.setdefault(int(i), st)
            for i, lab in enumerate(labels):
                when = f"tau {first[i] * args.dtau:.0f}" if i in first else "not converged"
                print(f"  {lab:24s} N_s {specs[i].n_s:4d} S {specs[i].scale:4.0f} "
                      f"J_arc {Ja[i]:.3e}  {when}", flush=True)
    print(f"done: steps {log.steps} tau {log.tau:.3f} dtype {log.dtype} J max {J.max():.3e} "
          f"converged {int(np.sum(ok))}/{len(J)} wall {time.time() - t0:.1f}s", flush=True)
    for st, ev in log.events[-10:]:
        print(f"  event at step {st}: {ev}", flush=True)
    if args.history:
        arc = dict((st, list(map(float, a))) for st, a in log.Jarc_history)
        with open(args.history, "w") as fh:
            json.dump({"curves": [f"{sp.n_x}x{sp.n_s} L={sp.L} S={sp.scale}" for sp in specs],
                       "labels": labels,
                       "connection": args.connection, "ds": ds, "space": space,
                       "dtau0": args.dtau, "scheme": args.scheme,
                       "records": [{"step": st, "tau": st * args.dtau, "J": list(map(float, j)),
                                    "J_arc": arc.get(st)} for st, j in log.J_history],
                       "events": log.events}, fh)
    return 0 if np.all(ok) else 1


if __name__ == "__main__":
    raise SystemExit(main())
