"""GPU: the autograd Function, the batched autograd-path workload (64 curves,
L=66, N_x=128, N_s=1024) against central finite differences and the FP64
oracle, and multi-step descents against the oracle."""
import numpy as np
import pytest

import ksinputs
import oracle
from helpers import (directional_rel_err, elementwise_rel_err, oracle_curve, oracle_descent,
                     precond_rel_err, seeded_state)

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _prob(specs, dtype):
    import paper_2301_11704_amd as ksc
    return ksc.Problem([ksc.CurveDesc(s.n_s, s.n_x, s.L, s.map, s.scale, s.s0) for s in specs],
                       dtype=dtype)


def test_autograd_backward_equals_scaled_gradient():
    import paper_2301_11704_amd as ksc
    specs = [ksinputs.CurveSpec(300, 64, 39.0, 6, 1.0, 6, 0.2, True, (60, i)) for i in range(3)]
    prob = _prob(specs, torch.float32)
    X = prob.new_state()
    for c, s in enumerate(specs):
        prob.upload(X, c, seeded_state(s, np.float32))
    Xr = X.clone().requires_grad_(True)
    J2 = ksc.curve_J2(Xr, prob)
    w = torch.tensor([0.5, -2.0, 3.0], dtype=torch.float64, device="cuda")
    (J2 * w).sum().backward()
    G, _ = prob.eval_grad(X, scale=w)
    torch.cuda.synchronize()
    assert torch.equal(Xr.grad, G)
    J2b = prob.eval_J(X)
    assert torch.equal(J2.detach(), J2b)


def test_autograd_path_workload_vs_fd_and_oracle():
    """64 curves, FP32 autograd gradient: directional derivatives against FP64
    central differences of the oracle's J^2 (eps = 1e-4, 16 smooth directions
    spanning all curves) and the per-curve preconditioned error against the
    oracle adjoint."""
    import paper_2301_11704_amd as ksc
    specs, Us = ksinputs.config4_curves(64)
    prob = _prob(specs, torch.float32)
    X = prob.new_state()
    Ur = []
    for c, U in enumerate(Us):
        U = ksinputs.round_to(U, np.float32)
        U[:, 0] = U[:, 0].real
        Ur.append(U)
        prob.upload(X, c, U)
    Xr = X.clone().requires_grad_(True)
    ksc.curve_J2(Xr, prob).sum().backward()
    torch.cuda.synchronize()
    curves = [oracle_curve(s) for s in specs]
    worst_pre = worst_el = 0.0
    for c in range(64):  # oracle adjoint of every curve
        Gg = prob.download(Xr.grad, c)
        Gr = oracle.grad(curves[c], Ur[c])
        worst_pre = max(worst_pre, precond_rel_err(curves[c], Gg, Gr))
        worst_el = max(worst_el, elementwise_rel_err(curves[c], Gg, Gr))
    print(f"autograd path, 64 curves: preconditioned {worst_pre:.2e}, element-wise {worst_el:.2e}",
          flush=True)
    assert worst_pre <= 1e-5, worst_pre
    assert worst_el <= 1e-5, worst_el
    eps = 1e-4
    worst = 0.0
    for d in range(16):
        Vs = [ksinputs.random_direction((44, d, c), s.n_s, curves[c].K + 1) for c, s in
              enumerate(specs)]
        fd = 0.0
        dot = 0.0
        mag = 0.0
        for c in range(0, 64, 8):  # 8 curves per direction keep the CPU work small
            V = Vs[c]
            fd += (oracle.J2(curves[c], Ur[c] + eps * V) - oracle.J2(curves[c], Ur[c] - eps * V)) \
                / (2 * eps)
            Gg = prob.download(Xr.grad, c)
            dot += float(np.sum(Gg.real * V.real + Gg.imag * V.imag))
            Gr = oracle.grad(curves[c], Ur[c])
            mag += float(np.sum(np.abs(Gr.real * V.real) + np.abs(Gr.imag * V.imag)))
        worst = max(worst, abs(dot - fd) / mag)
    assert worst <= 1e-5, worst


def test_workload4_fp64_matches_oracle():
    """The FP64 finish evaluates the workload-4 batch (trajectory pieces:
    every mode populated) like the oracle: J2 of 8 curves to 1e-12 and the
    gradient of 2 curves in the preconditioned norm."""
    specs, Us = ksinputs.config4_curves(64)
    prob = _prob(specs, torch.float64)
    X = prob.new_state()
    for c, U in enumerate(Us):
        U = U.copy()
        U[:, 0] = U[:, 0].real
        prob.upload(X, c, U)
    J2 = prob.eval_J(X).cpu().numpy()
    G, _ = prob.eval_grad(X)
    torch.cuda.synchronize()
    for c in range(0, 64, 8):
        U = prob.download(X, c)
        cur = oracle_curve(specs[c])
        ref = oracle.J2(cur, U)
        assert abs(J2[c] - ref) <= 1e-12 * ref, (c, J2[c], ref)
        if c in (0, 32):
            assert precond_rel_err(cur, prob.download(G, c), oracle.grad(cur, U)) <= 1e-12


@pytest.mark.parametrize("dtype,tol", [(np.float64, 1e-12), (np.float32, 1e-5)])
def test_workload0_descent_2000_steps(dtype, tol):
    """2000 steps of workload 0.  An FP32 state is rounded to FP32 after every
    step, so the FP32 run is compared with the oracle run that rounds its state
    the same way (each of its steps still in FP64); the plain FP64 oracle run
    is reported beside it."""
    spec = ksinputs.config_specs(0)[0]
    tdt = torch.float64 if dtype == np.float64 else torch.float32
    prob = _prob([spec], tdt)
    X = prob.new_state()
    U = seeded_state(spec, dtype)
    prob.upload(X, 0, U)
    tr = prob.descend(X, 2000, 1e-3, every=100)
    c = oracle_curve(spec)
    store = np.float32 if dtype == np.float32 else None
    Uo, Jo = oracle_descent(c, U, 2000, 1e-3, storage=store, trace_every=100)
    got = prob.download(X, 0)
    err = np.abs(got - Uo).max() / np.abs(Uo).max()
    print(f"workload 0 dtype={dtype.__name__}: state error after 2000 steps {err:.3e}")
    assert err <= tol
    trc = tr.cpu().numpy()[:, 0]
    ref = np.array(Jo)  # cost of the state entering each traced step
    assert np.all(np.abs(trc - ref) <= tol * ref)
    assert np.all(np.diff(trc) < 0)


def test_workload1_descent_10k_steps():
    """The whole 10^4-step FP32 descent of workload 1 (L=39, N_x=64, N_s=512)
    against the oracle run that rounds its state to FP32 after every step: the
    state and the traced cost at 1e-5.  The plain FP64 oracle run drifts away
    from both (7e-5 after 10^4 steps): increments below half an FP32 ulp of
    their coefficient are lost in every FP32 run, a property of the FP32 state,
    not of the kernels."""
    spec = ksinputs.config_specs(1)[0]
    prob = _prob([spec], torch.float32)
    X = prob.new_state()
    U = seeded_state(spec, np.float32)
    prob.upload(X, 0, U)
    tr = prob.descend(X, 10000, 1e-3, every=500).cpu().numpy()[:, 0]
    c = oracle_curve(spec)
    Uo, Jo = oracle_descent(c, U, 10000, 1e-3, storage=np.float32, trace_every=500)
    got = prob.download(X, 0)
    err = np.abs(got - Uo).max() / np.abs(Uo).max()
    print(f"workload 1: FP32 state error after 10^4 steps {err:.3e}", flush=True)
    assert err <= 1e-5
    ref = np.array(Jo)
    assert np.all(np.abs(tr - ref) <= 1e-5 * ref)
    assert np.all(np.diff(tr) < 0)


def test_driver_fp32_then_fp64_finish():
    """Curves sampled from KS trajectories (finite map) with a small perturbation:
    the driver descends in FP32, promotes to FP64 and reaches a J target."""
    from paper_2301_11704_amd.driver import GpuBackend, descend_to
    L, n_x, n_s, T = 22.0, 32, 65, 2.0
    c0 = oracle.Curve(3, n_x, L)
    specs, Us = [], []
    for i in range(2):
        rng = np.random.default_rng(np.random.SeedSequence([61, i]))
        u0 = ksinputs.smooth_coeffs(rng, 4, 1.0, c0.K + 1)
        traj = oracle.etdrk4_integrate(c0, u0, T / 256, 256, sample_every=4)  # 65 samples
        p = ksinputs.smooth_coeffs(rng, 4, 0.02, c0.K + 1)
        sig = np.arange(n_s) / (n_s - 1)
        U = traj + np.sin(np.pi * sig)[:, None] * p[None, :]
        specs.append(ksinputs.CurveSpec(n_s, n_x, L, 4, 1.0, 4, 0.02, True, (61, i), "finite", T))
        Us.append(U)
    prob = _prob(specs, torch.float32)
    X = prob.new_state()
    for c, U in enumerate(Us):
        prob.upload(X, c, U)
    b = GpuBackend(prob, X)
    J0 = np.sqrt(b.J2())
    # J first drops fast, then decays slowly along the slowest s-mode: a 20x
    # reduction with the FP64 switch at 2x exercises the whole policy
    b2, log = descend_to(b, dtau=1e-3, J_target=float(J0.min()) / 20, max_steps=300000,
                         every=100, chunk=1000, switch_J=float(J0.min()) / 2, stall_records=4)
    print("events:", log.events[-5:], "steps:", log.steps)
    assert b2.dtype == "f64"
    assert log.converged.all()
    Js = np.array([j for _, j in log.J_history])
    assert np.all(np.diff(Js, axis=0) <= 1e-3 * Js[:-1])
