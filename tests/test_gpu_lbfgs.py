"""GPU parity of the implicit-in-s preconditioner (ksc_precondition) and of
the batched L-BFGS built on it (paper_2301_11704_amd/lbfgs.py) against the
same L-BFGS with the FP64 oracle as its model.  Tolerances: FP32 1e-5, FP64
1e-12 relative to the largest entry for the preconditioner; the L-BFGS
iterates after 6 iterations within 1e-9 of the state (FP64)."""
import numpy as np
import pytest

import ksinputs
import oracle
from helpers import OracleOps, oracle_curve, seeded_state

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _specs(n=2, n_s=33, n_x=16):
    return [ksinputs.CurveSpec(n_s + 8 * i, n_x, 22.0, 4, 1.0, 4, 0.3, True, (150, i),
                               "finite" if i % 2 == 0 else "rational", 5.0 + 20 * i)
            for i in range(n)]


def _problem(specs, tdt):
    import paper_2301_11704_amd as ksc
    prob = ksc.Problem([ksc.CurveDesc(s.n_s, s.n_x, s.L, s.map, s.scale, s.s0) for s in specs],
                       dtype=tdt)
    prob.set_scheme("implicit_s")
    return prob


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_precondition_matches_oracle(dtype):
    tdt = torch.float64 if dtype == np.float64 else torch.float32
    tol = 1e-12 if dtype == np.float64 else 1e-5
    specs = _specs(3, 40, 32)
    prob = _problem(specs, tdt)
    G = prob.new_state()
    rng = np.random.default_rng(5)
    refs = []
    for c, s in enumerate(specs):
        cur = oracle_curve(s)
        g = rng.standard_normal((s.n_s, cur.K + 1)) + 1j * rng.standard_normal((s.n_s, cur.K + 1))
        g[0] = g[-1] = 0
        g[:, 0] = g[:, 0].real
        g = ksinputs.round_to(g, dtype)
        prob.upload(G, c, g)
        refs.append(oracle.precondition_implicit_s(cur, g, 0.05))
    out = prob.precondition(G, dtau=0.05)
    torch.cuda.synchronize()
    for c, ref in enumerate(refs):
        got = prob.download(out, c)
        err = np.abs(got - ref).max() / np.abs(ref).max()
        print(f"curve {c}: preconditioner error {err:.2e}", flush=True)
        assert err <= tol, err
        assert np.all(got[0] == 0) and np.all(got[-1] == 0) and np.all(got[:, 0].imag == 0)


def test_precondition_needs_the_implicit_s_scheme():
    import paper_2301_11704_amd as ksc
    s = _specs(1)[0]
    prob = ksc.Problem([ksc.CurveDesc(s.n_s, s.n_x, s.L, s.map, s.scale, s.s0)],
                       dtype=torch.float64)
    G = prob.new_state()
    with pytest.raises(Exception):
        prob.precondition(G)


def test_lbfgs_iterates_match_the_oracle_model():
    """Six batched L-BFGS iterations (memory 4) on the GPU and with the
    oracle as the model, from the same FP64 curves: the iterates agree to
    1e-9 of the state and J^2 never rises."""
    from paper_2301_11704_amd.lbfgs import BatchLBFGS, TorchOps
    specs = _specs(2)
    prob = _problem(specs, torch.float64)
    X = prob.new_state()
    Us = []
    for c, s in enumerate(specs):
        U = seeded_state(s, np.float64)
        prob.upload(X, c, U)
        Us.append(U)
    curves = [oracle_curve(s) for s in specs]
    dtau = 0.05
    gpu = BatchLBFGS(TorchOps(prob, dtau), m=4)
    cpu_ops = OracleOps(curves, dtau)
    cpu = BatchLBFGS(cpu_ops, m=4)
    gpu.start(X)
    cpu.start(cpu_ops.flat(Us))
    act_g = torch.ones(2, dtype=torch.bool, device=X.device)
    act_c = torch.ones(2, dtype=torch.bool)
    prev = gpu.J2.cpu().clone()
    for it in range(6):
        Jg = gpu.iterate(act_g).cpu()
        cpu.iterate(act_c)
        assert torch.all(Jg <= prev * (1 + 1e-12))
        prev = Jg.clone()
        for c in range(2):
            got = prob.download(gpu.x, c)
            ref = cpu_ops.unflat(cpu.x, c)
            err = np.abs(got - ref).max() / np.abs(ref).max()
            assert err <= 1e-9, (it, c, err)
    print("L-BFGS J2 after 6 iterations:", prev.numpy(), "from",
          [oracle.J2(c, U) for c, U in zip(curves, Us)], flush=True)


def test_workload4_reduced_descent_reaches_1e8_with_lbfgs():
    """Two curves of workload 4 on 256 rows: implicit-in-s steps in FP32, the
    FP64 switch at J = 2e-3, then batched L-BFGS (memory 8) to J < 1e-8; the
    final J agrees with the oracle's J of the downloaded state."""
    import paper_2301_11704_amd as ksc
    from paper_2301_11704_amd.driver import GpuBackend, descend_to
    specs, Us = ksinputs.config4_curves(4, 256)
    pick = [0, 3]
    specs, Us = [specs[i] for i in pick], [Us[i] for i in pick]
    prob = ksc.Problem([ksc.CurveDesc(s.n_s, s.n_x, s.L, s.map, s.scale, s.s0) for s in specs],
                       dtype=torch.float32)
    prob.set_scheme("implicit_s")
    X = prob.new_state()
    for c, U in enumerate(Us):
        prob.upload(X, c, ksinputs.round_to(U, np.float32))
    b, log = descend_to(GpuBackend(prob, X), dtau=0.05, J_target=1e-8, max_steps=400_000,
                        every=1000, chunk=20000, switch_J=2e-3, stall_records=5, lbfgs=8,
                        lbfgs_chunk=500)
    print("events:", log.events, "steps:", log.steps, flush=True)
    assert b.dtype == "f64" and log.converged.all()
    J = np.sqrt(b.J2())
    for c, s in enumerate(specs):
        U = b.prob.download(b.state, c)
        ref = np.sqrt(oracle.J2(oracle_curve(s), U))
        assert J[c] < 1e-8 and abs(J[c] - ref) <= 1e-5 * ref, (J[c], ref)
