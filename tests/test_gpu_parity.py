"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.  Tolerances: FP32 1e-5 relative, FP64 1e-12 relative."""
import numpy as np
import pytest

import ksinputs
import oracle
from helpers import (directional_rel_err, elementwise_rel_err, oracle_curve, oracle_descent,
                     precond_rel_err, seeded_state)

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

TOL = {np.float32: 1e-5, np.float64: 1e-12}


def _tdt(dtype):
    return torch.float32 if dtype == np.float32 else torch.float64


def _problem(specs, dtype, waves=None, policy=None):
    import paper_2301_11704_amd as ksc
    descs = [ksc.CurveDesc(s.n_s, s.n_x, s.L, s.map, s.scale, s.s0) for s in specs]
    prob = ksc.Problem(descs, dtype=_tdt(dtype))
    if waves is not None or policy is not None:
        prob.set_launch(policy or ksc.KSC_LAUNCH_AUTO, waves or 0)
    return prob


def _load(prob, specs, dtype):
    X = prob.new_state()
    Us = []
    for c, s in enumerate(specs):
        U = seeded_state(s, dtype)
        prob.upload(X, c, U)
        Us.append(U)
    return X, Us


def _spec(n_s, n_x, L=22.0, seed=(90, 0), map_="rational", scale=40.0):
    return ksinputs.CurveSpec(n_s, n_x, L, min(6, (n_x - 1) // 3), 1.0, min(6, (n_x - 1) // 3),
                              0.2, True, seed, map_, scale)


# ---------------------------------------------------------------- boundary --

@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("n_x", [8, 16, 32, 64, 128, 256])
def test_phys_spec_conversions(dtype, n_x):
    print(f"conversions n_x={n_x} dtype={dtype.__name__}", flush=True)
    spec = _spec(37, n_x)
    prob = _problem([spec], dtype)
    K1 = oracle.n_modes(n_x)
    rng = np.random.default_rng(n_x)
    phys = rng.standard_normal((spec.n_s, n_x)).astype(dtype)
    P = torch.from_numpy(phys.ravel()).cuda()
    X = prob.phys_to_spec(P)
    got = prob.download(X, 0)
    ref = oracle.to_spectral(phys.astype(np.float64), K1 - 1)
    ref[:, 0] = ref[:, 0].real
    tol = TOL[dtype] * 10
    assert np.abs(got - ref).max() <= tol * np.abs(ref).max()
    back = prob.spec_to_phys(X).cpu().numpy().reshape(spec.n_s, n_x)
    ref_back = oracle.to_physical(prob.download(X, 0), n_x)
    assert np.abs(back - ref_back).max() <= tol * np.abs(ref_back).max()


# ------------------------------------------------------------ cost / grad --

CASES = [
    # (n_s, n_x, map, scale): several tiles and ragged tails for every tile shape
    (3, 32, "rational", 40.0),
    (4, 16, "finite", 3.0),
    (64, 32, "rational", 40.0),
    (127, 64, "rational", 40.0),
    (200, 64, "finite", 5.0),
    (131, 128, "rational", 40.0),
    (70, 256, "rational", 40.0),
    (300, 8, "finite", 2.0),
    # rows split over lanes (16 per row at N_x = 256 in FP32: 4W-row tiles; a
    # lane pair per row at N_x >= 128 in FP64: 32W-row tiles): several tiles
    (300, 256, "finite", 4.0),
    (520, 128, "finite", 6.0),
]


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("waves", [1, 2, 4])
def test_J2_and_gradient_parity(dtype, case, waves):
    n_s, n_x, map_, scale = case
    print(f"parity n_s={n_s} n_x={n_x} map={map_} waves={waves} dtype={dtype.__name__}", flush=True)
    spec = _spec(n_s, n_x, 39.0, (91, n_s), map_, scale)
    import paper_2301_11704_amd as ksc
    try:
        prob = _problem([spec], dtype, waves=waves)
    except ksc.KscError as e:
        assert e.status == -3  # tile does not fit in LDS for this shape
        pytest.skip("tile shape exceeds LDS")
    X, (U,) = _load(prob, [spec], dtype)
    c = oracle_curve(spec)
    J2, Jarc = prob.eval_J(X, arc=True)
    G, J2g = prob.eval_grad(X)
    torch.cuda.synchronize()
    J2_ref = oracle.J2(c, U)
    tol = TOL[dtype]
    assert abs(J2.item() - J2_ref) <= tol * J2_ref
    assert abs(J2g.item() - J2_ref) <= tol * J2_ref
    Ja_ref = oracle.J_arc(c, U)
    assert abs(Jarc.item() - Ja_ref) <= tol * Ja_ref
    Gg = prob.download(G, 0)
    Gr = oracle.grad(c, U)
    assert np.all(Gg[0] == 0) and np.all(Gg[-1] == 0)
    assert np.all(Gg[:, 0].imag == 0)
    e_pre = precond_rel_err(c, Gg, Gr)
    e_dir = directional_rel_err(c, Gg, Gr, [(7, i) for i in range(16)])
    e_el = elementwise_rel_err(c, Gg, Gr)
    assert e_pre <= tol, e_pre
    assert e_dir <= tol, e_dir
    assert e_el <= tol, e_el


FULL = [(16, 300), (32, 300), (64, 300), (128, 300), (256, 300)]


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("n_x,n_s", FULL)
@pytest.mark.parametrize("waves", [1, 4])
def test_full_spectrum_parity(dtype, n_x, n_s, waves):
    """Every kept mode populated and independent noise from row to row (the
    smooth seeded states fill only k <= 6): J2, J_arc, the gradient and one
    step against the oracle, for both lane layouts (one lane per row; a lane
    pair for N_x = 256 and for FP64 N_x = 128) and for odd and even K+1."""
    print(f"full spectrum n_x={n_x} n_s={n_s} waves={waves} dtype={dtype.__name__}", flush=True)
    spec = _spec(n_s, n_x, 39.0, (96, n_x), "finite", 4.0)
    import paper_2301_11704_amd as ksc
    try:
        prob = _problem([spec], dtype, waves=waves)
    except ksc.KscError as e:
        assert e.status == -3
        pytest.skip("tile shape exceeds LDS")
    K1 = oracle.n_modes(n_x)
    U = ksinputs.round_to(ksinputs.full_spectrum_curve(n_s, K1, (96, n_x, n_s)), dtype)
    U[:, 0] = U[:, 0].real
    X = prob.new_state()
    prob.upload(X, 0, U)
    c = oracle_curve(spec)
    J2, Jarc = prob.eval_J(X, arc=True)
    G, J2g = prob.eval_grad(X)
    Y = torch.empty_like(X)
    prob.step(X, Y, 1e-4)
    torch.cuda.synchronize()
    tol = TOL[dtype]
    J2_ref = oracle.J2(c, U)
    assert abs(J2.item() - J2_ref) <= tol * J2_ref
    assert abs(J2g.item() - J2_ref) <= tol * J2_ref
    Ja_ref = oracle.J_arc(c, U)
    assert abs(Jarc.item() - Ja_ref) <= tol * Ja_ref
    Gg = prob.download(G, 0)
    Gr = oracle.grad(c, U)
    assert precond_rel_err(c, Gg, Gr) <= tol
    assert elementwise_rel_err(c, Gg, Gr) <= tol
    assert directional_rel_err(c, Gg, Gr, [(8, i) for i in range(8)]) <= tol
    got = prob.download(Y, 0)
    ref = oracle.step(c, U, 1e-4)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= tol


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("n_s,n_x", [(150, 64), (300, 128), (300, 256)])
def test_step_parity(dtype, n_s, n_x):
    print(f"step parity n_s={n_s} n_x={n_x} dtype={dtype.__name__}", flush=True)
    spec = _spec(n_s, n_x, 22.0 if n_x < 256 else 60.0, (92, n_x))
    prob = _problem([spec], dtype)
    X, (U,) = _load(prob, [spec], dtype)
    c = oracle_curve(spec)
    Y = torch.empty_like(X)
    J2 = prob.step(X, Y, 1e-3, want_J2=True)
    torch.cuda.synchronize()
    got = prob.download(Y, 0)
    ref = oracle.step(c, U, 1e-3)
    assert abs(J2.item() - oracle.J2(c, U)) <= TOL[dtype] * oracle.J2(c, U)
    assert np.array_equal(got[0], U[0]) and np.array_equal(got[-1], U[-1])
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert err <= TOL[dtype], err
    # every element of the state after the step
    assert np.abs(got - ref).max() <= TOL[dtype] * np.abs(ref).max()


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_descend_matches_oracle_and_single_steps(dtype):
    spec = ksinputs.config_specs(0)[0]
    prob = _problem([spec], dtype)
    X, (U,) = _load(prob, [spec], dtype)
    c = oracle_curve(spec)
    n, every = 40, 8
    X2 = X.clone()
    tr = prob.descend(X, n, 1e-3, every=every)
    # the same steps one at a time must agree bitwise (same kernels, same order)
    Y = torch.empty_like(X2)
    for i in range(n):
        prob.step(X2, Y, 1e-3)
        X2, Y = Y, X2
    torch.cuda.synchronize()
    assert torch.equal(X, X2)
    Ur = U.copy()
    Jr = []
    for i in range(n):
        Jr.append(oracle.J2(c, Ur))
        Ur = oracle.step(c, Ur, 1e-3)
    got = prob.download(X, 0)
    assert np.linalg.norm(got - Ur) / np.linalg.norm(Ur) <= 4 * TOL[dtype]
    trc = tr.cpu().numpy()[:, 0]
    for g in range(n // every):
        ref = Jr[(g + 1) * every - 1]
        assert abs(trc[g] - ref) <= 4 * TOL[dtype] * ref


@pytest.mark.parametrize("dtype,n_curves", [(np.float32, 256), (np.float64, 24)])
def test_batched_uneven_curves_match_oracle(dtype, n_curves):
    """One launch over curves of different n_x, n_s and L (the mixed kernel;
    in FP64 its N_x = 128 tiles use two lanes per row): in FP32 every curve of
    the 256-curve uneven workload (N_s up to 2048), in FP64 the first 24 - the
    cost, J_arc, the gradient (norm, directions, every element) and one step,
    under both launch policies."""
    specs = ksinputs.config_specs(3, n_curves=n_curves)
    tol = TOL[dtype]
    dtau = 1e-3
    for policy in (0, 2):
        print(f"uneven batch dtype={dtype.__name__} curves={n_curves} policy={policy}", flush=True)
        prob = _problem(specs, dtype, policy=policy)
        X, Us = _load(prob, specs, dtype)
        J2, Ja = prob.eval_J(X, arc=True)
        G, J2g = prob.eval_grad(X)
        Y = torch.empty_like(X)
        prob.step(X, Y, dtau)
        torch.cuda.synchronize()
        J2, Ja, J2g = J2.cpu().numpy(), Ja.cpu().numpy(), J2g.cpu().numpy()
        worst = {}
        for i, (s, U) in enumerate(zip(specs, Us)):
            c = oracle_curve(s)
            ref = oracle.J2(c, U)
            Gg, Gr = prob.download(G, i), oracle.grad(c, U)
            St, Sr = prob.download(Y, i), oracle.step(c, U, dtau)
            errs = {
                "J2": abs(J2[i] - ref) / ref, "J2_grad": abs(J2g[i] - ref) / ref,
                "J_arc": abs(Ja[i] - oracle.J_arc(c, U)) / oracle.J_arc(c, U),
                "pre": precond_rel_err(c, Gg, Gr), "elem": elementwise_rel_err(c, Gg, Gr),
                "dir": directional_rel_err(c, Gg, Gr, [(7, k) for k in range(4)]),
                "step": np.abs(St - Sr).max() / np.abs(Sr).max(),
            }
            for k, v in errs.items():
                if v > worst.get(k, (0.0,))[0]:
                    worst[k] = (v, i, s.n_s, s.n_x)
            assert max(errs.values()) <= tol, (i, s, errs)
        print("  worst per metric (error, curve, n_s, n_x):", worst, flush=True)


def test_uneven_batch_graph_descent_matches_oracle_steps():
    """The captured-graph descent (ksc_descend) of an uneven batch against the
    oracle's steps, curve by curve: 100 steps in graphs of 10, J^2 traced
    after every graph; the FP32 state is compared with the oracle run whose
    state is rounded to FP32 after every step (what an FP32 state holds)."""
    specs = ksinputs.config_specs(3, n_curves=256)
    # both ends of the length range and every grid size
    pick = sorted({min(range(256), key=lambda i: specs[i].n_s),
                   max(range(256), key=lambda i: specs[i].n_s)} |
                  {next(i for i in range(256) if specs[i].n_x == nx) for nx in (32, 64, 128)})
    sub = [specs[i] for i in pick]
    prob = _problem(sub, np.float32)
    X, Us = _load(prob, sub, np.float32)
    n, every, dtau = 100, 10, 1e-3
    tr = prob.descend(X, n, dtau, every=every).cpu().numpy()
    for i, (s, U) in enumerate(zip(sub, Us)):
        c = oracle_curve(s)
        ref, jr = oracle_descent(c, U, n, dtau, storage=np.float32, trace_every=every)
        got = prob.download(X, i)
        err = np.abs(got - ref).max() / np.abs(ref).max()
        print(f"curve {pick[i]} n_s={s.n_s} n_x={s.n_x}: state error after {n} steps {err:.2e}",
              flush=True)
        assert err <= 1e-5, err
        # the trace holds the cost of the state the last step of each graph started from
        assert np.all(np.abs(tr[:, i] - jr) <= 1e-5 * np.array(jr)), (tr[:, i], jr)


def test_plain_policy_matches_batched_bitwise():
    import paper_2301_11704_amd as ksc
    specs = ksinputs.config_specs(4, n_curves=4)
    specs = [ksinputs.CurveSpec(256, s.n_x, s.L, 6, 1.0, 4, 0.1, True, s.seed, s.map, s.scale)
             for s in specs]
    prob = _problem(specs, np.float32)
    X, _ = _load(prob, specs, np.float32)
    G1, J1 = prob.eval_grad(X)
    prob.set_launch(ksc.KSC_LAUNCH_PLAIN, 0)
    G2, J2 = prob.eval_grad(X)
    prob.set_launch(ksc.KSC_LAUNCH_PERSISTENT, 0)
    G3, J3 = prob.eval_grad(X)
    torch.cuda.synchronize()
    assert torch.equal(G1, G2) and torch.equal(G1, G3)
    assert torch.equal(J1, J2) and torch.equal(J1, J3)


def test_deterministic():
    spec = ksinputs.config_specs(1)[0]
    prob = _problem([spec], np.float32)
    X, _ = _load(prob, [spec], np.float32)
    a, ja = prob.eval_grad(X)
    b, jb = prob.eval_grad(X)
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(ja, jb)


def test_config2_full_size_parity():
    """The large single curve (L=100, N_x=256, N_s=8192) against the oracle:
    the cost, J_arc, the gradient (norm, directions, every element) and one
    step, all at the FP32 tolerance."""
    spec = ksinputs.config_specs(2)[0]
    prob = _problem([spec], np.float32)
    X, (U,) = _load(prob, [spec], np.float32)
    c = oracle_curve(spec)
    J2, Ja = prob.eval_J(X, arc=True)
    G, _ = prob.eval_grad(X)
    Y = torch.empty_like(X)
    prob.step(X, Y, 1e-4)
    torch.cuda.synchronize()
    ref = oracle.J2(c, U)
    assert abs(J2.item() - ref) <= 1e-5 * ref
    assert abs(Ja.item() - oracle.J_arc(c, U)) <= 1e-5 * oracle.J_arc(c, U)
    Gg = prob.download(G, 0)
    Gr = oracle.grad(c, U)
    e = (precond_rel_err(c, Gg, Gr), elementwise_rel_err(c, Gg, Gr),
         directional_rel_err(c, Gg, Gr, [(8, i) for i in range(16)]))
    print("workload 2 gradient errors (preconditioned, element-wise, directional):", e, flush=True)
    assert max(e) <= 1e-5, e
    St, Sr = prob.download(Y, 0), oracle.step(c, U, 1e-4)
    assert np.abs(St - Sr).max() <= 1e-5 * np.abs(Sr).max()


def test_flags_nonfinite_isolated_per_curve():
    specs = [_spec(40, 32, 22.0, (93, i)) for i in range(3)]
    prob = _problem(specs, np.float32)
    X, _ = _load(prob, specs, np.float32)
    v = prob.view(X, 1)
    v[5, 2, 0] = float("nan")
    Y = torch.empty_like(X)
    act = torch.ones(3, dtype=torch.uint8, device="cuda")
    prob.descend(X, 4, 1e-3, every=2, scratch=Y, active=act)
    flags = prob.query_flags()
    assert flags[1] & 1
    assert flags[0] == 0 and flags[2] == 0


def test_argument_errors():
    import paper_2301_11704_amd as ksc
    with pytest.raises(ksc.KscError) as e:
        ksc.Problem([ksc.CurveDesc(2, 32, 22.0)])
    assert e.value.status == -2
    with pytest.raises(ksc.KscError) as e:
        ksc.Problem([ksc.CurveDesc(10, 48, 22.0)])
    assert e.value.status == -3
    with pytest.raises(ksc.KscError):
        ksc.Problem([ksc.CurveDesc(10, 32, -1.0)])
    prob = ksc.Problem([ksc.CurveDesc(10, 32, 22.0)])
    X = prob.new_state()
    with pytest.raises(ksc.KscError):
        prob.step(X, X, 1e-3)


def test_kernel_timing_window():
    """Timed evaluations give the same results; descend's graphs are not timed."""
    spec = ksinputs.config_specs(1)[0]
    prob = _problem([spec], np.float32)
    X, _ = _load(prob, [spec], np.float32)
    G0, J0 = prob.eval_grad(X)
    prob.set_timing(True)
    for _ in range(5):
        G1, J1 = prob.eval_grad(X)
    prob.eval_J(X)
    Y = torch.empty_like(X)
    prob.step(X, Y, 1e-3)
    Z = X.clone()
    prob.descend(Z, 4, 1e-3, every=2, scratch=Y)
    fused, post, n = prob.read_timing()
    prob.set_timing(False)
    torch.cuda.synchronize()
    assert n == 7
    assert fused > 0 and post > 0
    assert torch.equal(G0, G1) and torch.equal(J0, J1)
    prob.set_timing(True)
    assert prob.read_timing()[2] == 0
    prob.set_timing(False)
