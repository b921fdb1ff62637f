"""GPU parity of the spectral d/ds (the paper's rational Chebyshev D_t applied
along s on matrix cores) against the FP64 oracle's Curve(ds="spectral"), on
the same seeded inputs.  Tolerances as for the stencil path, FP32 1e-5 and
FP64 1e-12 relative, except for FP64 gradients whose s-part sum cancels
strongly: the adjoint's s-part sums D_t[j, i] w_j r_j over j, and the ratio
kappa of the sum of the magnitudes of the terms to the result (2-norms over
the curve) reaches 421 at N_s = 552.  The FP64 oracle itself is then off by
2.5e-12 (measured against a long-double evaluation of the s-products, about
6e-15 kappa), so an FP64 gradient is gated at max(1e-12, 2e-14 kappa)."""
import numpy as np
import pytest

import ksinputs
import oracle
from helpers import directional_rel_err, precond_rel_err

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

TOL = {np.float32: 1e-5, np.float64: 1e-12}


def _tdt(dtype):
    return torch.float32 if dtype == np.float32 else torch.float64


def _spec(n_s, n_x, L=22.0, seed=(110, 0), scale=8.0):
    kmax = min(6, (n_x - 1) // 3)
    return ksinputs.CurveSpec(n_s, n_x, L, kmax, 1.0, kmax, 0.2, True, seed, "rational", scale)


def _curve(spec):
    return oracle.Curve(spec.n_s, spec.n_x, spec.L, "rational", spec.scale, spec.s0, ds="spectral")


def _problem(specs, dtype, waves=None, policy=None):
    import paper_2301_11704_amd as ksc
    descs = [ksc.CurveDesc(s.n_s, s.n_x, s.L, s.map, s.scale, s.s0) for s in specs]
    prob = ksc.Problem(descs, dtype=_tdt(dtype), ds="spectral")
    if waves is not None or policy is not None:
        prob.set_launch(policy or ksc.KSC_LAUNCH_AUTO, waves or 0)
    return prob


def _state(spec, dtype, full_spectrum=False):
    K1 = oracle.n_modes(spec.n_x)
    if full_spectrum:
        U = ksinputs.full_spectrum_curve(spec.n_s, K1, spec.seed, amp=0.3, rough=0.02)
    else:
        _, _, U = ksinputs.make_curve(spec, K1)
    U[:, 0] = U[:, 0].real
    return ksinputs.round_to(U, dtype)


def _kappa(c, U):
    """Cancellation factor of the s-part of the adjoint for this curve."""
    R = oracle.residual(c, U)
    WR = c.w[:, None] * R
    S = c.D.T @ WR
    M = np.abs(c.D.T) @ np.abs(WR)
    return float(np.linalg.norm(M[1:-1]) / np.linalg.norm(S[1:-1]))


def _grad_tol(c, U, dtype):
    if dtype == np.float32:
        return TOL[dtype]
    return max(TOL[dtype], 2e-14 * _kappa(c, U))


def _check(prob, X, c, U, dtype, i=0, dtau=1e-4):
    J2, Jarc = prob.eval_J(X, arc=True)
    G, J2g = prob.eval_grad(X)
    Y = torch.empty_like(X)
    J2s = prob.step(X, Y, dtau, want_J2=True)
    torch.cuda.synchronize()
    tol = TOL[dtype]
    ref = oracle.J2(c, U)
    for v in (J2[i].item(), J2g[i].item(), J2s[i].item()):
        assert abs(v - ref) <= tol * ref, (v, ref)
    Ja = oracle.J_arc(c, U)
    assert abs(Jarc[i].item() - Ja) <= tol * Ja
    Gg = prob.download(G, i)
    Gr = oracle.grad(c, U)
    assert np.all(Gg[0] == 0) and np.all(Gg[-1] == 0) and np.all(Gg[:, 0].imag == 0)
    e_pre = precond_rel_err(c, Gg, Gr)
    e_dir = directional_rel_err(c, Gg, Gr, [(111, j) for j in range(8)])
    tg = _grad_tol(c, U, dtype)
    print(f"gradient errors: preconditioned {e_pre:.2e}, directional {e_dir:.2e} (gate {tg:.1e})",
          flush=True)
    assert e_pre <= tg, e_pre
    assert e_dir <= tg, e_dir
    got = prob.download(Y, i)
    want = oracle.step(c, U, dtau)
    assert np.array_equal(got[0], U[0]) and np.array_equal(got[-1], U[-1])
    err = np.linalg.norm(got - want) / np.linalg.norm(want)
    assert err <= tol, err


CASES = [
    # (n_s, n_x): ragged against the 64-row product blocks and the row tiles
    (3, 16), (17, 8), (64, 32), (65, 64), (130, 32), (300, 64), (200, 128), (552, 64),
]


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("waves", [1, 2])
def test_spectral_parity(dtype, case, waves):
    n_s, n_x = case
    print(f"spectral parity n_s={n_s} n_x={n_x} waves={waves} dtype={dtype.__name__}", flush=True)
    if dtype == np.float64 and n_x > 64:
        pytest.skip("the spectral d/ds in FP64 supports n_x <= 64")
    spec = _spec(n_s, n_x, 22.0 if n_x <= 64 else 39.0, (110, n_s, n_x))
    prob = _problem([spec], dtype, waves=waves)
    U = _state(spec, dtype)
    X = prob.new_state()
    prob.upload(X, 0, U)
    _check(prob, X, _curve(spec), U, dtype)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("n_x", [16, 64])
def test_spectral_full_spectrum(dtype, n_x):
    """Every kept mode populated and row-to-row noise (content at every
    s-frequency the matrix can represent)."""
    spec = _spec(160, n_x, 22.0, (112, n_x), scale=20.0)
    prob = _problem([spec], dtype)
    U = _state(spec, dtype, full_spectrum=True)
    X = prob.new_state()
    prob.upload(X, 0, U)
    _check(prob, X, _curve(spec), U, dtype)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_spectral_batched_uneven_and_policies(dtype):
    """Curves of different n_s, n_x, L and S in one problem (one product
    launch per n_x group); every launch policy gives the same bits."""
    import paper_2301_11704_amd as ksc
    shapes = [(130, 32, 22.0, 8.0), (67, 64, 22.0, 20.0), (201, 16, 12.0, 5.0), (64, 32, 30.0, 40.0),
              (300, 64, 39.0, 55.0)]
    specs = [ksinputs.CurveSpec(n_s, n_x, L, min(6, (n_x - 1) // 3), 1.0, min(6, (n_x - 1) // 3), 0.2,
                                True, (113, i), "rational", S)
             for i, (n_s, n_x, L, S) in enumerate(shapes)]
    prob = _problem(specs, dtype)
    X = prob.new_state()
    Us = []
    for i, s in enumerate(specs):
        U = _state(s, dtype)
        prob.upload(X, i, U)
        Us.append(U)
    outs = []
    for policy in (ksc.KSC_LAUNCH_AUTO, ksc.KSC_LAUNCH_PLAIN, ksc.KSC_LAUNCH_PERSISTENT):
        prob.set_launch(policy, 0)
        G, J2 = prob.eval_grad(X)
        outs.append((G.clone(), J2.clone()))
    torch.cuda.synchronize()
    for G, J2 in outs[1:]:
        assert torch.equal(G, outs[0][0]) and torch.equal(J2, outs[0][1])
    tol = TOL[dtype]
    J2 = outs[0][1].cpu().numpy()
    for i, (s, U) in enumerate(zip(specs, Us)):
        c = _curve(s)
        ref = oracle.J2(c, U)
        assert abs(J2[i] - ref) <= tol * ref, i
        assert precond_rel_err(c, prob.download(outs[0][0], i), oracle.grad(c, U)) <= \
            _grad_tol(c, U, dtype), i


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_spectral_descend_matches_single_steps_and_oracle(dtype):
    spec = _spec(100, 32, 22.0, (114, 0), scale=10.0)
    prob = _problem([spec], dtype)
    U = _state(spec, dtype)
    X = prob.new_state()
    prob.upload(X, 0, U)
    X2 = X.clone()
    n, every, dtau = 24, 8, 1e-3
    tr = prob.descend(X, n, dtau, every=every)
    Y = torch.empty_like(X2)
    for _ in range(n):
        prob.step(X2, Y, dtau)
        X2, Y = Y, X2
    torch.cuda.synchronize()
    assert torch.equal(X, X2)
    c = _curve(spec)
    Ur = U.copy()
    Jr = []
    for _ in range(n):
        Jr.append(oracle.J2(c, Ur))
        Ur = oracle.step(c, Ur, dtau)
    got = prob.download(X, 0)
    assert np.linalg.norm(got - Ur) / np.linalg.norm(Ur) <= 4 * TOL[dtype]
    trc = tr.cpu().numpy()[:, 0]
    for g in range(n // every):
        ref = Jr[(g + 1) * every - 1]
        assert abs(trc[g] - ref) <= 4 * TOL[dtype] * ref


def test_spectral_autograd_matches_eval_grad_and_is_deterministic():
    import paper_2301_11704_amd as ksc
    spec = _spec(90, 32, 22.0, (115, 0))
    prob = _problem([spec], np.float64)
    X = prob.new_state()
    prob.upload(X, 0, _state(spec, np.float64))
    Xr = X.clone().requires_grad_(True)
    J = ksc.curve_J2(Xr, prob)
    (3.0 * J.sum()).backward()
    G, _ = prob.eval_grad(X)
    G2, _ = prob.eval_grad(X)
    torch.cuda.synchronize()
    assert torch.equal(G, G2)
    assert torch.allclose(Xr.grad, 3.0 * G, rtol=1e-14, atol=0)


def test_spectral_descent_from_E1_to_E2_matches_oracle():
    """The paper's first connection (E1 -> E2, N_x = 64, N_s = 552, S = 55,
    dtau = 0.01) for 60 steps in FP64 against 60 oracle steps."""
    spec, U = ksinputs.l22_connection_curve("E1", "E2")
    prob = _problem([spec], np.float64)
    X = prob.new_state()
    prob.upload(X, 0, U)
    tr = prob.descend(X, 60, 0.01, every=20)
    torch.cuda.synchronize()
    c = _curve(spec)
    Ur = U.copy()
    Jr = []
    for _ in range(60):
        Jr.append(oracle.J2(c, Ur))
        Ur = oracle.step(c, Ur, 0.01)
    # per-step rounding differences of at most 1e-12 add up over 60 steps
    got = prob.download(X, 0)
    assert np.linalg.norm(got - Ur) / np.linalg.norm(Ur) <= 60 * TOL[np.float64]
    trc = tr.cpu().numpy()[:, 0]
    for g in range(3):
        assert abs(trc[g] - Jr[20 * g + 19]) <= 60 * TOL[np.float64] * Jr[20 * g + 19]


def _embed(B):
    U = np.zeros((B.shape[0], B.shape[1] + 1), dtype=np.complex128)
    U[:, 1:] = 1j * B
    return U


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("n_s,n_x", [(3, 16), (17, 8), (130, 32), (300, 64), (552, 64), (200, 128)])
def test_spectral_odd_parity(dtype, n_s, n_x):
    """The spectral d/ds in the inversion-symmetric subspace (rows of K reals)
    against the oracle's restriction to it."""
    import paper_2301_11704_amd as ksc
    print(f"spectral odd parity n_s={n_s} n_x={n_x} dtype={dtype.__name__}", flush=True)
    if dtype == np.float64 and n_x > 64:
        pytest.skip("the spectral d/ds in FP64 supports n_x <= 64")
    spec = _spec(n_s, n_x, 22.0 if n_x <= 64 else 39.0, (116, n_s, n_x))
    descs = [ksc.CurveDesc(spec.n_s, spec.n_x, spec.L, spec.map, spec.scale, spec.s0)]
    prob = ksc.Problem(descs, dtype=_tdt(dtype), ds="spectral", space="odd")
    U = _state(spec, dtype)
    B = np.ascontiguousarray(U[:, 1:].imag)
    X = prob.new_state()
    prob.upload(X, 0, B)
    c = _curve(spec)
    J2, Jarc = prob.eval_J(X, arc=True)
    G, J2g = prob.eval_grad(X)
    Y = torch.empty_like(X)
    prob.step(X, Y, 1e-4)
    torch.cuda.synchronize()
    tol = TOL[dtype]
    ref = oracle.J2_odd(c, B)
    assert abs(J2.item() - ref) <= tol * ref and abs(J2g.item() - ref) <= tol * ref
    Ja = oracle.J_arc_odd(c, B)
    assert abs(Jarc.item() - Ja) <= tol * Ja
    Gg, Gr = _embed(prob.download(G, 0)), _embed(oracle.grad_odd(c, B))
    tg = _grad_tol(c, _embed(B), dtype)
    e_pre = precond_rel_err(c, Gg, Gr)
    e_dir = directional_rel_err(c, Gg, Gr, [(117, j) for j in range(8)])
    print(f"gradient errors: preconditioned {e_pre:.2e}, directional {e_dir:.2e} (gate {tg:.1e})",
          flush=True)
    assert e_pre <= tg and e_dir <= tg
    got, want = prob.download(Y, 0), oracle.step_odd(c, B, 1e-4)
    assert np.array_equal(got[0], B[0]) and np.array_equal(got[-1], B[-1])
    assert np.linalg.norm(got - want) / np.linalg.norm(want) <= tol


def test_spectral_odd_descent_matches_full_space():
    """E1 -> E2 for 60 steps in the odd subspace and in the full space: the
    same trajectory (the full-space run's imaginary parts) to rounding."""
    import paper_2301_11704_amd as ksc
    spec, U = ksinputs.l22_connection_curve("E1", "E2")
    d = [ksc.CurveDesc(spec.n_s, spec.n_x, spec.L, spec.map, spec.scale, spec.s0)]
    pf = ksc.Problem(d, dtype=torch.float64, ds="spectral")
    po = ksc.Problem(d, dtype=torch.float64, ds="spectral", space="odd")
    Xf, Xo = pf.new_state(), po.new_state()
    pf.upload(Xf, 0, U)
    po.upload(Xo, 0, np.ascontiguousarray(U[:, 1:].imag))
    tf = pf.descend(Xf, 60, 0.01, every=20)
    to = po.descend(Xo, 60, 0.01, every=20)
    torch.cuda.synchronize()
    uf, bo = pf.download(Xf, 0), po.download(Xo, 0)
    assert np.abs(uf.real).max() <= 1e-14 * np.abs(uf).max()
    assert np.linalg.norm(bo - uf[:, 1:].imag) <= 60 * TOL[np.float64] * np.linalg.norm(bo)
    assert np.allclose(to.cpu().numpy(), tf.cpu().numpy(), rtol=60 * TOL[np.float64], atol=0)


def test_spectral_paper_shape_batch_in_the_bench_configuration():
    """The 64-curve paper-shape batch (N_x = 64, N_s = 552, S = 55; FP32 state)
    with the launch shape the benchmark uses: J2 of every curve, and the
    gradient and a step of three sampled curves, against the oracle."""
    import os
    import paper_2301_11704_amd as ksc
    specs = ksinputs.paper_shape_specs(64)
    prob = ksc.Problem([ksc.CurveDesc(s.n_s, s.n_x, s.L, s.map, s.scale, s.s0) for s in specs],
                       dtype=torch.float32, ds="spectral")
    prob.tune(os.path.join(os.path.dirname(ksc.__file__), "tuning_gfx950.json"))
    X = prob.new_state()
    Us = []
    for i, s in enumerate(specs):
        U = ksinputs.round_to(ksinputs.make_curve(s, (s.n_x - 1) // 3 + 1)[2], np.float32)
        U[:, 0] = U[:, 0].real
        prob.upload(X, i, U)
        Us.append(U)
    J2 = prob.eval_J(X).cpu().numpy()
    for i, s in enumerate(specs):
        ref = oracle.J2(_curve(s), Us[i])
        assert abs(J2[i] - ref) <= TOL[np.float32] * ref, (i, J2[i], ref)
    for i in (0, 31, 63):
        print(f"paper-shape batch, curve {i}", flush=True)
        _check(prob, X, _curve(specs[i]), Us[i], np.float32, i=i, dtau=0.01)
