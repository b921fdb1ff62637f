"""GPU parity of the inversion-symmetric subspace (state space "odd": rows of
K reals b_k with u_hat_k = i b_k) against the FP64 oracle's restriction of the
full method to that subspace, on the same seeded inputs.  Tolerances as for
the full space: FP32 1e-5 relative, FP64 1e-12 relative."""
import numpy as np
import pytest

import ksinputs
import oracle
from helpers import directional_rel_err, oracle_curve, precond_rel_err

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

TOL = {np.float32: 1e-5, np.float64: 1e-12}


def _tdt(dtype):
    return torch.float32 if dtype == np.float32 else torch.float64


def _problem(specs, dtype, waves=None, policy=None, space="odd"):
    import paper_2301_11704_amd as ksc
    descs = [ksc.CurveDesc(s.n_s, s.n_x, s.L, s.map, s.scale, s.s0) for s in specs]
    prob = ksc.Problem(descs, dtype=_tdt(dtype), space=space)
    if waves is not None or policy is not None:
        prob.set_launch(policy or ksc.KSC_LAUNCH_AUTO, waves or 0)
    return prob


def _spec(n_s, n_x, L=39.0, seed=(97, 0), map_="finite", scale=4.0):
    return ksinputs.CurveSpec(n_s, n_x, L, min(6, (n_x - 1) // 3), 1.0, min(6, (n_x - 1) // 3),
                              0.2, True, seed, map_, scale)


def _odd_state(n_s, n_x, seed, dtype):
    """Every sine mode populated, row-to-row noise: b_k = Im of the seeded
    full-spectrum curve, rounded to the run precision."""
    K1 = oracle.n_modes(n_x)
    U = ksinputs.full_spectrum_curve(n_s, K1, seed)
    B = np.ascontiguousarray(U[:, 1:].imag)
    return B.astype(dtype).astype(np.float64)


def _embed(B):
    """[n_s, K] reals -> [n_s, K+1] complex array with i B in modes 1..K
    (to reuse the full-space parity metrics)."""
    U = np.zeros((B.shape[0], B.shape[1] + 1), dtype=np.complex128)
    U[:, 1:] = 1j * B
    return U


def _check_all(prob, X, c, B, dtype, dtau=1e-4):
    J2, Jarc = prob.eval_J(X, arc=True)
    G, J2g = prob.eval_grad(X)
    Y = torch.empty_like(X)
    J2s = prob.step(X, Y, dtau, want_J2=True)
    torch.cuda.synchronize()
    tol = TOL[dtype]
    J2_ref = oracle.J2_odd(c, B)
    assert abs(J2.item() - J2_ref) <= tol * J2_ref
    assert abs(J2g.item() - J2_ref) <= tol * J2_ref
    assert abs(J2s.item() - J2_ref) <= tol * J2_ref
    Ja_ref = oracle.J_arc_odd(c, B)
    assert abs(Jarc.item() - Ja_ref) <= tol * Ja_ref
    Gg = prob.download(G, 0)
    Gr = oracle.grad_odd(c, B)
    assert np.all(Gg[0] == 0) and np.all(Gg[-1] == 0)
    e_pre = precond_rel_err(c, _embed(Gg), _embed(Gr))
    e_dir = directional_rel_err(c, _embed(Gg), _embed(Gr), [(98, i) for i in range(8)])
    assert e_pre <= tol, e_pre
    assert e_dir <= tol, e_dir
    got = prob.download(Y, 0)
    ref = oracle.step_odd(c, B, dtau)
    assert np.array_equal(got[0], B[0]) and np.array_equal(got[-1], B[-1])
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert err <= tol, err


# ---------------------------------------------------------------- boundary --

@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("n_x", [8, 16, 32, 64, 128, 256])
def test_odd_conversions(dtype, n_x):
    print(f"odd conversions n_x={n_x} dtype={dtype.__name__}", flush=True)
    if dtype == np.float64 and n_x == 256:
        pytest.skip("the odd subspace in FP64 supports n_x <= 128")
    spec = _spec(37, n_x)
    prob = _problem([spec], dtype)
    K = oracle.n_modes(n_x) - 1
    rng = np.random.default_rng(n_x)
    # a generic field: phys -> spec keeps Im u_hat_k (its odd part)
    phys = rng.standard_normal((spec.n_s, n_x)).astype(dtype)
    P = torch.from_numpy(phys.ravel()).cuda()
    X = prob.phys_to_spec(P)
    got = prob.download(X, 0)
    ref = oracle.to_spectral(phys.astype(np.float64), K)[:, 1:].imag
    tol = TOL[dtype] * 10
    assert got.shape == (spec.n_s, K)
    assert np.abs(got - ref).max() <= tol * np.abs(ref).max()
    back = prob.spec_to_phys(X).cpu().numpy().reshape(spec.n_s, n_x)
    ref_back = oracle.to_physical(_embed(got), n_x)
    assert np.abs(back - ref_back).max() <= tol * np.abs(ref_back).max()
    # the synthesized field is odd: u_0 = u_{N/2} = 0, u_{N-n} = -u_n
    assert np.all(back[:, 0] == 0) and np.all(back[:, n_x // 2] == 0)
    assert np.array_equal(back[:, 1:], -back[:, :0:-1])


# ------------------------------------------------------- cost / grad / step --

CASES = [
    # (n_s, n_x): several tiles and ragged tails for every tile shape
    (3, 32), (4, 16), (300, 8), (131, 16), (200, 32), (127, 64), (300, 64),
    (131, 128), (520, 128), (70, 256), (300, 256),
]


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("waves", [1, 4])
def test_odd_parity(dtype, case, waves):
    n_s, n_x = case
    print(f"odd parity n_s={n_s} n_x={n_x} waves={waves} dtype={dtype.__name__}", flush=True)
    if dtype == np.float64 and n_x == 256:
        pytest.skip("the odd subspace in FP64 supports n_x <= 128")
    spec = _spec(n_s, n_x, 39.0, (97, n_s, n_x))
    prob = _problem([spec], dtype, waves=waves)
    B = _odd_state(n_s, n_x, (97, n_s, n_x), dtype)
    X = prob.new_state()
    prob.upload(X, 0, B)
    _check_all(prob, X, oracle_curve(spec), B, dtype)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_odd_rational_map_smooth_curve(dtype):
    """A smooth seeded curve on the rational grid (most rows cluster at the
    ends, where g_j is small)."""
    spec = ksinputs.CurveSpec(257, 64, 22.0, 6, 1.0, 6, 0.2, True, (97, 1), "rational", 40.0)
    K1 = oracle.n_modes(spec.n_x)
    _, _, U = ksinputs.make_curve(spec, K1)
    B = np.ascontiguousarray(U[:, 1:].imag).astype(dtype).astype(np.float64)
    prob = _problem([spec], dtype)
    X = prob.new_state()
    prob.upload(X, 0, B)
    _check_all(prob, X, oracle_curve(spec), B, dtype, dtau=1e-3)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("n_x", [32, 128])
def test_odd_space_matches_full_space(dtype, n_x):
    """The odd kernels and the full-space kernels on the embedded state give
    the same cost, gradient and step, to the run precision."""
    spec = _spec(300, n_x, 39.0, (99, n_x))
    B = _odd_state(spec.n_s, n_x, (99, n_x), dtype)
    po = _problem([spec], dtype)
    pf = _problem([spec], dtype, space="full")
    Xo = po.new_state()
    po.upload(Xo, 0, B)
    Xf = pf.new_state()
    pf.upload(Xf, 0, _embed(B))
    Go, Jo = po.eval_grad(Xo)
    Gf, Jf = pf.eval_grad(Xf)
    Yo, Yf = torch.empty_like(Xo), torch.empty_like(Xf)
    po.step(Xo, Yo, 1e-4)
    pf.step(Xf, Yf, 1e-4)
    torch.cuda.synchronize()
    tol = TOL[dtype]
    assert abs(Jo.item() - Jf.item()) <= 2 * tol * Jf.item()
    c = oracle_curve(spec)
    gf = pf.download(Gf, 0)
    assert precond_rel_err(c, _embed(po.download(Go, 0)), 1j * gf.imag) <= 2 * tol
    yo, yf = po.download(Yo, 0), pf.download(Yf, 0)
    assert np.linalg.norm(yo - yf[:, 1:].imag) <= 2 * tol * np.linalg.norm(yf)
    # the full step keeps the subspace: real parts and mode 0 stay at rounding level
    assert np.abs(yf.real).max() <= 10 * tol * np.abs(yf).max()


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_odd_descend_matches_single_steps_and_oracle(dtype):
    spec = _spec(150, 64, 22.0, (100, 1), "rational", 40.0)
    K1 = oracle.n_modes(spec.n_x)
    _, _, U = ksinputs.make_curve(spec, K1)
    B = np.ascontiguousarray(U[:, 1:].imag).astype(dtype).astype(np.float64)
    prob = _problem([spec], dtype)
    X = prob.new_state()
    prob.upload(X, 0, B)
    X2 = X.clone()
    n, every = 24, 8
    tr = prob.descend(X, n, 1e-3, every=every)
    Y = torch.empty_like(X2)
    for _ in range(n):
        prob.step(X2, Y, 1e-3)
        X2, Y = Y, X2
    torch.cuda.synchronize()
    assert torch.equal(X, X2)
    c = oracle_curve(spec)
    Br = B.copy()
    Jr = []
    for _ in range(n):
        Jr.append(oracle.J2_odd(c, Br))
        Br = oracle.step_odd(c, Br, 1e-3)
    got = prob.download(X, 0)
    assert np.linalg.norm(got - Br) / np.linalg.norm(Br) <= 4 * TOL[dtype]
    trc = tr.cpu().numpy()[:, 0]
    for g in range(n // every):
        ref = Jr[(g + 1) * every - 1]
        assert abs(trc[g] - ref) <= 4 * TOL[dtype] * ref


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_odd_batched_uneven_curves(dtype):
    """Curves of different n_x, n_s and L in one problem (one launch per n_x
    group); every launch policy gives the same bits."""
    import paper_2301_11704_amd as ksc
    specs = [_spec(n_s, n_x, L, (101, i)) for i, (n_s, n_x, L) in enumerate(
        [(130, 64, 22.0), (67, 32, 30.0), (300, 128, 39.0), (45, 16, 12.0), (129, 64, 50.0)])]
    tol = TOL[dtype]
    prob = _problem(specs, dtype)
    X = prob.new_state()
    Bs = []
    for i, s in enumerate(specs):
        B = _odd_state(s.n_s, s.n_x, (101, i), dtype)
        prob.upload(X, i, B)
        Bs.append(B)
    outs = []
    for policy in (ksc.KSC_LAUNCH_AUTO, ksc.KSC_LAUNCH_PLAIN, ksc.KSC_LAUNCH_PERSISTENT):
        prob.set_launch(policy, 0)
        G, J2 = prob.eval_grad(X)
        outs.append((G.clone(), J2.clone()))
    torch.cuda.synchronize()
    for G, J2 in outs[1:]:
        assert torch.equal(G, outs[0][0]) and torch.equal(J2, outs[0][1])
    G, J2 = outs[0]
    J2 = J2.cpu().numpy()
    for i, (s, B) in enumerate(zip(specs, Bs)):
        c = oracle_curve(s)
        ref = oracle.J2_odd(c, B)
        assert abs(J2[i] - ref) <= tol * ref
        e = precond_rel_err(c, _embed(prob.download(G, i)), _embed(oracle.grad_odd(c, B)))
        assert e <= tol, (i, e)


def test_odd_autograd_and_endpoints():
    """Autograd over the odd state equals eval_grad; set_endpoints writes rows
    of K reals."""
    import paper_2301_11704_amd as ksc
    spec = _spec(96, 32, 22.0, (102, 0))
    prob = _problem([spec], np.float64)
    B = _odd_state(spec.n_s, spec.n_x, (102, 0), np.float64)
    X = prob.new_state()
    prob.upload(X, 0, B)
    K = oracle.n_modes(spec.n_x) - 1
    a = torch.arange(1, K + 1, dtype=torch.float64, device="cuda") * 0.01
    b = -a
    prob.set_endpoints(X, 0, a, b)
    Bn = prob.download(X, 0)
    assert np.array_equal(Bn[0], a.cpu().numpy()) and np.array_equal(Bn[-1], b.cpu().numpy())
    assert np.array_equal(Bn[1:-1], B[1:-1])
    Xr = X.clone().requires_grad_(True)
    J = ksc.curve_J2(Xr, prob)
    J.sum().backward()
    G, _ = prob.eval_grad(X)
    torch.cuda.synchronize()
    assert torch.equal(Xr.grad, G)
    c = oracle_curve(spec)
    assert abs(J.item() - oracle.J2_odd(c, Bn)) <= 1e-12 * J.item()


def test_odd_flags_and_inactive_curves():
    specs = [_spec(40, 32, 22.0, (103, i)) for i in range(3)]
    prob = _problem(specs, np.float32)
    X = prob.new_state()
    for i, s in enumerate(specs):
        prob.upload(X, i, _odd_state(s.n_s, s.n_x, (103, i), np.float32))
    X0 = X.clone()
    prob.view(X, 1)[5, 2] = float("nan")
    act = torch.tensor([1, 1, 0], dtype=torch.uint8, device="cuda")
    prob.descend(X, 4, 1e-3, every=2, active=act)
    flags = prob.query_flags()
    assert flags[1] & 1
    assert flags[0] == 0 and flags[2] == 0
    torch.cuda.synchronize()
    # the inactive curve is left unchanged
    assert torch.equal(prob.view(X, 2), prob.view(X0, 2))
