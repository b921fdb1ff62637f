"""GPU parity of the implicit-in-s descent step (KSC_SCHEME_IMPLICIT_S: the
whole linear part of the adjoint flow implicit, banded solves along s) against
the FP64 oracle's ``step_implicit_s`` on the same seeded inputs.

Tolerances: FP32 1e-5 and FP64 1e-12 relative to the state (as for the
paper's step); the increment u_next - u itself is also checked element by
element, to 1e-5 (FP32) and 1e-10 (FP64) of its largest entry, beyond the
half ulp by which a stored FP32 state necessarily misses the exact one (with
a small step the increment is a few ulps of the state, so its FP32 rounding
alone would otherwise be a large fraction of it).  Where the solve shrinks
its input dtau L^dagger r (the stiff components, far past the explicit bound)
the increment is measured against that input instead: the FP32 rounding of
the fused evaluation's L^dagger passes through the solve unshrunk in its
smooth components."""
import numpy as np
import pytest

import ksinputs
import oracle
from helpers import oracle_curve, seeded_state

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

TOL = {np.float32: 1e-5, np.float64: 1e-12}
TOL_INC = {np.float32: 1e-5, np.float64: 1e-10}


def _tdt(dtype):
    return torch.float32 if dtype == np.float32 else torch.float64


def _problem(specs, dtype, space="full"):
    import paper_2301_11704_amd as ksc
    descs = [ksc.CurveDesc(s.n_s, s.n_x, s.L, s.map, s.scale, s.s0) for s in specs]
    prob = ksc.Problem(descs, dtype=_tdt(dtype), space=space)
    prob.set_scheme("implicit_s")
    assert prob.scheme == "implicit_s"
    return prob


def _spec(n_s, n_x, L=22.0, seed=(120, 0), map_="rational", scale=40.0):
    return ksinputs.CurveSpec(n_s, n_x, L, min(6, (n_x - 1) // 3), 1.0, min(6, (n_x - 1) // 3),
                              0.2, True, seed, map_, scale)


def _storage_excess(got, ref, dtype):
    """|got - ref| beyond the rounding of the exact value to the state dtype
    (half an ulp of the larger of |got| and |ref|), for the real and the
    imaginary parts."""
    out = []
    for g, r in ((np.real(got), np.real(ref)), (np.imag(got), np.imag(ref))):
        g, r = np.asarray(g, np.float64), np.asarray(r, np.float64)
        mag = np.maximum(np.abs(g), np.abs(r)).astype(dtype)
        half_ulp = 0.5 * np.spacing(mag).astype(np.float64)
        out.append(np.maximum(np.abs(g - r) - half_ulp, 0.0))
    return np.maximum(out[0], out[1])


def _check(got, ref, U, dtype, solve_in=0.0):
    """State-relative error, and the increment's error beyond storage
    rounding relative to the larger of the increment and the solve's input
    (max |dtau L^dagger r|, when given)."""
    assert np.array_equal(got[0], U[0]) and np.array_equal(got[-1], U[-1])
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    inc = _storage_excess(got, ref, dtype).max() / max(np.abs(ref - U).max(), solve_in)
    assert err <= TOL[dtype], err
    assert inc <= TOL_INC[dtype], inc
    return err, inc


CASES = [  # n_s, n_x, map, scale, dtau: chains of 1 row, ragged chunk counts, up to 512 chunks of rows
    (3, 16, "rational", 40.0, 0.1),
    (4, 16, "finite", 3.0, 0.1),
    (5, 32, "rational", 20.0, 0.05),
    (17, 8, "rational", 40.0, 1.0),
    (40, 32, "finite", 5.0, 0.02),
    (130, 64, "rational", 30.0, 0.3),
    (300, 128, "finite", 20.0, 0.01),
    (1100, 32, "finite", 20.0, 0.05),
    (300, 256, "rational", 40.0, 1e-3),
    (257, 32, "finite", 5.0, 1.0),  # 700x the explicit bound of the s-part (dtau beta^2 = 655)
]


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("n_s,n_x,map_,scale,dtau", CASES)
def test_step_parity(dtype, n_s, n_x, map_, scale, dtau):
    print(f"implicit-s step n_s={n_s} n_x={n_x} {map_} dtau={dtau} dtype={dtype.__name__}",
          flush=True)
    spec = _spec(n_s, n_x, 22.0 if n_x < 256 else 60.0, (121, n_s, n_x), map_, scale)
    prob = _problem([spec], dtype)
    X = prob.new_state()
    U = seeded_state(spec, dtype)
    prob.upload(X, 0, U)
    c = oracle_curve(spec)
    Y = torch.empty_like(X)
    J2 = prob.step(X, Y, dtau, want_J2=True)
    torch.cuda.synchronize()
    got = prob.download(Y, 0)
    ref = oracle.step_implicit_s(c, U, dtau)
    assert abs(J2.item() - oracle.J2(c, U)) <= TOL[dtype] * oracle.J2(c, U)
    solve_in = dtau * np.abs(oracle.adjoint(c, U)[1:-1]).max()
    err, inc = _check(got, ref, U, dtype, solve_in)
    print(f"  state-relative {err:.2e} increment-relative {inc:.2e} "
          f"(solve input / increment {solve_in / np.abs(ref - U).max():.1f})", flush=True)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_step_parity_odd_subspace(dtype):
    spec = _spec(77, 64, 39.0, (122, 0), "finite", 4.0)
    c = oracle_curve(spec)
    U = ksinputs.full_spectrum_curve(spec.n_s, c.K + 1, (123, 0))
    B = np.ascontiguousarray(U[:, 1:].imag).astype(dtype).astype(np.float64)
    prob = _problem([spec], dtype, space="odd")
    X = prob.new_state()
    prob.upload(X, 0, B)
    Y = torch.empty_like(X)
    prob.step(X, Y, 0.05)
    torch.cuda.synchronize()
    got = prob.download(Y, 0)
    ref = oracle.step_implicit_s_odd(c, B, 0.05)
    _check(got, ref, B, dtype)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_batched_uneven_curves_and_active_mask(dtype):
    """Curves of different n_s, n_x, L and map in one problem; an inactive
    curve is copied unchanged."""
    specs = [_spec(3 + 37 * i, (16, 32, 64, 128)[i % 4], 22.0 + 3 * i, (124, i),
                   "rational" if i % 2 else "finite", 5.0 + 10 * i) for i in range(7)]
    prob = _problem(specs, dtype)
    X = prob.new_state()
    Us = []
    for i, s in enumerate(specs):
        U = seeded_state(s, dtype)
        prob.upload(X, i, U)
        Us.append(U)
    active = torch.ones(len(specs), dtype=torch.uint8, device=X.device)
    active[3] = 0
    prob.descend(X, 1, 0.02, every=1, active=active)
    torch.cuda.synchronize()
    for i, s in enumerate(specs):
        got = prob.download(X, i)
        if i == 3:
            assert np.array_equal(got, Us[i])
            continue
        ref = oracle.step_implicit_s(oracle_curve(s), Us[i], 0.02)
        _check(got, ref, Us[i], dtype)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_descend_matches_single_steps_and_oracle(dtype):
    spec = ksinputs.config_specs(0)[0]
    prob = _problem([spec], dtype)
    X = prob.new_state()
    U = seeded_state(spec, dtype)
    prob.upload(X, 0, U)
    c = oracle_curve(spec)
    n, every, dtau = 24, 8, 0.02
    X2 = X.clone()
    tr = prob.descend(X, n, dtau, every=every)
    Y = torch.empty_like(X2)
    for _ in range(n):
        prob.step(X2, Y, dtau)
        X2, Y = Y, X2
    torch.cuda.synchronize()
    assert torch.equal(X, X2)
    Ur = U.copy()
    Jr = []
    for _ in range(n):
        Jr.append(oracle.J2(c, Ur))
        Ur = oracle.step_implicit_s(c, Ur, dtau)
    got = prob.download(X, 0)
    assert np.linalg.norm(got - Ur) / np.linalg.norm(Ur) <= 4 * TOL[dtype]
    trc = tr.cpu().numpy()[:, 0]
    for g in range(n // every):
        ref = Jr[(g + 1) * every - 1]
        assert abs(trc[g] - ref) <= 4 * TOL[dtype] * ref
    # J2 decreases along the descent
    assert all(b < a for a, b in zip(Jr, Jr[1:]))


def test_largest_curve_satisfies_the_banded_system():
    """n_s = 8194 (each chain 4096 rows: 256 chunks of 16, the solver's
    limit): the increment solves (I + dtau B_k) delta = -dtau L^dagger_k,
    checked row by row with the oracle's d/ds and adjoint; n_s = 8195 is
    refused."""
    import paper_2301_11704_amd as ksc
    spec = _spec(8194, 8, 22.0, (125, 0), "finite", 400.0)
    prob = _problem([spec], np.float64)
    X = prob.new_state()
    U = seeded_state(spec, np.float64)
    prob.upload(X, 0, U)
    Y = torch.empty_like(X)
    dtau = 0.5
    prob.step(X, Y, dtau)
    torch.cuda.synchronize()
    c = oracle_curve(spec)
    delta = prob.download(Y, 0) - U
    Ad = oracle.adjoint(c, U)
    from oracle.ks import _ds
    inner = _ds(c, delta)                 # d/ds on interior rows, zero on the end rows
    DmD = _ds(c, inner)
    lhs = delta + dtau * (c.A[None, :] ** 2 * delta - DmD)
    res = np.abs(lhs[1:-1] + dtau * Ad[1:-1]).max() / np.abs(dtau * Ad[1:-1]).max()
    assert res < 1e-12, res
    big = _spec(8195, 8, 22.0, (125, 0), "finite", 400.0)
    p2 = ksc.Problem([ksc.CurveDesc(big.n_s, big.n_x, big.L, big.map, big.scale, big.s0)],
                     dtype=torch.float64)
    with pytest.raises(ksc.KscError):
        p2.set_scheme("implicit_s")


def test_spectral_ds_is_refused_and_scheme_switches_back():
    import paper_2301_11704_amd as ksc
    spec = _spec(40, 32)
    p = ksc.Problem([ksc.CurveDesc(spec.n_s, spec.n_x, spec.L, spec.map, spec.scale, spec.s0)],
                    dtype=torch.float64, ds="spectral")
    with pytest.raises(ksc.KscError):
        p.set_scheme("implicit_s")
    assert p.scheme == "paper"
    prob = _problem([spec], np.float64)
    X = prob.new_state()
    U = seeded_state(spec, np.float64)
    prob.upload(X, 0, U)
    prob.set_scheme("paper")
    Y = torch.empty_like(X)
    prob.step(X, Y, 1e-3)
    torch.cuda.synchronize()
    ref = oracle.step(oracle_curve(spec), U, 1e-3)
    got = prob.download(Y, 0)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= TOL[np.float64]


def test_large_step_descends_on_the_64_curve_batch_shape():
    """Curves of the 64-curve batch (finite map, T = 20, N_s = 1024, N_x = 128)
    at dtau 20 times the paper's step bound for them: J2 decreases at every
    step for every curve."""
    specs, Us = ksinputs.config4_curves(4, 1024)
    prob = _problem(specs, np.float32)
    X = prob.new_state()
    for i, U in enumerate(Us):
        prob.upload(X, i, U)
    tr = prob.descend(X, 200, 0.01, every=1).cpu().numpy()
    assert np.all(np.isfinite(tr))
    assert np.all(np.diff(tr, axis=0) < 0), tr[:5]


def test_driver_promotion_keeps_the_scheme():
    """The descent driver's FP32 -> FP64 promotion continues with the same
    scheme (and the FP64 step of the promoted problem matches the oracle)."""
    from paper_2301_11704_amd.driver import GpuBackend
    spec = ksinputs.config_specs(0)[0]
    prob = _problem([spec], np.float32)
    X = prob.new_state()
    U = seeded_state(spec, np.float32)
    prob.upload(X, 0, U)
    b64 = GpuBackend(prob, X).promote()
    assert b64.prob.scheme == "implicit_s"
    Y = torch.empty_like(b64.state)
    b64.prob.step(b64.state, Y, 0.02)
    torch.cuda.synchronize()
    ref = oracle.step_implicit_s(oracle_curve(spec), U, 0.02)
    _check(b64.prob.download(Y, 0), ref, U, np.float64)


def test_64_curve_batch_sampled_against_the_oracle():
    """The benchmark's 64-curve batch (N_x = 128, N_s = 1024, FP32) with the
    tuned launch: one implicit-in-s step at dtau = 0.05 for every curve, two
    sampled curves checked against the oracle's dense solves."""
    import os
    import paper_2301_11704_amd as ksc
    specs, Us = ksinputs.config4_curves(64, 1024)
    prob = _problem(specs, np.float32)
    prob.tune(os.path.join(os.path.dirname(ksc.__file__), "tuning_gfx950.json"))
    X = prob.new_state()
    Ur = []
    for i, U in enumerate(Us):
        U = ksinputs.round_to(U, np.float32)
        U[:, 0] = U[:, 0].real
        prob.upload(X, i, U)
        Ur.append(U)
    Y = torch.empty_like(X)
    prob.step(X, Y, 0.05)
    torch.cuda.synchronize()
    for i in (0, 63):
        got = prob.download(Y, i)
        ref = oracle.step_implicit_s(oracle_curve(specs[i]), Ur[i], 0.05)
        err, inc = _check(got, ref, Ur[i], np.float32)
        print(f"batch curve {i}: state-relative {err:.2e} increment-relative {inc:.2e}", flush=True)


def test_driver_cli_runs_the_implicit_scheme(tmp_path, capsys):
    """The descent driver's command line with --scheme implicit_s: a short run
    of four batch curves at dtau = 0.05 lowers every curve's J."""
    import json
    from paper_2301_11704_amd import driver
    hist = tmp_path / "h.json"
    driver.main(["--scheme", "implicit_s", "--dtau", "0.05", "--curves", "4", "--max-steps", "400",
                 "--chunk", "200", "--every", "100", "--history", str(hist)])
    out = capsys.readouterr().out
    assert "implicit_s step" in out
    h = json.loads(hist.read_text())
    assert h["scheme"] == "implicit_s"
    J0, J1 = np.array(h["records"][0]["J"]), np.array(h["records"][-1]["J"])
    assert np.all(J1 < J0), (J0, J1)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_momentum_descent_matches_oracle(dtype):
    """ksc_descend with heavy-ball momentum (and its restart on a cost rise)
    against the oracle's iteration, on three uneven curves: 40 steps in graphs
    of 10; the FP32 run against the oracle run that rounds its state to FP32
    after every step."""
    import paper_2301_11704_amd as ksc
    specs = [ksinputs.CurveSpec(n, nx, 22.0, 4, 1.0, 4, 0.1, False, (97, i))
             for i, (n, nx) in enumerate([(64, 32), (91, 64), (40, 32)])]
    tdt = torch.float64 if dtype == np.float64 else torch.float32
    prob = ksc.Problem([ksc.CurveDesc(s.n_s, s.n_x, s.L) for s in specs], dtype=tdt)
    prob.set_scheme("implicit_s")
    prob.set_momentum(0.9)
    X = prob.new_state()
    Us = []
    for c, s in enumerate(specs):
        U = seeded_state(s, dtype)
        prob.upload(X, c, U)
        Us.append(U)
    prob.descend(X, 40, 0.01, every=10)
    tol = 1e-12 if dtype == np.float64 else 1e-5
    for c, (s, U) in enumerate(zip(specs, Us)):
        cur = oracle.Curve(s.n_s, s.n_x, s.L, s.map, s.scale)
        ref = oracle.descend_implicit_s_momentum(cur, U, 40, 0.01, 0.9,
                                                 storage=None if dtype == np.float64 else np.float32)
        got = prob.download(X, c)
        err = np.abs(got - ref).max() / np.abs(ref).max()
        print(f"curve {c}: momentum descent error {err:.2e}", flush=True)
        assert err <= tol
    with pytest.raises(ksc.KscError):
        prob.descend(X, 10, 0.01, every=5)  # momentum needs an even `every`
    prob.set_scheme("paper")
    with pytest.raises(ksc.KscError):
        prob.descend(X, 10, 0.001, every=10)  # and the implicit-in-s scheme


def test_workload4_reduced_descent_reaches_1e8_through_fp64():
    """Two curves of workload 4 (KS trajectory pieces plus the smooth
    perturbation) on 256 rows descend to J < 1e-8: implicit-in-s steps in
    FP32, the switch to FP64 at J = 2e-3 (near the FP32 rounding floor of the
    cost), then heavy-ball momentum; the final J agrees with the oracle's J of
    the downloaded state."""
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
    b, log = descend_to(GpuBackend(prob, X), dtau=0.05, J_target=1e-8, max_steps=1_200_000,
                        every=1000, chunk=20000, switch_J=2e-3, stall_records=5, momentum=0.9995)
    print("events:", log.events, "steps:", log.steps, flush=True)
    assert b.dtype == "f64" and log.converged.all()
    J = np.sqrt(b.J2())
    for c, s in enumerate(specs):
        U = b.prob.download(b.state, c)
        ref = np.sqrt(oracle.J2(oracle_curve(s), U))
        assert J[c] < 1e-8 and abs(J[c] - ref) <= 1e-5 * ref, (J[c], ref)


def test_set_scheme_again_keeps_the_descent_graph_valid():
    """Selecting the implicit-in-s scheme a second time keeps the solve table
    (and the captured descent graph that points at it) valid: 20 graph steps,
    set_scheme again, 20 more graph steps equal 40 eager steps."""
    spec = _spec(70, 32, 22.0, (126, 0), "finite", 5.0)
    prob = _problem([spec], np.float64)
    X = prob.new_state()
    prob.upload(X, 0, seeded_state(spec, np.float64))
    Y = X.clone()
    prob.descend(X, 20, 0.05, every=10, trace=False)
    prob.set_scheme("implicit_s")
    prob.descend(X, 20, 0.05, every=10, trace=False)
    Z = torch.empty_like(Y)
    for _ in range(20):
        prob.step(Y, Z, 0.05)
        prob.step(Z, Y, 0.05)
    torch.cuda.synchronize()
    assert torch.equal(X, Y)
