"""Seeded synthetic inputs for Kuramoto-Sivashinsky connecting-curve problems.

This module only draws random numbers and lays them out; it holds none of the
method's arithmetic (no residual, cost, adjoint or step).  Both the FP64 CPU
oracle and the GPU library consume what it returns, so the two sides always
see the same numbers.

State layout shared by both sides: one complex array per curve of shape
``[n_s, n_modes]`` holding the Fourier coefficients of every s-row (row 0 is
the endpoint at s = -inf, row n_s-1 the endpoint at s = +inf).  ``n_modes``
is supplied by the caller; mode 0 is real.

Smooth random state (the recipe of every workload):
    u(x) = amp * sum_{k=1..kmax} (a_k cos(2 pi k x / L) + b_k sin(2 pi k x / L)) / k^2
with a_k, b_k ~ N(0, 1), i.e. coefficient u_hat_k = amp * (a_k - i b_k) / (2 k^2)
and u_hat_0 = 0.  Draw order per curve: a(B), b(B), [a(A), b(A)], a(p), b(p),
from ``numpy.random.default_rng(SeedSequence([config, curve]))``.

Initial curve: u_j = (1 - sigma_j) A + sigma_j B + sin(pi sigma_j) p with
sigma_j = j / (n_s - 1); for workload 4 the blend is replaced by samples of
a stored KS trajectory from A to B (config4_curves).
"""
from __future__ import annotations

import os
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "CurveSpec",
    "smooth_coeffs",
    "blend_curve",
    "config_specs",
    "make_curve",
    "round_to",
    "random_direction",
    "config4_curves",
    "interpolate_samples",
]


@dataclass(frozen=True)
class CurveSpec:
    """Shape and seeds of one synthetic curve."""

    n_s: int
    n_x: int
    L: float
    kmax_end: int          # highest mode of the random endpoint(s)
    amp_end: float
    kmax_pert: int         # highest mode of the sin(pi sigma) perturbation
    amp_pert: float
    random_A: bool         # False: A = 0 (the trivial equilibrium)
    seed: tuple = field(default=(0, 0))
    map: str = "rational"  # "rational" (s = s0 + S cot(theta)) or "finite" (s = T sigma)
    scale: float = 40.0    # S for the rational map, T for the finite map
    s0: float = 0.0


def smooth_coeffs(rng: np.random.Generator, kmax: int, amp: float, n_modes: int) -> np.ndarray:
    """Coefficients u_hat_k = amp (a_k - i b_k) / (2 k^2), k = 1..kmax; zero elsewhere."""
    a = rng.standard_normal(kmax)
    b = rng.standard_normal(kmax)
    out = np.zeros(n_modes, dtype=np.complex128)
    k = np.arange(1, kmax + 1)
    kk = min(kmax, n_modes - 1)
    out[1:kk + 1] = (amp * (a - 1j * b) / (2.0 * k.astype(np.float64) ** 2))[:kk]
    return out


def full_spectrum_coeffs(rng: np.random.Generator, amp: float, n_modes: int) -> np.ndarray:
    """Every kept mode populated: u_hat_k = amp (a_k - i b_k) / (1 + k), k = 0..n_modes-1,
    a_k, b_k ~ N(0, 1); mode 0 real."""
    a = rng.standard_normal(n_modes)
    b = rng.standard_normal(n_modes)
    k = np.arange(n_modes, dtype=np.float64)
    out = amp * (a - 1j * b) / (1.0 + k)
    out[0] = out[0].real
    return out


def full_spectrum_curve(n_s: int, n_modes: int, seed, amp: float = 0.3, rough: float = 0.02):
    """A curve whose rows populate every kept mode (unlike the smooth seeded
    states, which fill only k <= kmax): endpoints and the sin(pi sigma)
    perturbation from full_spectrum_coeffs, plus row-to-row independent noise of
    relative size `rough` on the interior rows (content at every s-frequency)."""
    rng = np.random.default_rng(np.random.SeedSequence(list(seed)))
    A = full_spectrum_coeffs(rng, amp, n_modes)
    B = full_spectrum_coeffs(rng, amp, n_modes)
    p = full_spectrum_coeffs(rng, amp, n_modes)
    U = blend_curve(A, B, p, n_s)
    k = np.arange(n_modes, dtype=np.float64)
    noise = (rng.standard_normal((n_s - 2, n_modes)) - 1j * rng.standard_normal((n_s - 2, n_modes)))
    U[1:-1] += rough * amp * noise / (1.0 + k)[None, :]
    U[:, 0] = U[:, 0].real
    return U


def blend_curve(A: np.ndarray, B: np.ndarray, p: np.ndarray, n_s: int) -> np.ndarray:
    """u_j = (1 - sigma_j) A + sigma_j B + sin(pi sigma_j) p, sigma_j = j / (n_s - 1)."""
    sig = np.arange(n_s, dtype=np.float64) / (n_s - 1)
    U = (1.0 - sig)[:, None] * A[None, :] + sig[:, None] * B[None, :] \
        + np.sin(np.pi * sig)[:, None] * p[None, :]
    U[0] = A
    U[-1] = B
    return U


def make_curve(spec: CurveSpec, n_modes: int):
    """Return (A_hat, B_hat, U_hat[n_s, n_modes]) for one seeded curve."""
    rng = np.random.default_rng(np.random.SeedSequence(list(spec.seed)))
    B = smooth_coeffs(rng, spec.kmax_end, spec.amp_end, n_modes)
    if spec.random_A:
        A = smooth_coeffs(rng, spec.kmax_end, spec.amp_end, n_modes)
    else:
        A = np.zeros(n_modes, dtype=np.complex128)
    p = smooth_coeffs(rng, spec.kmax_pert, spec.amp_pert, n_modes)
    return A, B, blend_curve(A, B, p, spec.n_s)


def config_specs(cfg: int, n_curves: int | None = None) -> list[CurveSpec]:
    """The synthetic workloads.

    0: one curve, L=22, N_x=32, N_s=64, A=0, B=smooth(4,1), p=smooth(4,0.1), FP64.
    1: one curve, L=39, N_x=64, N_s=512, modes <= 6, perturbation 0.2, FP32.
    2: one curve, L=100, N_x=256, N_s=8192, random A and B with modes <= 12,
       perturbation 0.3, FP32.
    3: 256 curves of uneven shape, N_x in {32,64,128}, N_s in [128, 2048],
       L in {22,39,66}, each seeded as workload 0.
    4: 64 curves, L=66, N_x=128, N_s=1024, finite map T=20 (the curves are
       stored KS trajectory pieces plus a seeded perturbation, config4_curves;
       this spec gives the shape only).
    """
    if cfg == 0:
        return [CurveSpec(64, 32, 22.0, 4, 1.0, 4, 0.1, False, (0, 0))]
    if cfg == 1:
        return [CurveSpec(512, 64, 39.0, 6, 1.0, 6, 0.2, False, (1, 0))]
    if cfg == 2:
        return [CurveSpec(8192, 256, 100.0, 12, 1.0, 12, 0.3, True, (2, 0))]
    if cfg == 3:
        n = 256 if n_curves is None else n_curves
        srng = np.random.default_rng(np.random.SeedSequence([3, 10**6]))
        nxs = srng.choice([32, 64, 128], size=n)
        nss = srng.integers(128, 2048, size=n, endpoint=True)
        Ls = srng.choice([22.0, 39.0, 66.0], size=n)
        return [CurveSpec(int(nss[c]), int(nxs[c]), float(Ls[c]), 4, 1.0, 4, 0.1, False, (3, c))
                for c in range(n)]
    if cfg == 4:
        n = 64 if n_curves is None else n_curves
        return [CurveSpec(1024, 128, 66.0, 6, 1.0, 4, 0.1, True, (4, c), "finite", 20.0)
                for c in range(n)]
    raise ValueError(f"unknown workload {cfg}")


def paper_shape_specs(n_curves: int = 64) -> list[CurveSpec]:
    """Curves with the discretization of the paper's first KS run (L = 22,
    N = 64 Fourier modes in x, M = 550 interior rational Chebyshev points,
    S = 55, s0 = 0): N_x = 64, N_s = 552, rational map.  The endpoints are
    seeded smooth states standing in for the equilibria (which the paper shows
    only as figures); interior = blend + sin(pi sigma) perturbation."""
    return [CurveSpec(552, 64, 22.0, 6, 1.0, 6, 0.2, True, (5, c), "rational", 55.0)
            for c in range(n_curves)]


L22_EQUILIBRIA = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                              "tests", "golden", "L22_equilibria.npz")


def l22_equilibrium(name: str) -> np.ndarray:
    """Stored equilibrium of KS at L = 22, N_x = 64 (coefficients u_hat_k,
    k = 0..21): "E0" (u = 0), "E1", "E2", "E3"; a suffix "+L/2" or "+L/4"
    shifts it by that fraction of the period (u_hat_k e^{i q_k L/2}, ...)."""
    base, _, shift = name.partition("+")
    d = np.load(L22_EQUILIBRIA)
    U = np.zeros(22, dtype=np.complex128) if base == "E0" else np.array(d[base])
    if shift:
        frac = {"L/2": 0.5, "L/4": 0.25, "L/3": 1.0 / 3.0, "L/6": 1.0 / 6.0}[shift]
        V = U * np.exp(2j * np.pi * np.arange(U.size) * frac)
        if np.all(U.real == 0):
            # these shifts map each equilibrium to another copy that is
            # inversion symmetric about x = 0: drop the rounding residue
            assert np.abs(V.real).max() < 1e-12 * max(np.abs(V).max(), 1.0)
            V = 1j * V.imag
        U = V
    return U


def rational_s(n_s: int, S: float, s0: float = 0.0) -> np.ndarray:
    """s_j = s0 + S cot(pi (1 - j / (n_s - 1))) on the rows (row 0: -inf)."""
    th = np.pi * (1.0 - np.arange(n_s) / (n_s - 1))
    with np.errstate(divide="ignore"):
        s = s0 + S * np.cos(th) / np.sin(th)
    s[0], s[-1] = -np.inf, np.inf
    return s


def l22_connection_curve(src: str, dst: str, n_s: int = 552, S: float = 55.0, s0: float = 0.0):
    """The initial connecting curve of eq. KSE_initial_curve with a = 0 from
    u_- = src to u_+ = dst on the rational grid:
    u_0(s) = ((1 + tanh s) u_+ + (1 - tanh s) u_-) / 2 (end rows exactly u_-, u_+).
    Returns (CurveSpec, U_hat [n_s, 22])."""
    um, up = l22_equilibrium(src), l22_equilibrium(dst)
    th = np.tanh(rational_s(n_s, S, s0))
    U = 0.5 * ((1.0 + th)[:, None] * up[None, :] + (1.0 - th)[:, None] * um[None, :])
    U[0], U[-1] = um, up
    spec = CurveSpec(n_s, 64, 22.0, 0, 0.0, 0, 0.0, False, (22, 0), "rational", S, s0)
    return spec, U


# Connections of the paper's Table II (tab:parameters): row, from, to, M, S
# (N = 64, s0 = 0, dtau = 0.01 for all).  Row 6 ends at E2 shifted by L/4.
TABLE2 = [
    (1, "E0", "E1", 80, 40.0), (2, "E0", "E2", 130, 35.0), (3, "E0", "E3", 120, 40.0),
    (4, "E1", "E2", 550, 55.0), (5, "E1", "E3", 500, 60.0), (6, "E2", "E2+L/4", 400, 35.0),
    (7, "E2", "E3", 450, 50.0), (8, "E3", "E2", 600, 50.0), (9, "E3", "E2", 500, 40.0),
]
# Each equilibrium's other inversion-symmetric copy (about x = 0): E1 shifted
# by L/2, E2 by L/4, E3 by L/6; and its translation period in units of L.
OTHER_PHASE = {"E1": "E1+L/2", "E2": "E2+L/4", "E2+L/4": "E2", "E3": "E3+L/6", "E0": None}
_SHIFT = {"E1": 0.0, "E1+L/2": 0.5, "E2": 0.0, "E2+L/4": 0.25, "E3": 0.0, "E3+L/6": 1.0 / 6.0}
_PERIOD = {"E1": 1.0, "E2": 0.5, "E3": 1.0 / 3.0}


def _phase_class(a: str, b: str) -> float:
    """The relative shift of destination against source, modulo the shifts
    that map either equilibrium to itself (a connection and its common
    translation are the same run)."""
    pa, pb = _PERIOD[a.split("+")[0]], _PERIOD[b.split("+")[0]]
    # the smallest positive combination of the two periods (both are 1/n)
    g = 1.0 / np.lcm(int(round(1 / pa)), int(round(1 / pb)))
    return round((_SHIFT[b] - _SHIFT[a]) % g, 9) % g


def table2_connections(both_phases: bool = True):
    """Initial curves (eq. KSE_initial_curve, a = 0) for the rows of Table II:
    a list of (label, CurveSpec, U_hat).  With both_phases, a row whose two
    equilibria have another relative phase that keeps the curve
    inversion-symmetric (the table does not print it) appears once more with
    it: the destination's other copy, or the source's when that copy is
    equivalent (E2 -> E3 and E2 -> E3 + L/6 differ by a symmetry of E3 and a
    common shift).  Rows from E0 have no distinct phases; row 6 with a = 0 is
    the run the paper reports stuck at a local minimum."""
    out = []
    for row, a, b, M, S in TABLE2:
        pairs = [(a, b)]
        if both_phases and a != "E0" and row != 6:
            seen = {_phase_class(a, b)}
            for cand in ((a, OTHER_PHASE[b]), (OTHER_PHASE[a], b)):
                c = _phase_class(*cand)
                if c not in seen:
                    seen.add(c)
                    pairs.append(cand)
                    break
        for src, dst in pairs:
            spec, U = l22_connection_curve(src, dst, M + 2, S)
            out.append((f"row{row}:{src}->{dst}", spec, U))
    return out


def round_to(U: np.ndarray, dtype) -> np.ndarray:
    """Round complex128 data to the run precision (complex64 for FP32) and back."""
    if np.dtype(dtype) == np.float32:
        return U.astype(np.complex64).astype(np.complex128)
    return U.astype(np.complex128)


def random_direction(seed, n_s: int, n_modes: int, kmax: int = 8) -> np.ndarray:
    """Smooth seeded direction: sin(pi sigma) in s times random modes k <= kmax."""
    rng = np.random.default_rng(np.random.SeedSequence(list(seed)))
    sig = np.arange(n_s, dtype=np.float64) / (n_s - 1)
    v = np.zeros((n_s, n_modes), dtype=np.complex128)
    kk = min(kmax, n_modes - 1)
    coef = rng.standard_normal(kk + 1) + 1j * rng.standard_normal(kk + 1)
    coef[0] = coef[0].real
    amp = np.sin(np.pi * sig)
    # a second, faster s-profile so the direction is not rank one
    amp2 = np.sin(2 * np.pi * sig)
    coef2 = rng.standard_normal(kk + 1) + 1j * rng.standard_normal(kk + 1)
    coef2[0] = coef2[0].real
    v[:, :kk + 1] = amp[:, None] * coef[None, :] + 0.5 * amp2[:, None] * coef2[None, :]
    v[0] = 0
    v[-1] = 0
    return v


C4_TRAJECTORIES = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                               "tests", "golden", "c4_trajectories.npz")


def interpolate_samples(samples: np.ndarray, t_new: np.ndarray, order: int = 6) -> np.ndarray:
    """Values at t_new in [0, 1] of uniformly spaced samples (axis 0 at t =
    m / (M - 1)) by local Lagrange interpolation through the `order` nearest
    samples (degree order - 1; windows are clamped at the ends).  Exact at the
    sample points."""
    M = samples.shape[0]
    x = np.asarray(t_new, dtype=np.float64) * (M - 1)
    start = np.clip(np.floor(x).astype(int) - (order // 2 - 1), 0, M - order)
    out = np.zeros((len(x),) + samples.shape[1:], dtype=np.result_type(samples, np.complex128))
    for a in range(order):
        w = np.ones(len(x))
        for b in range(order):
            if b != a:
                w *= (x - (start + b)) / (a - b)
        out += w.reshape((-1,) + (1,) * (samples.ndim - 1)) * samples[start + a]
    return out


def config4_curves(n_curves: int = 64, n_s: int = 1024, replicas: int = 1):
    """Workload 4 (finite map s = T sigma, T = 20): curve i starts as the
    stored KS trajectory piece from A_i to B_i = Phi_T(A_i), sampled at
    s_j = T sigma_j (interpolated to the n_s rows from its 129 stored
    samples), plus the perturbation sin(pi sigma) smooth(4, 0.1) seeded
    (4, i, 1); the end rows are A_i and B_i exactly.  replicas > 1 repeats
    the batch (used to stream more than the caches hold).
    Returns (specs, list of U_hat [n_s, 43])."""
    d = np.load(C4_TRAJECTORIES)
    traj = d["traj"]
    specs, Us = [], []
    base = config_specs(4, n_curves)
    sig = np.arange(n_s, dtype=np.float64) / (n_s - 1)
    for r in range(replicas):
        for i in range(n_curves):
            sp = base[i]
            if n_s != sp.n_s:
                sp = CurveSpec(n_s, sp.n_x, sp.L, sp.kmax_end, sp.amp_end, sp.kmax_pert,
                               sp.amp_pert, sp.random_A, sp.seed, sp.map, sp.scale, sp.s0)
            tr = traj[i % traj.shape[0]].astype(np.complex128)
            rng = np.random.default_rng(np.random.SeedSequence([4, i, 1]))
            p = smooth_coeffs(rng, 4, 0.1, tr.shape[1])
            U = interpolate_samples(tr, sig) + np.sin(np.pi * sig)[:, None] * p[None, :]
            U[0], U[-1] = tr[0], tr[-1]
            U[:, 0] = U[:, 0].real
            specs.append(sp)
            Us.append(U)
    return specs, Us
