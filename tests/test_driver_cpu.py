"""The descent driver's decisions (roll back and halve dtau on a rise, freeze
converged curves, promote to FP64, checkpoint and resume) exercised on the CPU
with a backend built on the FP64 oracle.  No GPU."""
import numpy as np
import pytest

import ksinputs
import oracle
from paper_2301_11704_amd.driver import descend_to


class OracleBackend:
    """Same methods as the GPU backend; the state is a list of complex arrays.
    `noise` adds a deterministic float32-like rounding after every step when the
    dtype is f32 (to create a noise floor); `inject_nan` poisons one curve."""

    def __init__(self, specs, Us, dtype="f32", inject_nan_at=None, dtype_floor=True):
        self.specs = specs
        self.curves = [oracle.Curve(s.n_s, s.n_x, s.L, s.map, s.scale) for s in specs]
        self.U = [np.array(u, dtype=np.complex128) for u in Us]
        self._dtype = dtype
        self.active = np.ones(len(specs), dtype=bool)
        self.calls = 0
        self.inject_nan_at = inject_nan_at
        self.dtype_floor = dtype_floor

    @property
    def dtype(self):
        return self._dtype

    def n_curves(self):
        return len(self.U)

    def _round(self, U):
        if self._dtype == "f32" and self.dtype_floor:
            return U.astype(np.complex64).astype(np.complex128)
        return U

    def run(self, n_steps, dtau, every):
        self.calls += 1
        rows = []
        for i in range(n_steps):
            J = np.zeros(len(self.U))
            for c in range(len(self.U)):
                if not self.active[c]:
                    continue
                J[c] = oracle.J2(self.curves[c], self.U[c])
                self.U[c] = self._round(oracle.step(self.curves[c], self.U[c], dtau))
                if self.inject_nan_at is not None and self.calls == self.inject_nan_at[0] \
                        and c == self.inject_nan_at[1]:
                    self.U[c][3, 2] = np.nan
            if (i + 1) % every == 0:
                rows.append(J)
        return np.array(rows)

    def J2(self):
        return np.array([oracle.J2(c, u) for c, u in zip(self.curves, self.U)])

    def J_arc(self):
        return np.array([oracle.J_arc(c, u) for c, u in zip(self.curves, self.U)])

    def set_active(self, mask):
        self.active = np.array(mask, dtype=bool)

    def snapshot(self):
        return np.concatenate([u.ravel() for u in self.U]).copy()

    def restore(self, arr):
        off = 0
        for i, u in enumerate(self.U):
            n = u.size
            self.U[i] = arr[off:off + n].reshape(u.shape).copy()
            off += n

    def promote(self):
        b = OracleBackend(self.specs, self.U, "f64", dtype_floor=False)
        b.active = self.active.copy()
        return b


def _specs(n=2):
    specs = [ksinputs.CurveSpec(24, 16, 22.0, 3, 1.0, 3, 0.1, False, (70, i)) for i in range(n)]
    Us = [ksinputs.make_curve(s, 6)[2] for s in specs]
    return specs, Us


@pytest.mark.filterwarnings("ignore::RuntimeWarning")  # the chunk overflows on purpose
def test_rollback_and_halving_on_divergence():
    specs, Us = _specs(1)
    b = OracleBackend(specs, Us, "f64")
    # far above the explicit s-part stability bound: the first chunk blows up
    b2, log = descend_to(b, dtau=100.0, J_target=0.0, max_steps=40, every=10, fp64_finish=False)
    assert any("rollback" in e[1] for e in log.events)
    assert log.dtau < 100.0
    Js = [float(j[0]) for _, j in log.J_history]
    assert all(np.isfinite(Js)) and all(a >= b_ for a, b_ in zip(Js, Js[1:]))


def test_nan_in_one_curve_rolls_back_the_batch():
    specs, Us = _specs(2)
    b = OracleBackend(specs, Us, "f64", inject_nan_at=(1, 1))
    _, log = descend_to(b, dtau=1e-3, J_target=0.0, max_steps=20, every=10, fp64_finish=False)
    assert any("rollback" in e[1] for e in log.events)
    assert all(np.all(np.isfinite(j)) for _, j in log.J_history)


def test_converged_curves_are_frozen():
    specs, Us = _specs(2)
    b = OracleBackend(specs, Us, "f64")
    J0 = np.sqrt(b.J2())
    target = float(np.max(J0)) * 1.5   # every curve is already below target
    _, log = descend_to(b, dtau=1e-3, J_target=target, max_steps=50, every=10)
    assert log.converged.all()
    assert log.steps <= 10


def test_fp32_stall_promotes_to_fp64():
    specs, Us = _specs(1)
    b = OracleBackend(specs, Us, "f32")
    b2, log = descend_to(b, dtau=1e-3, J_target=0.0, max_steps=60, every=10,
                         switch_J=1e30, stall_records=1)
    assert b2.dtype == "f64"
    assert any("FP64" in e[1] for e in log.events)


def test_checkpoint_resume_is_bitwise(tmp_path):
    specs, Us = _specs(2)
    ck = str(tmp_path / "ck.npz")
    b = OracleBackend(specs, Us, "f64")
    b_full, log_full = descend_to(b, dtau=1e-3, J_target=0.0, max_steps=40, every=10,
                                  fp64_finish=False)
    b1 = OracleBackend(specs, Us, "f64")
    descend_to(b1, dtau=1e-3, J_target=0.0, max_steps=20, every=10, fp64_finish=False,
               checkpoint=ck)
    b2 = OracleBackend(specs, Us, "f64")
    b2, log2 = descend_to(b2, dtau=1e-3, J_target=0.0, max_steps=40, every=10,
                          fp64_finish=False, checkpoint=ck, resume=True)
    assert log2.steps == 40
    assert np.array_equal(b2.snapshot(), b_full.snapshot())


class _MomentumBackend:
    """A scripted backend: J falls by 10% per chunk, except that the first
    chunk run with the momentum on makes it rise (an overshoot)."""

    dtype = "f64"

    def __init__(self):
        self.J = np.array([1.0])
        self.beta = 0.0
        self.momentum_chunks = 0
        self.betas = []

    def n_curves(self):
        return 1

    def run(self, n_steps, dtau, every):
        self.betas.append(self.beta)
        if self.beta > 0:
            self.momentum_chunks += 1
            self.J = self.J * (3.0 if self.momentum_chunks == 1 else 0.5)
        else:
            self.J = self.J * 0.9
        return np.tile(self.J ** 2, (max(1, n_steps // every), 1))

    def J2(self):
        return self.J ** 2

    def set_active(self, mask):
        pass

    def snapshot(self):
        return self.J.copy()

    def restore(self, arr):
        self.J = arr.copy()

    def set_momentum(self, beta):
        self.beta = beta


def test_rise_with_momentum_redoes_the_chunk_without_it():
    """With the momentum on, a rising chunk is rolled back and redone with
    plain steps at the same dtau; the momentum then resumes (and here
    converges); dtau is never halved."""
    b = _MomentumBackend()
    _, log = descend_to(b, dtau=0.05, J_target=1e-3, max_steps=300, every=10, chunk=10,
                        momentum=0.9)
    msgs = [e[1] for e in log.events]
    assert "J rose with momentum; rollback, plain chunk" in msgs
    assert not any("dtau ->" in m for m in msgs)
    assert log.dtau == 0.05 and log.converged.all()
    # a plain chunk, the overshooting momentum chunk, its plain redo, then
    # momentum to the end
    assert b.betas[:4] == [0.0, 0.9, 0.0, 0.9] and set(b.betas[3:]) == {0.9}


class _LbfgsBackend(_MomentumBackend):
    """Scripted: steps reduce J by 10% per chunk; L-BFGS chunks halve it."""

    def __init__(self):
        super().__init__()
        self.lbfgs_calls = []

    def run_lbfgs(self, n_iter, dtau, every, m):
        self.lbfgs_calls.append((n_iter, dtau, m))
        self.J = self.J * 0.5
        return np.tile(self.J ** 2, (max(1, n_iter // every), 1))


def test_lbfgs_runs_the_late_fp64_phase():
    """With lbfgs = m the driver runs the chunks after the first FP64 chunk as
    L-BFGS chunks (lbfgs_chunk iterations each, counted as steps, tau frozen)
    and never turns the momentum on."""
    b = _LbfgsBackend()
    _, log = descend_to(b, dtau=0.05, J_target=1e-3, max_steps=10_000, every=10, chunk=10,
                        momentum=0.9, lbfgs=5, lbfgs_chunk=7)
    assert b.lbfgs_calls and all(c == (7, 0.05, 5) for c in b.lbfgs_calls)
    assert set(b.betas) == {0.0} and len(b.betas) == 1
    assert log.converged.all()
    assert log.tau == 10 * 0.05 and log.steps == 10 + 7 * len(b.lbfgs_calls)
