"""Python view of a batch of KS connecting curves on the GPU.

Thin wrapper over the C ABI (include/ksc.h): every computation runs in the HIP
library; this module only marshals tensor pointers, shapes and the current
torch stream.  PyTorch supplies device memory and streams.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib
from ._lib import check, lib


@dataclass(frozen=True)
class CurveDesc:
    """One curve: n_s rows (including both endpoints), n_x grid points in x,
    domain length L, s-map ("rational": s = s0 + scale cot(theta); "finite":
    s = scale * sigma)."""

    n_s: int
    n_x: int
    L: float
    map: str = "rational"
    scale: float = 40.0
    s0: float = 0.0

    def to_c(self) -> _lib.CurveDescC:
        m = {"rational": _lib.KSC_MAP_RATIONAL, "finite": _lib.KSC_MAP_FINITE}[self.map]
        return _lib.CurveDescC(int(self.n_s), int(self.n_x), float(self.L), m, float(self.scale),
                               float(self.s0))


def n_modes(n_x: int) -> int:
    k = lib().ksc_n_modes(int(n_x))
    if k < 0:
        raise ValueError(f"unsupported n_x={n_x}")
    return k


def _ptr(t: torch.Tensor | None) -> int | None:
    if t is None:
        return None
    return t.data_ptr()


class Problem:
    """A batch of curves sharing one dtype (torch.float32 or torch.float64).

    space="full": states are flat device tensors of ``numel`` scalars
    (curve-major, row-major, interleaved re/im); ``view(state, c)`` gives curve
    c as [n_s, K+1, 2].
    space="odd" (inversion-symmetric subspace, u_hat_k = i b_k): rows of the K
    reals b_1..b_K; ``view(state, c)`` gives [n_s, K].
    ds="spectral": d/ds is the paper's rational Chebyshev D_t (rational map).
    """

    def __init__(self, curves, dtype=torch.float32, device="cuda", space="full", ds="stencil"):
        self.curves = [c if isinstance(c, CurveDesc) else CurveDesc(**c) for c in curves]
        if dtype not in (torch.float32, torch.float64):
            raise ValueError("dtype must be torch.float32 or torch.float64")
        spaces = {"full": _lib.KSC_SPACE_FULL, "odd": _lib.KSC_SPACE_ODD}
        if space not in spaces:
            raise ValueError("space must be 'full' or 'odd'")
        dss = {"stencil": _lib.KSC_DS_STENCIL, "spectral": _lib.KSC_DS_SPECTRAL}
        if ds not in dss:
            raise ValueError("ds must be 'stencil' or 'spectral'")
        self.space = space
        self.ds = ds
        self.dtype = dtype
        self.device = torch.device(device)
        self._dev_index = self.device.index if self.device.index is not None \
            else torch.cuda.current_device()
        arr = (_lib.CurveDescC * len(self.curves))(*[c.to_c() for c in self.curves])
        h = ctypes.c_void_p()
        dt = _lib.KSC_F64 if dtype == torch.float64 else _lib.KSC_F32
        opts = _lib.OptionsC(dt, spaces[space], dss[ds], 0)
        with torch.cuda.device(self.device):
            s0 = self._stream()
            check(lib().ksc_create_opts(arr, len(self.curves), ctypes.byref(opts), s0,
                                        ctypes.byref(h)))
        self._h = h
        self._bound_stream = s0  # the stream the library launches on
        L = lib()
        self.numel = int(L.ksc_state_numel(h))
        self.phys_numel = int(L.ksc_phys_numel(h))
        self.offsets = [int(L.ksc_state_offset(h, c)) for c in range(len(self.curves))]
        self.phys_offsets = [int(L.ksc_phys_offset(h, c)) for c in range(len(self.curves))]
        self.modes = [n_modes(c.n_x) for c in self.curves]

    # -- plumbing ----------------------------------------------------------
    def _stream(self) -> int:
        return torch._C._cuda_getCurrentRawStream(self._dev_index)

    def _sync_stream(self):
        # rebind only when torch's current stream changed since the last call
        s = self._stream()
        if s != self._bound_stream:
            check(lib().ksc_set_stream(self._h, s))
            self._bound_stream = s

    def close(self):
        if getattr(self, "_h", None):
            lib().ksc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def n_curves(self) -> int:
        return len(self.curves)

    def _check_state(self, t: torch.Tensor, name="state"):
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError(f"{name} must be a CUDA (HIP) tensor")
        if t.dtype != self.dtype or t.numel() != self.numel or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous {self.dtype} tensor of {self.numel} scalars")

    def _f64(self, n: int) -> torch.Tensor:
        return torch.empty(n, dtype=torch.float64, device=self.device)

    # -- state helpers -----------------------------------------------------
    def new_state(self) -> torch.Tensor:
        return torch.zeros(self.numel, dtype=self.dtype, device=self.device)

    def view(self, state: torch.Tensor, c: int) -> torch.Tensor:
        cd = self.curves[c]
        if self.space == "odd":
            n = cd.n_s * (self.modes[c] - 1)
            return state[self.offsets[c]:self.offsets[c] + n].view(cd.n_s, self.modes[c] - 1)
        n = cd.n_s * self.modes[c] * 2
        return state[self.offsets[c]:self.offsets[c] + n].view(cd.n_s, self.modes[c], 2)

    def upload(self, state: torch.Tensor, c: int, U: np.ndarray) -> None:
        """Copy host coefficients of curve c into the state: complex [n_s, K+1]
        (full space) or real b [n_s, K] (odd subspace)."""
        U = np.asarray(U)
        if self.space == "odd":
            if np.iscomplexobj(U):
                raise ValueError("the odd subspace takes the real coefficients b [n_s, K]")
            v = U
        else:
            v = np.stack([U.real, U.imag], axis=-1)
        self.view(state, c).copy_(torch.from_numpy(np.ascontiguousarray(v)).to(self.dtype))

    def download(self, state: torch.Tensor, c: int) -> np.ndarray:
        v = self.view(state, c).detach().double().cpu().numpy()
        if self.space == "odd":
            return v
        return v[..., 0] + 1j * v[..., 1]

    # -- the C ABI calls ----------------------------------------------------
    def set_endpoints(self, state, c: int, a_hat: torch.Tensor, b_hat: torch.Tensor):
        self._check_state(state)
        self._sync_stream()
        check(lib().ksc_set_endpoints(self._h, _ptr(state), int(c), _ptr(a_hat), _ptr(b_hat)))

    def phys_to_spec(self, phys: torch.Tensor, state: torch.Tensor | None = None):
        state = self.new_state() if state is None else state
        self._check_state(state)
        if phys.numel() != self.phys_numel or phys.dtype != self.dtype or not phys.is_contiguous():
            raise ValueError("phys must be a contiguous tensor of phys_numel scalars")
        self._sync_stream()
        check(lib().ksc_phys_to_spec(self._h, _ptr(phys), _ptr(state)))
        return state

    def spec_to_phys(self, state: torch.Tensor, phys: torch.Tensor | None = None):
        self._check_state(state)
        if phys is None:
            phys = torch.empty(self.phys_numel, dtype=self.dtype, device=self.device)
        self._sync_stream()
        check(lib().ksc_spec_to_phys(self._h, _ptr(state), _ptr(phys)))
        return phys

    def eval_J(self, state: torch.Tensor, arc: bool = False, out: torch.Tensor | None = None):
        """J2 per curve (FP64 tensor); with arc=True also J_arc."""
        self._check_state(state)
        J2 = self._f64(self.n_curves) if out is None else out
        Ja = self._f64(self.n_curves) if arc else None
        self._sync_stream()
        check(lib().ksc_eval_J(self._h, _ptr(state), _ptr(J2), _ptr(Ja)))
        return (J2, Ja) if arc else J2

    def eval_grad(self, state: torch.Tensor, grad: torch.Tensor | None = None,
                  scale: torch.Tensor | None = None, want_J2: bool = True):
        """Euclidean gradient of J2 (state layout), optionally times scale[c];
        returns (grad, J2 or None)."""
        self._check_state(state)
        grad = torch.empty_like(state) if grad is None else grad
        self._check_state(grad, "grad")
        if scale is not None:
            if scale.dtype != torch.float64 or scale.numel() != self.n_curves:
                raise ValueError("scale must be an FP64 tensor of n_curves entries")
            if not scale.is_contiguous():
                scale = scale.contiguous()
        J2 = self._f64(self.n_curves) if want_J2 else None
        self._sync_stream()
        check(lib().ksc_eval_grad(self._h, _ptr(state), _ptr(grad), _ptr(J2), _ptr(scale)))
        return grad, J2

    def step(self, state_in: torch.Tensor, state_out: torch.Tensor, dtau: float,
             want_J2: bool = False):
        self._check_state(state_in)
        self._check_state(state_out, "state_out")
        J2 = self._f64(self.n_curves) if want_J2 else None
        self._sync_stream()
        check(lib().ksc_step(self._h, _ptr(state_in), _ptr(state_out), float(dtau), _ptr(J2)))
        return J2

    def descend(self, state: torch.Tensor, n_steps: int, dtau: float, every: int = 16,
                scratch: torch.Tensor | None = None, active: torch.Tensor | None = None,
                trace: bool = True):
        """n_steps in-place descent steps; returns the J2 trace
        [n_steps // every, n_curves] (FP64) or None."""
        self._check_state(state)
        scratch = torch.empty_like(state) if scratch is None else scratch
        self._check_state(scratch, "scratch")
        if active is not None:
            if active.dtype != torch.uint8 or active.numel() != self.n_curves:
                raise ValueError("active must be a uint8 tensor of n_curves entries")
        n_rows = int(n_steps) // int(every)
        tr = self._f64(max(n_rows, 1) * self.n_curves).view(max(n_rows, 1), self.n_curves) \
            if trace else None
        self._sync_stream()
        check(lib().ksc_descend(self._h, _ptr(state), _ptr(scratch), int(n_steps), float(dtau),
                                _ptr(tr), int(every), _ptr(active)))
        if tr is not None:
            tr = tr[:n_rows]
        return tr

    def tune(self, cache_path: str | None = None):
        self._sync_stream()
        check(lib().ksc_tune(self._h, cache_path.encode() if cache_path else None))
        return self.launch

    def set_launch(self, policy: int = _lib.KSC_LAUNCH_AUTO, waves: int = 0):
        check(lib().ksc_set_launch(self._h, int(policy), int(waves)))

    SCHEMES = {"paper": _lib.KSC_SCHEME_PAPER, "implicit_s": _lib.KSC_SCHEME_IMPLICIT_S}

    def set_scheme(self, scheme: str = "paper"):
        """Descent scheme of later step / descend calls: "paper" (A_k^2
        implicit) or "implicit_s" (the whole linear part, d/ds included,
        implicit; include/ksc.h, ksc_set_scheme)."""
        if scheme not in self.SCHEMES:
            raise ValueError(f"unknown scheme {scheme!r}")
        check(lib().ksc_set_scheme(self._h, self.SCHEMES[scheme]))

    def set_momentum(self, beta: float = 0.0):
        """Heavy-ball momentum of later descend calls under the implicit_s
        scheme (include/ksc.h, ksc_set_momentum); 0 turns it off."""
        check(lib().ksc_set_momentum(self._h, float(beta)))

    def precondition(self, grad: torch.Tensor, out: torch.Tensor | None = None,
                     dtau: float = 0.05) -> torch.Tensor:
        """The implicit-in-s increment for the Euclidean gradient `grad`
        (include/ksc.h, ksc_precondition): -H0 grad with H0 symmetric positive
        definite; needs set_scheme("implicit_s")."""
        self._check_state(grad, "grad")
        out = torch.empty_like(grad) if out is None else out
        self._check_state(out, "out")
        self._sync_stream()
        check(lib().ksc_precondition(self._h, _ptr(grad), _ptr(out), float(dtau)))
        return out

    @property
    def momentum(self) -> float:
        v = ctypes.c_double()
        check(lib().ksc_get_momentum(self._h, ctypes.byref(v)))
        return float(v.value)

    @property
    def scheme(self) -> str:
        v = ctypes.c_int32()
        check(lib().ksc_get_scheme(self._h, ctypes.byref(v)))
        return {b: a for a, b in self.SCHEMES.items()}[int(v.value)]

    @property
    def launch(self):
        p, w = ctypes.c_int32(), ctypes.c_int32()
        check(lib().ksc_get_launch(self._h, ctypes.byref(p), ctypes.byref(w)))
        return int(p.value), int(w.value)

    def query_flags(self) -> np.ndarray:
        self._sync_stream()
        out = (ctypes.c_uint32 * self.n_curves)()
        check(lib().ksc_query_flags(self._h, out))
        return np.array(out, dtype=np.uint32)

    def set_timing(self, enable: bool = True) -> None:
        """Start (True) or stop (False) a kernel-timing window: HIP events on
        the problem's stream around the fused tile kernel and the post kernel
        of every eval_J / eval_grad / step call."""
        self._sync_stream()
        check(lib().ksc_set_timing(self._h, 1 if enable else 0))

    def read_timing(self):
        """(fused_ms_total, post_ms_total, n_evals) of the current window;
        blocks until the recorded events completed."""
        f, q, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
        check(lib().ksc_read_timing(self._h, ctypes.byref(f), ctypes.byref(q), ctypes.byref(n)))
        return float(f.value), float(q.value), int(n.value)
