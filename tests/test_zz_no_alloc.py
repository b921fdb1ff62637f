"""The allocation-free cost entry point (ksc_eval_J_noalloc, for callers that
cannot allocate device memory) against the problem-object entry point
ksc_eval_J, called through the C ABI: two calls in a row, the second on a
smaller batch; a batch beyond the fixed scratch size is refused."""
import ctypes

import numpy as np
import pytest

import ksinputs
from helpers import seeded_state

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _noalloc(desc, n_curves, dtype, X, J2):
    from paper_2301_11704_amd import _lib
    L = _lib.lib()
    d = desc.to_c()
    st = L.ksc_eval_J_noalloc(ctypes.byref(d), n_curves, _lib.KSC_F64 if dtype == torch.float64
                              else _lib.KSC_F32, ctypes.c_void_p(X.data_ptr()),
                              ctypes.c_void_p(J2.data_ptr()),
                              ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_noalloc_cost_matches_problem_entry_point(dtype):
    import paper_2301_11704_amd as ksc
    npdt = np.float32 if dtype == torch.float32 else np.float64
    tol = 1e-5 if dtype == torch.float32 else 1e-12
    # each call on a smaller batch than the one before (the last two: 16 lanes
    # per row in FP32 at N_x = 256, then one row per lane)
    cases = [(64, 1024, 128, 66.0, "finite", 20.0), (2, 2048, 256, 100.0, "rational", 40.0),
             (5, 300, 64, 39.0, "rational", 40.0)]
    for n_c, n_s, n_x, L, map_, scale in cases:
        desc = ksc.CurveDesc(n_s, n_x, L, map_, scale)
        prob = ksc.Problem([desc] * n_c, dtype=dtype)
        X = prob.new_state()
        for c in range(n_c):
            sp = ksinputs.CurveSpec(n_s, n_x, L, 6, 1.0, 4, 0.2, True, (98, c), map_, scale)
            prob.upload(X, c, seeded_state(sp, npdt))
        ref = prob.eval_J(X)
        J2 = torch.full((n_c,), float("nan"), dtype=torch.float64, device="cuda")
        assert _noalloc(desc, n_c, dtype, X, J2) == 0
        torch.cuda.synchronize()
        r, g = ref.cpu().numpy(), J2.cpu().numpy()
        err = np.abs(g - r).max() / np.abs(r).max()
        print(f"{n_c} curves n_s={n_s} n_x={n_x} {dtype}: noalloc vs eval_J {err:.2e}", flush=True)
        assert np.all(np.isfinite(g)) and err <= tol


def test_noalloc_refuses_a_batch_beyond_its_scratch():
    import paper_2301_11704_amd as ksc
    from paper_2301_11704_amd import _lib
    desc = ksc.CurveDesc(1 << 20, 128, 66.0, "finite", 20.0)
    X = torch.zeros(16, dtype=torch.float32, device="cuda")  # never read: refused first
    J2 = torch.zeros(16, dtype=torch.float64, device="cuda")
    assert _noalloc(desc, 4096, torch.float32, X, J2) == -2
    assert b"KSC_NOALLOC_SCRATCH_BYTES" in _lib.lib().ksc_last_error()
