"""Host-side contracts that need no GPU: the benchmark refuses more than one
GPU, its roofline bookkeeping (algorithmic bytes and flops, the recorded
HBM traffic and its validity) and its CPU-baseline record; the binding
fails loudly (no fallback) when the HIP library is missing.  CPU only."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_binding_raises_without_the_library(tmp_path, monkeypatch):
    from paper_2301_11704_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "libksc.so"))
    monkeypatch.setattr(_lib, "_lib", None)  # drop a library loaded by earlier tests
    with pytest.raises(Exception) as e:
        _lib.lib()
    assert "libksc.so" in str(e.value)


def _bench():
    # imported under its own name: the CPU baseline's worker processes
    # unpickle its task function as bench._oracle_eval
    import importlib
    return importlib.import_module("bench")


def test_bench_algorithmic_bytes_and_flops_of_the_headline_batch():
    """64 curves x 1024 rows x (K + 1 = 43) complex FP32 values, read and
    written once: 45.09 MB per launch; n_x (10 log2 n_x + 12) flops per row."""
    import ksinputs
    b = _bench()
    assert b.flops_per_row(128) == 128 * (10 * 7 + 12)
    assert b.flops_per_row(256) == 256 * (10 * 8 + 12)
    specs = ksinputs.config_specs(4)
    nbytes, flops = b._alg_per_launch(specs, 4, "full")
    assert nbytes == 2 * 2 * 4 * 64 * 1024 * 43 == 45088768
    assert flops == 64 * 1024 * 10496
    nb64, _ = b._alg_per_launch(specs, 8, "full")
    assert nb64 == 2 * nbytes
    nbo, _ = b._alg_per_launch(specs, 4, "odd")
    assert nbo == 2 * 4 * 64 * 1024 * 42


def test_bench_recorded_traffic_holds_only_for_the_profiled_sources(monkeypatch):
    """The committed counter summary gives the HBM bytes of the headline
    kernel (a little above the algorithmic bytes: halo rows, edge buffer),
    and nothing once the kernel sources hash differently."""
    import ksinputs
    b = _bench()
    alg, _ = b._alg_per_launch(ksinputs.config_specs(4), 4, "full")
    t = b.recorded_traffic("c4", "f32")
    assert t is not None and 1.0 < t / alg < 1.3
    assert b.recorded_traffic("c9", "f32") is None
    monkeypatch.setattr(b, "kernel_source_hash", lambda space="full": "0" * 64)
    assert b.recorded_traffic("c4", "f32") is None


def test_bench_cpu_baseline_record():
    """The oracle timed on the host: the fields the bench line carries, on a
    sample of a fraction of a second."""
    import ksinputs
    b = _bench()
    specs = ksinputs.config_specs(0)
    Us = [ksinputs.make_curve(s, (s.n_x - 1) // 3 + 1)[2] for s in specs]
    r = b.cpu_baseline(specs, Us, budget_s=0.3, single_s=0.2)
    assert r["kind"] == "oracle" and r["unit"] == "curve-point evals/s"
    assert r["value"] > 0 and r["single_thread"]["value"] > 0
    assert 1 <= r["cores"] <= 16 and "worker processes" in r["sample"]
    assert "cpu_model" in r
