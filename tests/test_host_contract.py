"""Host-side contracts that need no GPU: the benchmark refuses more than one
GPU, and the binding fails loudly (no fallback) when the HIP library is
missing.  CPU only."""
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
