"""Build the HIP library libksc.so in-tree for gfx950.

Every (dtype, n_x) kernel translation unit is compiled separately and in
parallel, then linked with the host runtime into one shared library next to
this file.  Usage: ``python -m paper_2301_11704_amd.build [-j N]``.
"""
from __future__ import annotations

import argparse
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libksc.so")
ARCH = os.environ.get("KSC_ARCH", "gfx950")
NXS = (8, 16, 32, 64, 128, 256)

# -packed-fp32-ops: no packed FP32 instructions are generated.
HIPFLAGS = [
    "-O3", f"--offload-arch={ARCH}", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def _hipcc() -> str:
    h = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    return h


def units():
    """(object name, source, defines) for every kernel translation unit."""
    out = []
    for tname, t in (("f32", "float"), ("f64", "double")):
        d = [f"-DKSC_T={t}", f"-DKSC_TNAME={tname}"]
        for nx in NXS:
            out.append((f"fused_{tname}_{nx}", "ksc_fused.hip", d + [f"-DKSC_NX={nx}"]))
            out.append((f"odd_{tname}_{nx}", "ksc_odd.hip", d + [f"-DKSC_NX={nx}"]))
        for nx in (n for n in NXS if n * (8 if t == "double" else 4) <= 512):
            out.append((f"spec_{tname}_{nx}", "ksc_spec.hip", d + [f"-DKSC_NX={nx}"]))
        out.append((f"mixed_{tname}", "ksc_fused.hip", d + ["-DKSC_MIXED"]))
        out.append((f"oddconv_{tname}", "ksc_odd.hip", d + ["-DKSC_ODD_CONV"]))
    out.append(("simp", "ksc_simp.hip", []))
    return out


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        msg = "\n".join(l for l in (r.stderr or "").splitlines() if "packed-fp32-ops" not in l)
        raise RuntimeError(f"command failed: {' '.join(cmd)}\n{msg}")
    return r


def build(jobs: int | None = None, verbose: bool = False) -> str:
    """Compile every translation unit and link libksc.so; returns its path."""
    os.makedirs(BUILD, exist_ok=True)
    hipcc = _hipcc()
    jobs = jobs or min(8, os.cpu_count() or 4)
    cmds = []
    for name, src, defs in units():
        obj = os.path.join(BUILD, name + ".o")
        cmds.append([hipcc, *HIPFLAGS, *defs, "-c", os.path.join(CSRC, src), "-o", obj])
    host_obj = os.path.join(BUILD, "host.o")
    cmds.append([hipcc, *HIPFLAGS, "-c", os.path.join(CSRC, "ksc_host.hip"), "-o", host_obj])
    # slowest units first
    cmds.sort(key=lambda c: ("256" not in " ".join(c), "128" not in " ".join(c)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        for r, c in zip(ex.map(_run, cmds), cmds):
            if verbose:
                print("built", c[-1], flush=True)
    objs = [c[-1] for c in cmds]
    tmp = LIB + ".tmp"
    _run([hipcc, "-shared", f"--offload-arch={ARCH}", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("-j", type=int, default=None)
    a = ap.parse_args()
    print(build(a.j, verbose=True))
    sys.exit(0)
