"""Build libodp.so (HIP kernels + host plan code) for gfx950 with hipcc.

Usage: python -m paper_2011_00162_amd.build [-v]
The shared library is written next to this file, where the binding loads it.

Every HIP source is compiled in two passes: the device pass (gfx950 code object,
bundled) carries the device-only target-feature flags, and the host pass embeds
that bundle.  So the packed-FP32 switch reaches only the AMDGPU backend and the
host compiler never sees a feature it does not know.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libodp.so")

HIP_SOURCES = ["kernels.hip", "pixel.hip", "blind.hip", "loss.hip", "dft_mfma.hip"]
HOST_SOURCES = ["plan.cpp"]

COMMON = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Wall", "-Wno-unused-function",
          "-Wno-unused-variable"]
# Packed-FP32 instructions stay disabled (-packed-fp32-ops): plain float code only.
DEVICE_ONLY = ["-munsafe-fp-atomics", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc() -> str:
    for c in ("/opt/rocm/bin/hipcc", shutil.which("hipcc") or ""):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed: " + " ".join(cmd))
    return res.stderr.strip()


def build(verbose: bool = False) -> str:
    cc = hipcc()
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    hip = [s for s in HIP_SOURCES if os.path.exists(os.path.join(CSRC, s))]
    host = [s for s in HOST_SOURCES if os.path.exists(os.path.join(CSRC, s))]
    tmpd = tempfile.mkdtemp(prefix="odp_build_")
    try:
        def compile_hip(name):
            src = os.path.join(CSRC, name)
            fb = os.path.join(tmpd, name + ".hipfb")
            obj = os.path.join(tmpd, name + ".o")
            w1 = _run([cc, *COMMON, *DEVICE_ONLY, *inc, "--offload-device-only", "-c", src, "-o", fb], verbose)
            w2 = _run([cc, *COMMON, *inc, "--offload-host-only", "-Xclang", "-fcuda-include-gpubinary", "-Xclang",
                       fb, "-c", src, "-o", obj], verbose)
            return obj, "\n".join(w for w in (w1, w2) if w)

        def compile_host(name):
            src = os.path.join(CSRC, name)
            obj = os.path.join(tmpd, name + ".o")
            return obj, _run([cc, *COMMON, *inc, "--offload-host-only", "-c", src, "-o", obj], verbose)

        with ThreadPoolExecutor(max_workers=min(6, os.cpu_count() or 1)) as ex:
            jobs = [ex.submit(compile_hip, s) for s in hip] + [ex.submit(compile_host, s) for s in host]
            results = [j.result() for j in jobs]
        warnings = "\n".join(w for _, w in results if w)
        if warnings:
            sys.stderr.write(warnings + "\n")
        tmp = LIB + ".tmp"
        _run([cc, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp, *[o for o, _ in results]], verbose)
        os.replace(tmp, LIB)
    finally:
        shutil.rmtree(tmpd, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
