"""Builds libpsl.so (HIP for gfx950 + host C++) in the package directory."""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpsl.so")
SOURCES = ["host_model.cpp", "physics.cpp", "schedule.cpp", "k_sample.hip", "k_transport.hip", "runtime.hip",
           "k_nnls.hip", "k_denoise.hip", "k_probe.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = ["-std=c++17", "-O3", "-fPIC", "-Wall", f"-I{os.path.join(ROOT, 'include')}",
          f"-I{CSRC}"]
DEVICE = ["-x", "hip", "--offload-arch=gfx950", "-munsafe-fp-atomics",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# Host-only units: no floating-point contraction, so the FP64 set-up is
# reproducible bit for bit.
HOST = ["-x", "hip", "--offload-arch=gfx950", "-ffp-contract=off", "-fno-fast-math"]


# Transport kernels: FP32 division and square root from the hardware
# reciprocal / square-root instructions (about 1 ulp) instead of the
# correctly rounded sequences.
PER_FILE = {"k_transport.hip": ["-fno-hip-fp32-correctly-rounded-divide-sqrt"]}


def _compile(src: str, obj: str) -> None:
    flags = (HOST if src.endswith(".cpp") else DEVICE) + PER_FILE.get(src, [])
    cmd = [HIPCC, *COMMON, *flags, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"compile failed: {src}")
    if r.stderr.strip():
        lines = [l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l]
        if any(l.strip() for l in lines):
            sys.stderr.write("\n".join(lines) + "\n")


def build(verbose: bool = True) -> str:
    with tempfile.TemporaryDirectory(prefix="psl_build_") as tmp:
        objs = [os.path.join(tmp, s + ".o") for s in SOURCES]
        with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
            list(ex.map(_compile, SOURCES, objs))
        out = LIB + f".tmp{os.getpid()}"
        cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", out, *objs]
        subprocess.check_call(cmd)
        os.replace(out, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build()
