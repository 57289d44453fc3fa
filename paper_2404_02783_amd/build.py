"""Build the pmhip shared library (hand-written HIP kernels for gfx950) in-tree.

``python -m paper_2404_02783_amd.build`` compiles every source under ``csrc/`` with
hipcc for gfx950 and links ``libpmhip.so`` next to this file.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libpmhip.so")
BUILD = os.path.join(HERE, "_build")
ARCH = os.environ.get("PM_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "-x", "hip", f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
    "-munsafe-fp-atomics",
    # keep the compiler away from packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]
SOURCES = ["fft.hip", "deposit.hip", "particles.hip", "spectra.hip", "adjoint.hip", "api.cpp", "cosmo.cpp",
           "batch.cpp", "microbench.hip"]


def source_digest() -> str:
    """sha256 over every file of csrc/ and include/pmhip.h (names and contents): the
    build record compiled into the library (pm_build_info) and compared with the
    tree by the tests and smoke()."""
    import hashlib
    h = hashlib.sha256()
    files = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if not f.startswith("."))
    files.append(os.path.join(os.path.dirname(HERE), "include", "pmhip.h"))
    for path in files:
        with open(path, "rb") as f:
            h.update(os.path.basename(path).encode() + b"\0" + f.read())
    return h.hexdigest()


def _compile(src: str, digest: str = "unknown") -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = ["hipcc", *FLAGS, f'-DPM_SOURCE_DIGEST="{digest}"', f'-DPM_OFFLOAD_ARCH="{ARCH}"', "-c",
           os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    if r.stderr.strip():
        sys.stderr.write(r.stderr)
    return obj


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    digest = source_digest()
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda src: _compile(src, digest), SOURCES))
    tmp = OUT + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT} (sources {digest[:16]})")
    return OUT


if __name__ == "__main__":
    build()
