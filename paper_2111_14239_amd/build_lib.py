"""Build librklt.so (the HIP kernels, the host ABI and the transform designer)
in-tree for gfx950 with hipcc.  Run as ``python -m paper_2111_14239_amd.build_lib``."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "librklt.so")
OBJDIR = os.path.join(PKG, "_build")

SOURCES = ["codec.hip", "codec_mfma.hip", "codec_panel.hip", "codec_quality.hip", "codec_mfma32.hip", "abi.cpp", "transform.cpp", "design.cpp"]

COMMON = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unknown-pragmas",
    "-I", INCLUDE, "-I", CSRC,
]


# per-file flags: the region matrix-core kernel keeps its accumulators
# in ordinary VGPRs (no accumulator-register copies; one more wave per SIMD)
PER_FILE = {"codec_mfma32.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}


def _hipcc() -> str:
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.exists(c) or c == "hipcc":
            return c
    raise RuntimeError("hipcc not found")


def _run(cmd):
    p = subprocess.run(cmd, capture_output=True, text=True)
    # the host pass does not know the packed-fp32 target feature: drop that note
    err = "\n".join(l for l in p.stderr.splitlines()
                    if "packed-fp32-ops" not in l and l.strip())
    if p.returncode != 0:
        raise RuntimeError(f"command failed ({p.returncode}): {' '.join(cmd)}\n{err}")
    return err


def build(verbose: bool = False, out: str = LIB, defines: tuple = ()) -> str:
    """Compile every source and link librklt.so (or `out`, with extra -D
    `defines`, for tuning experiments); returns the library path."""
    objdir = OBJDIR if out == LIB else out + ".objs"
    os.makedirs(objdir, exist_ok=True)
    hipcc = _hipcc()
    jobs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src.rsplit(".", 1)[0] + ".o")
        lang = ["-x", "hip"]
        defs = [f"-D{d}" for d in defines]
        extra = PER_FILE.get(src, [])
        jobs.append(([hipcc, *lang, *COMMON, *extra, *defs, "-c", os.path.join(CSRC, src), "-o", obj], obj))
    with ThreadPoolExecutor(max_workers=len(jobs)) as ex:
        outs = list(ex.map(lambda j: _run(j[0]), jobs))
    if verbose:
        for o in outs:
            if o:
                print(o, file=sys.stderr)
    tmp = out + ".tmp"
    _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *[o for _, o in jobs]])
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
