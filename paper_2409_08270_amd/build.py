"""Builds libflashsplat.so (HIP for gfx950) in-tree with hipcc.

Every translation unit is compiled for gfx950 only, with packed-FP32
instructions disabled and hardware float atomics enabled. The projection unit
is compiled without floating-point contraction because its binary32 results
are part of the bit-exact binning contract.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libflashsplat.so")
ARCH = "gfx950"

SOURCES = {
    "fs_project.hip": ["-ffp-contract=off"],
    "fs_sort.hip": ["-ffp-contract=off"],
    "fs_accum.hip": ["-ffp-contract=fast"],
    "fs_assign.hip": [],
    "fs_select.hip": [],
    "fs_render.hip": [],
    "fs_prompt.hip": ["-ffp-contract=off"],
    "fs_diag.hip": [],
    "fs_api.hip": [],
}

COMMON = [
    "-x", "hip", f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
    "-fhip-fp32-correctly-rounded-divide-sqrt", "-munsafe-fp-atomics",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _compile(src: str, extra, outdir: str, save_temps: bool) -> str:
    obj = os.path.join(outdir, os.path.splitext(os.path.basename(src))[0] + ".o")
    cmd = [hipcc()] + COMMON + extra + ["-c", src, "-o", obj]
    if save_temps:
        cmd.insert(1, "-save-temps=obj")
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, save_temps_dir: str | None = None) -> str:
    """Compile every source and link the shared library (always rebuilds)."""
    outdir = save_temps_dir or tempfile.mkdtemp(prefix="fsbuild_")
    os.makedirs(outdir, exist_ok=True)
    srcs = [(os.path.join(CSRC, s), f) for s, f in SOURCES.items() if os.path.exists(os.path.join(CSRC, s))]
    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda sf: _compile(sf[0], sf[1], outdir, save_temps_dir is not None), srcs))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if save_temps_dir is None:
        shutil.rmtree(outdir, ignore_errors=True)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, save_temps_dir=sys.argv[1] if len(sys.argv) > 1 else None)
