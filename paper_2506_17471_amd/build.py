"""Build the HIP library libfemx.so in-tree for gfx950 (hipcc, no JIT).

    python -m paper_2506_17471_amd.build            # build
    python -m paper_2506_17471_amd.build --asm DIR  # also keep the gfx950 assembly in DIR
"""
from __future__ import annotations

import argparse
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfemx.so")
SOURCES = ["kernels_neohookean.hip", "kernels_svk.hip", "kernels_elasticity.hip",
           "kernels_mass.hip", "kernels_laplace.hip", "kernels_helmholtz.hip", "kernels.hip",
           "plan.cpp", "refel.cpp", "tune.cpp", "batch.cpp"]
ARCH = "gfx950"

# Packed FP32 instructions are disabled for the whole library (the build never relies on
# them); FP64 code is unaffected.
HIPFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(HERE, "..", "include"),
]


def _hipcc() -> str:
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.exists(c) or c == "hipcc":
            return c
    raise RuntimeError("hipcc not found")


def build(asm_dir: str | None = None, verbose: bool = False) -> str:
    hipcc = _hipcc()
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)

    def compile_one(src: str) -> str:
        obj = os.path.join(objdir, src + ".o")
        cmd = [hipcc, "-x", "hip", *HIPFLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        if asm_dir and src.endswith(".hip"):
            os.makedirs(asm_dir, exist_ok=True)
            cmd += ["-save-temps=obj"]
            cmd[cmd.index("-o") + 1] = os.path.join(asm_dir, src + ".o")
            obj = cmd[cmd.index("-o") + 1]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
        warn = [l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip()]
        if verbose and warn:
            print("\n".join(warn), file=sys.stderr)
        return obj

    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--asm", default=None, help="directory to keep gfx950 assembly")
    ap.add_argument("-v", "--verbose", action="store_true")
    args = ap.parse_args()
    print(build(args.asm, args.verbose))
