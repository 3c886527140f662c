"""Builds libafmpb.so (all HIP sources, gfx950) next to this file."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libafmpb.so")
SOURCES = ["prims", "geometry", "tree", "near", "fmm", "matvec", "krylov", "api", "serve",
           "noalloc", "dual", "gmres"]
FLAGS = ["-std=c++17", "-O3", "--offload-arch=gfx950", "-fPIC",
         # no packed FP32 instructions anywhere in the device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # keep matrix-core accumulators in VGPRs (no per-step AGPR copies)
         "-mllvm", "-amdgpu-mfma-vgpr-form"]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    with tempfile.TemporaryDirectory(prefix="afmpb_build_") as tmp:
        def one(name):
            obj = os.path.join(tmp, name + ".o")
            cmd = [hipcc, *FLAGS, "-c", os.path.join(SRC, name + ".hip"), "-o", obj]
            r = subprocess.run(cmd, capture_output=True, text=True)
            if r.returncode != 0:
                raise RuntimeError(f"hipcc failed for {name}.hip:\n{r.stderr}")
            if verbose and r.stderr.strip():
                print(r.stderr)
            return obj

        with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
            objs = list(ex.map(one, SOURCES))
        out = LIB + ".tmp"
        cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", out, *objs]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"link failed:\n{r.stderr}")
        os.replace(out, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
