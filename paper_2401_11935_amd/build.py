"""Builds lib/libdcsd.so from csrc/ with hipcc for gfx950 (in-tree)."""
from __future__ import annotations

import glob
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "lib", "libdcsd.so")
OBJ = os.path.join(ROOT, "_build", "obj")
GEN = os.path.join(ROOT, "_build", "gen")

FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         # no packed-FP32 instructions anywhere in this library
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise FileNotFoundError("hipcc not found")


def generate_tables(verbose: bool = False) -> None:
    """Compile and run gen_coupling_tables.cpp (host C++), writing the coupling
    kernel's compile-time tables to _build/gen/coupling_tables.inc."""
    os.makedirs(GEN, exist_ok=True)
    exe = os.path.join(GEN, "gen_coupling_tables")
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        raise FileNotFoundError("a host C++ compiler (g++) is needed to generate the coupling tables")
    cmd = [cxx, "-std=c++17", "-O1", "-o", exe, os.path.join(CSRC, "gen_coupling_tables.cpp")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"table generator failed to compile:\n{r.stderr}")
    r = subprocess.run([exe], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"table generator failed:\n{r.stderr}")
    out = os.path.join(GEN, "coupling_tables.inc")
    tmp = out + ".tmp"
    with open(tmp, "w") as f:
        f.write(r.stdout)
    os.replace(tmp, out)
    if verbose:
        print(" ".join(cmd), "&&", exe, ">", out)


def build(verbose: bool = False) -> str:
    generate_tables(verbose)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))
    srcs = [x for x in srcs if not os.path.basename(x).startswith("gen_")]
    os.makedirs(OBJ, exist_ok=True)
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    cc = hipcc()

    def compile_one(src):
        obj = os.path.join(OBJ, os.path.basename(src) + ".o")
        cmd = [cc, *FLAGS, "-I", GEN, "-c", src, "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
        if verbose:
            print(" ".join(cmd))
        return obj

    jobs = max(1, min(len(srcs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(compile_one, srcs))
    tmp = OUT + ".tmp"
    cmd = [cc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
