"""Build libqw.so for gfx950 in-tree.

    python -m paper_2609_23664_amd.build

Compiles csrc/*.hip and csrc/*.cpp with hipcc (offload arch gfx950 only) and
links ``paper_2609_23664_amd/libqw.so``. Always recompiles.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libqw.so")
BUILD = os.path.join(HERE, "_build")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = [
    "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", "-ffp-contract=off",
    "-I", INCLUDE, "-I", CSRC,
]
# device code: gfx950 only; packed FP32 ops disabled
DEVICE = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
SOURCES = ["qw_kernels.hip", "qw_mlp.hip", "qw_noalloc.hip", "qw_api.cpp", "qw_plan.cpp", "qw_jit.cpp",
           "qw_tableau.cpp"]
# headers compiled again at run time by hipRTC (embedded as text)
EMBED = [("kEmbedDescH", "qw_desc.h"), ("kEmbedDevH", "qw_dev.h")]


def _embed() -> None:
    """Write the device headers as C++ string literals for the run-time
    compiler (qw_jit.cpp includes the result)."""
    os.makedirs(BUILD, exist_ok=True)
    out = ["// written by build.py: device headers for hipRTC"]
    for name, fn in EMBED:
        with open(os.path.join(CSRC, fn)) as f:
            text = f.read()
        if ")QWEMBED\"" in text:
            raise RuntimeError("embed delimiter inside " + fn)
        out.append(f'static const char {name}[] = R"QWEMBED({text})QWEMBED";')
    path = os.path.join(BUILD, "qw_embed.inc")
    data = "\n".join(out) + "\n"
    old = None
    if os.path.exists(path):
        with open(path) as f:
            old = f.read()
    if old != data:
        with open(path, "w") as f:
            f.write(data)


def _compile(src: str) -> str:
    os.makedirs(BUILD, exist_ok=True)
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    path = os.path.join(CSRC, src)
    if src.endswith(".hip"):
        cmd = [HIPCC, *DEVICE, *COMMON, "-c", path, "-o", obj]
    else:
        cmd = [HIPCC, *COMMON, "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include", "-I", BUILD, "-x", "c++",
               "-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    _embed()
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as pool:
        objs = list(pool.map(_compile, SOURCES))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, *DEVICE, "-shared", "-fPIC", *objs, "-o", tmp,
           "-L/opt/rocm/lib", "-lhiprtc", "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT, flush=True)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
