"""Build libqw.so for gfx950 in-tree.

    python -m paper_2609_23664_amd.build [--sanitize]

Compiles csrc/*.hip and csrc/*.cpp with hipcc (offload arch gfx950 only) and
links ``paper_2609_23664_amd/libqw.so``. Always recompiles.

``--sanitize`` builds ``libqw_asan.so`` instead, with the host code (the
planner, generator, tableau and C ABI; device code unchanged) instrumented
by AddressSanitizer and UndefinedBehaviorSanitizer, for host-only checks:

    QW_LIB=paper_2609_23664_amd/libqw_asan.so ASAN_OPTIONS=detect_leaks=0 \
    LD_PRELOAD=$(hipcc -print-file-name=libclang_rt.asan-x86_64.so) \
    python -m pytest tests -m "not gpu"
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
           "qw_tableau.cpp", "qw_persist.cpp"]
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


# host-code sanitizers of the --sanitize build (each flag for the host pass only)
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
BUILD_ASAN = os.path.join(HERE, "_build_asan")
OUT_ASAN = os.path.join(HERE, "libqw_asan.so")


def _compile(src: str, sanitize: bool = False) -> str:
    bdir = BUILD_ASAN if sanitize else BUILD
    os.makedirs(bdir, exist_ok=True)
    obj = os.path.join(bdir, os.path.splitext(src)[0] + ".o")
    path = os.path.join(CSRC, src)
    extra = SANITIZE if sanitize else []
    if src.endswith(".hip"):
        cmd = [HIPCC, *DEVICE, *COMMON, *extra, "-c", path, "-o", obj]
    else:
        cmd = [HIPCC, *COMMON, *extra, "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include", "-I", BUILD, "-x",
               "c++", "-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, sanitize: bool = False) -> str:
    _embed()
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as pool:
        objs = list(pool.map(lambda src: _compile(src, sanitize), SOURCES))
    out = OUT_ASAN if sanitize else OUT
    tmp = out + ".tmp"
    cmd = [HIPCC, *DEVICE, "-shared", "-fPIC", *(SANITIZE if sanitize else []), *objs, "-o", tmp,
           "-L/opt/rocm/lib", "-lhiprtc", "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out)
    if verbose:
        print("built", out, flush=True)
    return out


if __name__ == "__main__":
    build(verbose=True, sanitize="--sanitize" in sys.argv[1:])
    sys.exit(0)
