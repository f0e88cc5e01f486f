"""Builds libtpcf.so (HIP for gfx950) in-tree with hipcc.

    python -m paper_2408_03036_amd.build            # libtpcf.so
    python -m paper_2408_03036_amd.build --sanitize # libtpcf_san.so

The sanitized variant instruments the host code only (AddressSanitizer and
UndefinedBehaviorSanitizer, every -fsanitize= behind -Xarch_host; the device
code is built as usual). It is for CPU checks of the C ABI: load it with the
clang ASan runtime preloaded (see asan_runtime()) and TPCF_LIBRARY pointing
at it.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libtpcf.so")
BUILD = os.path.join(HERE, "_build")
BUILD_SAN = os.path.join(HERE, "_build_san")
OUT_SAN = os.path.join(BUILD_SAN, "libtpcf_san.so")
SOURCES = ["tpcf.cpp", "tpcf_grid.hip", "tpcf_pairs.hip", "tpcf_contract.hip", "tpcf_xi.hip", "tpcf_cov.hip",
           "tpcf_edge.hip"]
ARCH = os.environ.get("TPCF_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Packed FP32 instructions are kept out of every kernel.
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result"]


# host-only sanitizers: each -fsanitize= directly after -Xarch_host
SAN_FLAGS = ["-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def _compile(src: str, sanitize: bool = False) -> str:
    obj = os.path.join(BUILD_SAN if sanitize else BUILD, src + ".o")
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    cmd = [HIPCC] + FLAGS + (SAN_FLAGS if sanitize else []) + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{res.stdout}\n{res.stderr}")
    return obj


def asan_runtime() -> str:
    """The clang AddressSanitizer runtime matching hipcc, to LD_PRELOAD into a
    process that loads libtpcf_san.so."""
    import glob
    rocm = os.path.dirname(os.path.dirname(os.path.realpath(HIPCC)))
    hits = sorted(glob.glob(os.path.join(rocm, "llvm", "lib", "clang", "*", "lib", "linux",
                                         "libclang_rt.asan-x86_64.so")))
    if not hits:
        raise FileNotFoundError("clang ASan runtime not found under " + rocm)
    return hits[-1]


def build(verbose: bool = False, sanitize: bool = False) -> str:
    """Compiles every source and links libtpcf.so (or, with sanitize, the
    host-sanitized libtpcf_san.so); returns its path."""
    out = OUT_SAN if sanitize else OUT
    os.makedirs(BUILD_SAN if sanitize else BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(6, len(SOURCES))) as ex:
        objs = list(ex.map(lambda src: _compile(src, sanitize), SOURCES))
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, out)
    if verbose:
        print("built", out)
    return out


if __name__ == "__main__":
    build(verbose=True, sanitize="--sanitize" in sys.argv[1:])
    sys.exit(0)
