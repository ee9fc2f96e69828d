"""Build the gfx950 stacking library (libvista.so) in-tree with hipcc.

Every HIP/C++ source is compiled with -ffp-contract=off (the index and table arithmetic
must follow its written FP64 sequence; fused multiply-adds are written explicitly where
wanted) and with packed-FP32 instructions disabled.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC_DIR = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUT_DIR, "libvista.so")
SOURCES = ["vista_kernels.hip", "vista_accum.hip", "vista_sort.hip", "vista_rebin.hip", "vista_image.hip",
           "vista_plan.cpp", "vista_runtime.cpp"]
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math", "-Wall",
          "-Wno-unused-parameter", "-Wno-unused-function", "-Wno-unused-command-line-argument",
          "-I" + os.path.join(HERE, "..", "include")]
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _hipcc() -> str:
    for p in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if p and os.path.exists(p):
            return p
    return "hipcc"


SANITIZERS = ("address", "undefined", "thread")


def _san_flags(sanitize):
    """Host-code sanitizer flags: each -fsanitize= goes after -Xarch_host, so device code
    is built as usual (no GPU sanitizer)."""
    if not sanitize:
        return []
    if sanitize not in SANITIZERS:
        raise ValueError("sanitize must be one of %s" % (SANITIZERS,))
    return ["-Xarch_host", "-fsanitize=" + sanitize, "-Xarch_host", "-fno-omit-frame-pointer"]


def _compile(src: str, verbose: bool, out_dir: str = OUT_DIR, sanitize=None) -> str:
    obj = os.path.join(out_dir, os.path.basename(src) + ".o")
    cmd = [_hipcc()] + COMMON + DEVICE + _san_flags(sanitize) + ["-c", os.path.join(SRC_DIR, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, r.stderr[-6000:]))
    return obj


def build(verbose: bool = False, sanitize: str | None = None) -> str:
    """Compile every source and link libvista.so; returns the library path.

    sanitize = "address", "undefined" or "thread" builds a host-sanitized copy instead, in
    _build_<sanitize>/ (the normal library is left alone).  Load it by pointing VISTA_LIB at
    it, with the sanitizer runtime preloaded, e.g. for AddressSanitizer:
        VISTA_LIB=paper_2609_01897_amd/_build_address/libvista.so \
        LD_PRELOAD=$(/opt/rocm/llvm/bin/clang -print-file-name=libclang_rt.asan-x86_64.so) \
        ASAN_OPTIONS=detect_leaks=0 python -m pytest tests -m "not gpu"
    (the interpreter itself is not instrumented, hence no leak check)."""
    out_dir = OUT_DIR if not sanitize else os.path.join(HERE, "_build_" + sanitize)
    lib = os.path.join(out_dir, "libvista.so")
    os.makedirs(out_dir, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, out_dir, sanitize), SOURCES))
    tmp = lib + ".tmp%d" % os.getpid()
    link_san = ["-fsanitize=" + sanitize, "-shared-libsan"] if sanitize else []
    cmd = [_hipcc(), "-shared", "-fPIC", "--offload-arch=" + ARCH] + link_san + objs + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s" % r.stderr[-6000:])
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    san = next((a.split("=", 1)[1] for a in sys.argv[1:] if a.startswith("--sanitize=")), None)
    print(build(verbose="-v" in sys.argv, sanitize=san))
