"""Build the native library librafem.so for gfx950 with hipcc (in-tree).

    python -m paper_2409_13036_amd.build          # or: from paper_2409_13036_amd.build import build

Every source is compiled into one shared object next to this file.  Packed FP32
instructions are disabled for all device code.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "librafem.so")
SOURCES = ["pcg.hip", "kernels.hip", "adjoint.hip", "gmres.hip", "solver.cpp", "abi.cpp",
           "structure.cpp", "mono.cpp", "noalloc.cpp"]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build librafem.so)")


# Host-side AddressSanitizer and UndefinedBehaviorSanitizer (the device code is built as
# usual): each option applies to the host compilation only.
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]


def asan_runtime() -> str:
    """The shared sanitizer runtime of hipcc's clang (linked into the sanitizer build, and
    preloaded into the Python process that loads it)."""
    import glob
    root = os.path.dirname(os.path.dirname(os.path.realpath(hipcc())))
    found = sorted(glob.glob(os.path.join(root, "llvm", "lib", "clang", "*", "lib", "linux",
                                          "libclang_rt.asan-x86_64.so")))
    if not found:
        raise RuntimeError("clang's shared AddressSanitizer runtime not found")
    return found[-1]


def build(verbose: bool = False, jobs: int = 4, sanitize: bool = False) -> str:
    """Compile every source for gfx950 and link librafem.so (librafem_asan.so with the host
    sanitizers); returns its path."""
    cc = hipcc()
    flags = ["-O3" if not sanitize else "-O1", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-I", INCLUDE, "-I", CSRC,
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-function", "-Wno-unused-variable"]
    if sanitize:
        flags += SANITIZE
    lib = LIB if not sanitize else os.path.join(HERE, "librafem_asan.so")
    objdir = tempfile.mkdtemp(prefix="rafem_build_")
    try:
        procs = []
        objs = []
        for src in SOURCES:
            obj = os.path.join(objdir, src + ".o")
            objs.append(obj)
            lang = ["-x", "hip"]
            cmd = [cc, *lang, *flags, "-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
            if len(procs) >= jobs:
                _wait(procs.pop(0))
        while procs:
            _wait(procs.pop(0))
        tmp = lib + ".tmp"
        cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
        if sanitize:
            cmd[1:1] = [asan_runtime()]
        if verbose:
            print(" ".join(cmd), flush=True)
        out = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        if out.returncode != 0:
            raise RuntimeError(f"link failed:\n{out.stdout}")
        os.replace(tmp, lib)
    finally:
        shutil.rmtree(objdir, ignore_errors=True)
    return lib


def _wait(item):
    src, p = item
    out, _ = p.communicate()
    text = out.decode(errors="replace")
    if p.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{text}")
    # keep warnings visible, drop the harmless host-pass note about the packed-fp32 feature
    lines = [l for l in text.splitlines() if "packed-fp32-ops" not in l and l.strip()]
    if lines:
        print(f"[{src}]\n" + "\n".join(lines), file=sys.stderr)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, sanitize="--sanitize" in sys.argv))
