"""Build the gfx950 shared library libfcrkpm.so in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfcrkpm.so")
SOURCES = ["kernels.hip", "sepconv.hip", "regpass.hip", "fcrkpm.hip"]

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return "hipcc"


# host-side AddressSanitizer + UBSan for a CPU-only check of the host code
# (argument checks, planning, setup logic); the device code is built as usual.
# Load the result with the clang ASan runtime preloaded (see SANITIZER_RUNTIME).
SANITIZE_FLAGS = "-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined " \
                 "-Xarch_host -fno-omit-frame-pointer -Xarch_host -fno-sanitize-recover=undefined"
SAN_LIB = os.path.join(HERE, "_build_san", "libfcrkpm.so")


def sanitizer_runtime() -> str:
    """The clang ASan runtime that matches hipcc's host compiler."""
    base = "/opt/rocm/llvm/lib/clang"
    for v in sorted(os.listdir(base), reverse=True):
        cand = os.path.join(base, v, "lib", "linux", "libclang_rt.asan-x86_64.so")
        if os.path.exists(cand):
            return cand
    raise FileNotFoundError("libclang_rt.asan-x86_64.so not found under " + base)


def build(verbose: bool = False, sanitize: bool = False) -> str:
    """Compile every HIP source into paper_2403_19854_amd/libfcrkpm.so, or with
    sanitize=True the host-sanitized copy _build_san/libfcrkpm.so."""
    objs = []
    bdir = os.path.join(HERE, "_build_san" if sanitize else "_build")
    os.makedirs(bdir, exist_ok=True)
    extra = SANITIZE_FLAGS.split() if sanitize else []
    procs = []
    for src in SOURCES:
        obj = os.path.join(bdir, src.replace(".hip", ".o"))
        cmd = [hipcc(), *HIPCC_FLAGS, *extra, "-I", os.path.join(ROOT, "include"), "-c",
               os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), cmd))
        objs.append(obj)
    for p, cmd in procs:
        if p.wait() != 0:
            raise RuntimeError("hipcc failed: " + " ".join(cmd))
    out = SAN_LIB if sanitize else LIB
    tmp = out + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, sanitize="--sanitize" in sys.argv))
