"""Build libprgd.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2501_13385_amd.build        # or build() from Python

Every HIP source under csrc/ is compiled to an object in _build/ and linked
into paper_2501_13385_amd/libprgd.so.  Sources are always recompiled.

build_host_sanitized(out_dir) makes a checking variant in out_dir: the same
sources with AddressSanitizer and UndefinedBehaviorSanitizer on the host code
only (device code is built as usual), linked against the shared sanitizer
runtime, which the loading process must preload.
"""

from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libprgd.so")
ARCH = "gfx950"

COMMON = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-fPIC",
    "-std=c++17",
    "-munsafe-fp-atomics",
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


# host-side sanitizers: each flag applies to the host compilation only
HOST_SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-omit-frame-pointer"]


def _compile(src: str, obj_dir: str = BUILD, extra=()) -> str:
    obj = os.path.join(obj_dir, os.path.basename(src)[:-4] + ".o")
    cmd = [hipcc(), *COMMON, *extra, "-c", src, "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    return obj


def _runtime_stub() -> str:
    """An empty link-time stand-in named libamdhip64.so.

    Linking against it records the dependency as ``libamdhip64.so`` (the name
    PyTorch's ROCm build loads its HIP runtime under) instead of the versioned
    ``libamdhip64.so.7``.  In a process that already holds a HIP runtime under
    that name the library then binds to it, so one process never ends up with
    two HIP runtimes; on its own it resolves to ROCm's runtime through the rpath.
    """
    d = os.path.join(BUILD, "stub")
    os.makedirs(d, exist_ok=True)
    src = os.path.join(d, "stub.c")
    with open(src, "w") as f:
        f.write("/* link-time stand-in; the real runtime is resolved at load time */\n")
    out = os.path.join(d, "libamdhip64.so")
    cmd = ["gcc", "-shared", "-fPIC", "-Wl,-soname,libamdhip64.so", "-o", out, src]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"stub build failed: {res.stderr}")
    return d


def _build_into(lib: str, obj_dir: str, extra=(), link_extra=()) -> str:
    os.makedirs(obj_dir, exist_ok=True)
    stub = _runtime_stub()
    srcs = sources()
    jobs = min(len(srcs), max(1, min(8, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, obj_dir, extra), srcs))
    tmp = lib + ".tmp"
    rocm_lib = os.path.join(os.path.dirname(os.path.dirname(os.path.realpath(hipcc()))), "lib")
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *link_extra, f"-L{stub}", "-Wl,--no-as-needed",
           f"-Wl,-rpath,{rocm_lib}", "-o", tmp, *objs]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, lib)
    return lib


def build(verbose: bool = False) -> str:
    _build_into(LIB, BUILD)
    if verbose:
        print(f"built {LIB}")
    return LIB


def build_host_sanitized(out_dir: str) -> str:
    """libprgd.so with host-side ASan + UBSan in out_dir (a checking build)."""
    link = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-shared-libsan"]
    return _build_into(os.path.join(out_dir, "libprgd.so"), os.path.join(out_dir, "obj"), HOST_SANITIZE, link)


def sanitizer_runtime() -> str:
    """Path of the shared ASan runtime of the compiler that builds the library."""
    clang = os.path.join(os.path.dirname(os.path.realpath(hipcc())), "..", "lib", "llvm", "bin", "clang")
    if not os.path.exists(clang):
        clang = "/opt/rocm/llvm/bin/clang"
    res = subprocess.run([clang, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    return res.stdout.strip()


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
