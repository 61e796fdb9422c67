"""Build the HIP library libfmg.so for gfx950 (in-tree, next to this file).

    python -m paper_1611_05677_amd.build

The device code is split over several translation units (the host recorder
and the multigrid kernels in fmg.hip; the nonlinearity-dependent kernels in
fmg_kind_*.hip), compiled in parallel and linked into one shared library.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfmg.so")
# the same library with AddressSanitizer and UndefinedBehaviorSanitizer on the
# host code (planner, launch sequence, C ABI); device code is built as usual.
# For CPU runs of the ABI tests: preload the ASan runtime (asan_runtime()).
LIB_HOSTSAN = os.path.join(HERE, "libfmg_hostsan.so")
HOSTSAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g"]
SOURCES = ["fmg.hip", "fmg_kind_2d_a.hip", "fmg_kind_2d_b.hip", "fmg_kind_3d_a.hip", "fmg_kind_3d_b.hip",
           "fmg_kind_2d_e.hip", "fmg_kind_3d_e.hip", "fmg_kind_2d_v.hip", "fmg_kind_3d_v.hip"]
ARCH = os.environ.get("FMG_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
    # packed float32 instructions are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def asan_runtime() -> str:
    """Path of the shared ASan runtime of the ROCm clang (to LD_PRELOAD)."""
    clang = os.path.join(os.path.dirname(os.path.realpath(hipcc())), "..", "lib", "llvm", "bin", "clang")
    if not os.path.exists(clang):
        clang = "/opt/rocm/lib/llvm/bin/clang"
    out = subprocess.run([clang, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    return out.stdout.strip()


def is_stale(lib: str) -> bool:
    """True if `lib` is missing or older than a device source or the C header."""
    if not os.path.exists(lib):
        return True
    t = os.path.getmtime(lib)
    srcs = [os.path.join(CSRC, f) for f in os.listdir(CSRC)]
    srcs.append(os.path.join(os.path.dirname(os.path.dirname(CSRC)), "include", "fmg.h"))
    return any(os.path.getmtime(f) > t for f in srcs if os.path.isfile(f))


def build_host_sanitized(verbose: bool = False) -> str:
    return build(verbose, lib=LIB_HOSTSAN, extra=HOSTSAN_FLAGS)


def build(verbose: bool = False, jobs: int | None = None, lib: str = LIB, extra=()) -> str:
    cc = hipcc()
    jobs = jobs or min(len(SOURCES), max(1, os.cpu_count() or 1))
    with tempfile.TemporaryDirectory(prefix="fmg_build_") as tmpdir:
        objs, pending = [], []
        for src in SOURCES:
            obj = os.path.join(tmpdir, os.path.splitext(src)[0] + ".o")
            cmd = [cc, *HIPCC_FLAGS, *extra, "-c", "-o", obj, os.path.join(CSRC, src)]
            if verbose:
                print(" ".join(cmd), flush=True)
            objs.append(obj)
            pending.append(cmd)
        running = []
        failed = []
        while pending or running:
            while pending and len(running) < jobs:
                cmd = pending.pop(0)
                running.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                                                      text=True)))
            cmd, proc = running.pop(0)
            out, _ = proc.communicate()
            if proc.returncode != 0:
                failed.append((cmd, out))
        if failed:
            for cmd, out in failed:
                sys.stderr.write(" ".join(cmd) + "\n" + out)
            raise RuntimeError("hipcc failed building libfmg.so")
        tmp = lib + ".tmp"
        link = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *extra, "-o", tmp, *objs]
        if verbose:
            print(" ".join(link), flush=True)
        res = subprocess.run(link, capture_output=True, text=True)
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError("linking libfmg.so failed")
        os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose=True))
