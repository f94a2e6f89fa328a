"""Builds libnlch.so (the HIP library behind include/nlch.h) for gfx950.

Each translation unit under csrc/ is compiled by hipcc in parallel into
``_build/`` and linked into ``libnlch.so`` next to this file.  Every HIP unit
is compiled with packed-FP32 instructions disabled.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libnlch.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = [
    "--offload-arch=" + ARCH, "-O3", "-fPIC", "-std=c++17",
    "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    # the row-run kernels rely on full unrolling for static register indices
    "-mllvm", "-pragma-unroll-threshold=2000000",
]


# roctx ranges around graph capture and replay (rocprofv3 --marker-trace)
LINK = ["-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib"]


def sources():
    return sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))


# Units whose arithmetic must not depend on the compiler's scheduling: no
# automatic contraction of a * b + c (every fused multiply-add of the stencil
# path is written out), so that kernels of different layouts that evaluate
# the same operations in the same order give bit-identical results.
NO_CONTRACT = ("kern_rowrun_f16.hip", "kern_rowrun_f32.hip", "kern_rowrun_f64.hip",
               "kern_resident4.hip", "kern_tile.hip",
               "kern_basic.hip", "nlch_noalloc.cpp")


def _compile(src):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    extra = ["-ffp-contract=off"] if src in NO_CONTRACT else []
    cmd = [HIPCC] + COMMON + extra + ["-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd = [HIPCC, "-x", "hip"] + COMMON + extra + ["-c", os.path.join(CSRC, src), "-o", obj]
    t0 = time.time()
    r = subprocess.run(cmd, capture_output=True, text=True)
    return src, obj, r.returncode, r.stdout + r.stderr, time.time() - t0


def _stale(src):
    """True unless the unit's object is newer than it and every header."""
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    if not os.path.exists(obj):
        return True
    deps = [os.path.join(CSRC, src)] + [
        os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")] + [
        os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))]
    return max(os.path.getmtime(f) for f in deps) > os.path.getmtime(obj)


# Host units of the C ABI (argument validation, tables, batches, graphs,
# MFMC selection): the ones the host sanitizer build instruments.
HOST_UNITS = ("nlch_api.cpp", "mfmc_select.cpp", "nlch_noalloc.cpp")
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-g"]


def asan_runtime() -> str:
    """The compiler's shared AddressSanitizer runtime (to preload into a
    process that loads the host sanitizer build)."""
    r = subprocess.run([HIPCC, "--print-file-name=libclang_rt.asan-x86_64.so"],
                       capture_output=True, text=True)
    path = r.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else ""


def build_host_sanitized(path: str, verbose: bool = False) -> str:
    """The library with its host units compiled with AddressSanitizer and
    UBSan (host code only; device code as in the normal build), linked with
    the normal build's kernel objects into ``path``.  Needs a completed
    build()."""
    objs = []
    for src in sources():
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        if src in HOST_UNITS:
            sobj = os.path.join(os.path.dirname(path), os.path.splitext(src)[0] + ".san.o")
            extra = ["-ffp-contract=off"] if src in NO_CONTRACT else []
            cmd = [HIPCC, "-x", "hip"] + COMMON + extra + SAN_HOST + [
                "-c", os.path.join(CSRC, src), "-o", sobj]
            r = subprocess.run(cmd, capture_output=True, text=True)
            if r.returncode != 0:
                raise RuntimeError("hipcc (sanitized) failed on %s:\n%s" % (src, r.stderr))
            objs.append(sobj)
        else:
            if not os.path.exists(obj):
                raise RuntimeError("%s is not built: run build() first" % obj)
            objs.append(obj)
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", path] + objs + LINK + [
        "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
        "-shared-libsan"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("sanitized link failed:\n" + r.stdout + r.stderr)
    return path


PEAKS_SRC = os.path.join(HERE, "peaks", "peaks.hip")
PEAKS = os.path.join(HERE, "peaks", "nlch_peaks")


def build_peaks(verbose: bool = True) -> str:
    """Compiles the peak-measurement program (HBM copy, LDS read, FP32/FP64
    issue rates) with the library's flags."""
    t0 = time.time()
    cmd = [HIPCC] + [f for f in COMMON if f != "-fPIC"] + [PEAKS_SRC, "-o", PEAKS]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed on peaks.hip:\n" + r.stdout + r.stderr)
    if verbose:
        print("  hipcc %-28s %6.1fs" % ("peaks/peaks.hip", time.time() - t0), flush=True)
    return PEAKS


def build(verbose: bool = True, jobs: int = None, incremental: bool = False) -> str:
    """Compiles every unit (or, with incremental, only those whose object is
    older than its sources) and links the library; also builds the
    peak-measurement program."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    todo = [s for s in srcs if _stale(s)] if incremental else srcs
    jobs = jobs or min(max(1, len(todo)), max(1, min(16, os.cpu_count() or 4)))
    objs = [os.path.join(BUILD, os.path.splitext(s)[0] + ".o") for s in srcs]
    with cf.ThreadPoolExecutor(jobs) as ex:
        for src, obj, rc, log, dt in ex.map(_compile, todo):
            if verbose:
                print("  hipcc %-28s %6.1fs" % (src, dt), flush=True)
            if rc != 0:
                raise RuntimeError("hipcc failed on %s:\n%s" % (src, log))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs + LINK
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    if not incremental or not os.path.exists(PEAKS) or (
            os.path.getmtime(PEAKS_SRC) > os.path.getmtime(PEAKS)):
        build_peaks(verbose)
    return LIB


if __name__ == "__main__":
    t = time.time()
    print(build(incremental="--incremental" in sys.argv))
    print("built in %.1fs" % (time.time() - t))
    sys.exit(0)
