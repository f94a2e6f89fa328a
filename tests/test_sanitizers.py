"""CPU-side robustness: the FP64 oracle (gcc) and the library's host units
(hipcc, host code only) built with AddressSanitizer and UBSan, each run under
its own sanitizer runtime in a child process over the CPU tests that exercise
it -- the oracle pins, and the argument validation, table building and MFMC
selection of the C ABI.  Every UBSan report is fatal, and each harness is
shown to report a planted heap overflow (built with the same flags), so a
run that checks nothing fails.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2310_10750_amd import build_lib  # noqa: E402

SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _gcc_asan():
    p = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                       text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else ""


def _run(env_extra, args, timeout=900):
    env = dict(os.environ, **SAN_ENV, **env_extra)
    env.pop("PYTEST_XDIST_WORKER", None)
    return subprocess.run([sys.executable] + args, cwd=ROOT, env=env, capture_output=True,
                          text=True, timeout=timeout)


PLANTED_C = r"""
#include <stdlib.h>
int planted(int i) { int *a = malloc(4 * sizeof(int)); a[i] = 1; int v = a[0]; free(a); return v; }
"""


def _check_planted(so, env, libvar):
    code = ("import ctypes; l = ctypes.CDLL(%r); l.planted(4)" % so)
    r = _run(env, ["-c", code], timeout=120)
    # (UBSan's object-size check or ASan's shadow memory, whichever fires first)
    assert r.returncode != 0 and ("heap-buffer-overflow" in r.stderr or
                                  "insufficient space" in r.stderr), r.stderr[-2000:]


def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    asan = _gcc_asan()
    if not asan:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    import oracle
    so = oracle.build_sanitized(str(tmp_path / "liboracle_san.so"))
    env = {"NLCH_ORACLE_LIB": so, "LD_PRELOAD": asan}
    # the harness reports a planted overflow built the same way
    src = tmp_path / "planted.c"
    src.write_text(PLANTED_C)
    planted = str(tmp_path / "libplanted.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", "-shared", "-fPIC", str(src), "-o",
                           planted])
    _check_planted(planted, env, "NLCH_ORACLE_LIB")
    # the child loads the sanitized oracle, and its pins pass
    r = _run(env, ["-c", "import oracle; oracle._load(); "
                         "assert 'liboracle_san.so' in open('/proc/self/maps').read()"])
    assert r.returncode == 0, r.stderr[-3000:]
    r = _run(env, ["-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-p", "no:xdist",
                   "tests/test_oracle_pins.py", "-m", "not gpu"])
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr


def test_host_units_under_address_and_ub_sanitizers(tmp_path):
    asan = build_lib.asan_runtime()
    if not asan:
        pytest.skip("the compiler's shared AddressSanitizer runtime is not installed")
    if not os.path.exists(os.path.join(build_lib.BUILD, "nlch_api.o")):
        pytest.skip("the library is not built (run __graft_entry__.build())")
    so = build_lib.build_host_sanitized(str(tmp_path / "libnlch_san.so"))
    env = {"NLCH_LIB_PATH": so, "LD_PRELOAD": asan}
    src = tmp_path / "planted.cpp"
    src.write_text('extern "C" ' + PLANTED_C.replace("int *a = malloc", "int *a = (int *)malloc"))
    planted = str(tmp_path / "libplanted.so")
    subprocess.check_call([build_lib.HIPCC, "-x", "hip", "--offload-arch=" + build_lib.ARCH,
                           "-fPIC", "-shared", "-shared-libsan"] + build_lib.SAN_HOST +
                          [str(src), "-o", planted])
    _check_planted(planted, env, "NLCH_LIB_PATH")
    r = _run(env, ["-c", "from paper_2310_10750_amd import nlch; nlch.load(); "
                         "assert 'libnlch_san.so' in open('/proc/self/maps').read()"])
    assert r.returncode == 0, r.stderr[-3000:]
    r = _run(env, ["-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-p", "no:xdist",
                   "tests/test_abi_cpu.py", "tests/test_mfmc_selection.py", "-m", "not gpu"])
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
