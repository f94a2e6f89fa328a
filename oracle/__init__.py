"""FP64 CPU oracle for the nonlocal obstacle-potential phase-field solve and the
multifidelity Monte Carlo estimator of arXiv 2310.10750.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
``cpu_baseline`` leg are the only callers.  The product library never imports
this package, and this package imports nothing from the product.

``nlch_oracle.c`` holds the lattice solver (plain C, FP64, direct disc sums in
canonical order); this module only marshals numpy arrays into it.  The MFMC
estimator formulas live in :mod:`oracle.mfmc`.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nlch_oracle.c")
# NLCH_ORACLE_LIB selects another build of the same source (the tests'
# AddressSanitizer/UBSan build).
_LIB_PATH = os.environ.get("NLCH_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")

KERNEL_CONSTANT = 0
KERNEL_GAUSSIAN = 1

_lib = None


def build(force: bool = True) -> str:
    """Compile ``nlch_oracle.c`` with gcc (no fast-math) into ``liboracle.so``."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-fno-fast-math", "-fopenmp", "-shared", "-fPIC",
             _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def build_sanitized(path: str) -> str:
    """Compile ``nlch_oracle.c`` with AddressSanitizer and UBSan (gcc; every
    undefined-behaviour report fatal) into ``path``, for a test process that
    preloads gcc's ASan runtime and sets NLCH_ORACLE_LIB."""
    subprocess.check_call(
        ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
         "-fno-sanitize-recover=all", "-fno-fast-math", "-fopenmp", "-shared", "-fPIC",
         _SRC, "-o", path, "-lm"])
    return path


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    i32, i64, f64 = ctypes.c_int, ctypes.c_int64, ctypes.c_double
    pd = ctypes.POINTER(ctypes.c_double)
    pi = ctypes.POINTER(ctypes.c_int)
    pi64 = ctypes.POINTER(ctypes.c_int64)
    lib.orc_disc.argtypes = [i32, f64, pi64, pi, pi64, pi, i32]
    lib.orc_disc.restype = i32
    lib.orc_gamma.argtypes = [i32, f64, f64, f64]
    lib.orc_gamma.restype = f64
    lib.orc_weights.argtypes = [i32, f64, i32, f64, f64, pi, pi, pd, i64, pd]
    lib.orc_weights.restype = i64
    lib.orc_constants.argtypes = [i32, f64, i32, f64, f64, f64, pd, pd, pi64]
    lib.orc_constants.restype = i32
    lib.orc_convolve.argtypes = [i32, f64, i32, f64, f64, pd, pd]
    lib.orc_convolve.restype = i32
    lib.orc_step.argtypes = [i32, f64, i32, f64, f64, f64, f64, f64, pd, pd]
    lib.orc_step.restype = i32
    lib.orc_step_sites.argtypes = [i32, f64, i32, f64, f64, f64, f64, f64, pd,
                                   pi64, i64, pd]
    lib.orc_step_sites.restype = i32
    lib.orc_energy.argtypes = [i32, f64, i32, f64, f64, f64, pd]
    lib.orc_energy.restype = f64
    lib.orc_solve.argtypes = [i32, f64, i32, f64, f64, f64, f64, f64, i32, pd,
                              pd, pd, pd]
    lib.orc_solve.restype = i32
    lib.orc_solve_many.argtypes = [i32, f64, i32, f64, f64, f64, i32, i64, pd,
                                   pd, pd, pd, pd]
    lib.orc_solve_many.restype = i32
    lib.orc_threads.argtypes = []
    lib.orc_threads.restype = i32
    _lib = lib
    return lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != shape:
        raise ValueError("expected shape %s, got %s" % (shape, a.shape))
    return a


class OracleError(RuntimeError):
    pass


def threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return _load().orc_threads()


def disc(n: int, delta: float):
    """Integer disc geometry: (R2, m, N, halfw[2m+1]) for dy = -m..m."""
    lib = _load()
    R2 = ctypes.c_int64()
    m = ctypes.c_int()
    N = ctypes.c_int64()
    if lib.orc_disc(n, delta, ctypes.byref(R2), ctypes.byref(m), ctypes.byref(N),
                    None, 0) != 0:
        raise OracleError("bad disc arguments")
    halfw = np.zeros(2 * m.value + 1, dtype=np.int32)
    lib.orc_disc(n, delta, None, None, None,
                 halfw.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), halfw.size)
    return R2.value, m.value, N.value, halfw


def gamma(kind: int, amp: float, sigma: float, r: float) -> float:
    return _load().orc_gamma(kind, amp, sigma, r)


def weights(n, delta, kind, amp, sigma):
    """Canonical-order disc offsets and weights: (ddy, ddx, w_d, c_gamma_h)."""
    lib = _load()
    _, _, N, _ = disc(n, delta)
    ddy = np.zeros(N, dtype=np.int32)
    ddx = np.zeros(N, dtype=np.int32)
    wd = np.zeros(N, dtype=np.float64)
    c = ctypes.c_double()
    got = lib.orc_weights(n, delta, kind, amp, sigma,
                          ddy.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                          ddx.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                          _dp(wd), N, ctypes.byref(c))
    if got != N:
        raise OracleError("weights failed")
    return ddy, ddx, wd, c.value


def constants(n, delta, kind, amp, sigma, c_F):
    """(c_gamma_h, xi_h, N) of one model."""
    c = ctypes.c_double()
    xi = ctypes.c_double()
    N = ctypes.c_int64()
    if _load().orc_constants(n, delta, kind, amp, sigma, c_F, ctypes.byref(c),
                             ctypes.byref(xi), ctypes.byref(N)) != 0:
        raise OracleError("bad model (need n > 2m)")
    return c.value, xi.value, N.value


def convolve(u, n, delta, kind, amp, sigma):
    u = _f64(u, (n, n))
    g = np.empty_like(u)
    if _load().orc_convolve(n, delta, kind, amp, sigma, _dp(u), _dp(g)) != 0:
        raise OracleError("bad model")
    return g


def step(u, n, delta, kind, amp, sigma, c_F, beta1, tau):
    """One step of the scheme from state u (no initial projection)."""
    u = _f64(u, (n, n))
    out = np.empty_like(u)
    if _load().orc_step(n, delta, kind, amp, sigma, c_F, beta1, tau, _dp(u),
                        _dp(out)) != 0:
        raise OracleError("bad model or 1 + tau*beta1*xi <= 0")
    return out


def step_sites(u, sites, n, delta, kind, amp, sigma, c_F, beta1, tau):
    """One step evaluated at the given flat site indices only."""
    u = _f64(u, (n, n))
    sites = np.ascontiguousarray(sites, dtype=np.int64)
    out = np.empty(sites.size, dtype=np.float64)
    if _load().orc_step_sites(
            n, delta, kind, amp, sigma, c_F, beta1, tau, _dp(u),
            sites.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), sites.size,
            _dp(out)) != 0:
        raise OracleError("bad model or site index")
    return out


def energy(u, n, delta, kind, amp, sigma, c_F):
    u = _f64(u, (n, n))
    e = _load().orc_energy(n, delta, kind, amp, sigma, c_F, _dp(u))
    if not np.isfinite(e):
        raise OracleError("bad model")
    return e


def solve(u0, nsteps, n, delta, kind, amp, sigma, c_F, beta1, tau,
          with_energy=False):
    """Project u0, take nsteps steps.  Returns (u, mean, f1[, energies])."""
    u0 = _f64(u0, (n, n))
    out = np.empty_like(u0)
    mf = np.zeros(2)
    en = np.zeros(nsteps + 1) if with_energy else None
    if _load().orc_solve(n, delta, kind, amp, sigma, c_F, beta1, tau, nsteps,
                         _dp(u0), _dp(out), _dp(mf),
                         _dp(en) if en is not None else None) != 0:
        raise OracleError("bad model or 1 + tau*beta1*xi <= 0")
    if with_energy:
        return out, mf[0], mf[1], en
    return out, mf[0], mf[1]


def solve_many(u0, nsteps, n, delta, kind, sigma, beta1, tau, c_F, amp,
               want_states=True):
    """Independent samples (u0 shape (S, n, n)) with per-sample c_F and
    amplitude.  Returns (states or None, mean[S], f1[S])."""
    u0 = np.ascontiguousarray(u0, dtype=np.float64)
    S = u0.shape[0]
    if u0.shape != (S, n, n):
        raise ValueError("u0 must be (S, n, n)")
    c_F = _f64(np.broadcast_to(np.asarray(c_F, dtype=np.float64), (S,)))
    amp = _f64(np.broadcast_to(np.asarray(amp, dtype=np.float64), (S,)))
    out = np.empty_like(u0) if want_states else None
    mf = np.zeros((S, 2))
    if _load().orc_solve_many(n, delta, kind, sigma, beta1, tau, nsteps, S,
                              _dp(c_F), _dp(amp), _dp(u0),
                              _dp(out) if out is not None else None,
                              _dp(mf)) != 0:
        raise OracleError("bad model or 1 + tau*beta1*xi <= 0")
    return out, mf[:, 0].copy(), mf[:, 1].copy()
