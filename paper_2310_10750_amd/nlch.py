"""Thin ctypes binding of ``libnlch.so`` (C ABI in ``include/nlch.h``).

Functions carry the C names and only marshal arguments: device buffers may be
torch tensors (their ``data_ptr()`` is passed) or raw integer addresses, and
streams may be ``torch.cuda.Stream`` objects, raw ``hipStream_t`` integers or
None (the null stream).  Every solver step runs inside the library's HIP
kernels; there is no fallback path, and a missing library raises.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# NLCH_LIB_PATH selects another build of the same library (the tests' host
# sanitizer build).
LIB_PATH = os.environ.get("NLCH_LIB_PATH") or os.path.join(_HERE, "libnlch.so")

NLCH_OK = 0
NLCH_EINVAL = -1
NLCH_EUNSUPPORTED = -2
NLCH_EDEVICE = -3
NLCH_ENOMEM = -4

NLCH_KERNEL_CONSTANT = 0
NLCH_KERNEL_GAUSSIAN = 1

NLCH_F64 = 0
NLCH_F32 = 1
NLCH_F16_STORE = 2

NLCH_ALGO_AUTO = 0
NLCH_ALGO_DIRECT = 1
NLCH_ALGO_ROWRUN = 2
NLCH_ALGO_RESIDENT = 3
NLCH_ALGO_ACC64 = 0x100
NLCH_ALGO_NOGRAPH = 0x200
NLCH_ALGO_CHECK_FINITE = 0x400
NLCH_ALGO_AUTOTUNE = 0x800

NLCH_BOUNDARY_PERIODIC = 0
NLCH_BOUNDARY_VOLUME = 1

NLCH_MFMC_MAX_K = 8
NLCH_MFMC_MAX_POOL = 16

PRECISIONS = {"f64": NLCH_F64, "f32": NLCH_F32, "f16": NLCH_F16_STORE}


class nlch_model(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("kernel", ctypes.c_int32),
                ("delta", ctypes.c_double), ("kernel_amp", ctypes.c_double),
                ("kernel_sigma", ctypes.c_double), ("c_F", ctypes.c_double),
                ("beta1", ctypes.c_double), ("beta2", ctypes.c_double),
                ("tau", ctypes.c_double), ("boundary", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class nlch_sample(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("c_F", ctypes.c_double), ("kernel_amp", ctypes.c_double),
                ("offset", ctypes.c_int64)]


_K8 = ctypes.c_double * NLCH_MFMC_MAX_K


class mfmc_result(ctypes.Structure):
    _fields_ = [("q_mfmc", ctypes.c_double), ("q_mc", ctypes.c_double),
                ("mean_mj", _K8), ("mean_mjm1", _K8), ("var", _K8),
                ("rho", _K8), ("alpha", _K8)]


class mfmc_subset(ctypes.Structure):
    _fields_ = [("size", ctypes.c_int32), ("models", ctypes.c_int32 * NLCH_MFMC_MAX_POOL),
                ("V", ctypes.c_double), ("bmin_over_c1", ctypes.c_double)]


class NlchError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("nlch error %d: %s" % (code, msg))
        self.code = code


_lib = None


def load():
    """Load libnlch.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libnlch.so is not built (%s); run __graft_entry__.build()"
                          % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    i32, i64 = ctypes.c_int32, ctypes.c_int64
    pd = ctypes.POINTER(ctypes.c_double)
    lib.nlch_disc.argtypes = [i32, ctypes.c_double, ctypes.POINTER(i64),
                              ctypes.POINTER(i32), ctypes.POINTER(i64),
                              ctypes.POINTER(i32), i32]
    lib.nlch_disc.restype = ctypes.c_int
    lib.nlch_model_constants.argtypes = [ctypes.POINTER(nlch_model), pd, pd, pd]
    lib.nlch_model_constants.restype = ctypes.c_int
    lib.nlch_step.argtypes = [ctypes.POINTER(nlch_model), i32, i32, vp, vp, vp, vp]
    lib.nlch_step.restype = ctypes.c_int
    lib.nlch_step_noalloc.argtypes = [ctypes.POINTER(nlch_model), i32, i32, vp, vp, vp, vp]
    lib.nlch_step_noalloc.restype = ctypes.c_int
    lib.nlch_solve_batch.argtypes = [ctypes.POINTER(nlch_model), i32,
                                     ctypes.POINTER(nlch_sample), i64, i32, i32,
                                     i32, vp, vp, vp, vp]
    lib.nlch_solve_batch.restype = ctypes.c_int
    lib.nlch_solve_batch_energy.argtypes = [ctypes.POINTER(nlch_model), i32,
                                            ctypes.POINTER(nlch_sample), i64, i32, i32,
                                            i32, vp, vp, vp, vp, vp]
    lib.nlch_solve_batch_energy.restype = ctypes.c_int
    lib.nlch_set_stream_shape.argtypes = [i32, i32, i32, i32]
    lib.nlch_set_stream_shape.restype = ctypes.c_int
    lib.nlch_set_stream_phases.argtypes = [i32]
    lib.nlch_set_stream_phases.restype = ctypes.c_int
    lib.nlch_set_resident_shape.argtypes = [i32, i32]
    lib.nlch_set_resident_shape.restype = ctypes.c_int
    lib.mfmc_estimate.argtypes = [i32, ctypes.POINTER(i64), ctypes.POINTER(vp), i64,
                                  pd, ctypes.POINTER(mfmc_result), vp]
    lib.mfmc_estimate.restype = ctypes.c_int
    lib.mfmc_select.argtypes = [i32, pd, pd, ctypes.POINTER(mfmc_subset), i32,
                                ctypes.POINTER(i32)]
    lib.mfmc_select.restype = ctypes.c_int
    lib.mfmc_allocate.argtypes = [i32, ctypes.POINTER(i32), pd, pd, ctypes.c_double, pd,
                                  ctypes.POINTER(i64), pd]
    lib.mfmc_allocate.restype = ctypes.c_int
    lib.nlch_rowrun_supported.argtypes = [i32, ctypes.POINTER(i64), i32]
    lib.nlch_rowrun_supported.restype = ctypes.c_int
    lib.nlch_last_error.argtypes = []
    lib.nlch_last_error.restype = ctypes.c_char_p
    lib.nlch_version.argtypes = []
    lib.nlch_version.restype = ctypes.c_int
    lib.nlch_debug_inject_device_error.argtypes = [i32]
    lib.nlch_debug_inject_device_error.restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc):
    if rc != NLCH_OK:
        raise NlchError(rc, nlch_last_error())


def _ptr(buf):
    if buf is None:
        return None
    if isinstance(buf, int):
        return buf
    return buf.data_ptr()


def _stream(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def nlch_last_error() -> str:
    return load().nlch_last_error().decode()


def nlch_version() -> int:
    return load().nlch_version()


def nlch_debug_inject_device_error(nth: int) -> None:
    """Make the nth checked HIP call from now on fail (0 disarms)."""
    _check(load().nlch_debug_inject_device_error(nth))


def nlch_rowrun_supported(precision: int = 1):
    """R2 values with row-run kernels for a precision (default NLCH_F32)."""
    lib = load()
    buf = (ctypes.c_int64 * 64)()
    cnt = lib.nlch_rowrun_supported(precision, buf, 64)
    _check(0 if cnt >= 0 else cnt)
    return [buf[i] for i in range(min(cnt, 64))]


def nlch_disc(n: int, delta: float):
    """(R2, m, N, halfw list for dy = -m..m)."""
    lib = load()
    R2 = ctypes.c_int64()
    m = ctypes.c_int32()
    N = ctypes.c_int64()
    _check(lib.nlch_disc(n, delta, ctypes.byref(R2), ctypes.byref(m), ctypes.byref(N),
                         None, 0))
    hw = (ctypes.c_int32 * (2 * m.value + 1))()
    _check(lib.nlch_disc(n, delta, None, None, None, hw, 2 * m.value + 1))
    return R2.value, m.value, N.value, list(hw)


def make_model(n, delta, kernel, amp, sigma=0.0, c_F=1.0, beta1=1.0, beta2=0.0,
               tau=0.01, boundary=0) -> nlch_model:
    return nlch_model(int(n), int(kernel), float(delta), float(amp), float(sigma),
                      float(c_F), float(beta1), float(beta2), float(tau), int(boundary), 0)


def nlch_model_constants(model: nlch_model):
    c = ctypes.c_double()
    xi = ctypes.c_double()
    c1 = ctypes.c_double()
    _check(load().nlch_model_constants(ctypes.byref(model), ctypes.byref(c),
                                       ctypes.byref(xi), ctypes.byref(c1)))
    return c.value, xi.value, c1.value


def nlch_step(model: nlch_model, precision: int, algo: int, u_in, u_out,
              ooi_out=None, stream=None) -> None:
    _check(load().nlch_step(ctypes.byref(model), precision, algo, _ptr(u_in),
                            _ptr(u_out), _ptr(ooi_out), _stream(stream)))


def nlch_step_noalloc(model: nlch_model, precision: int, algo: int, u_in, u_out,
                      ooi_out=None, stream=None) -> None:
    """nlch_step with every device table and partial sum in the library's
    static device area (no device allocation)."""
    _check(load().nlch_step_noalloc(ctypes.byref(model), precision, algo, _ptr(u_in),
                                    _ptr(u_out), _ptr(ooi_out), _stream(stream)))


def nlch_solve_batch(models, samples, nsteps: int, precision: int, algo: int, state,
                     scratch, ooi_out, stream=None) -> None:
    """models: sequence of nlch_model (or a ctypes array); samples: sequence of
    nlch_sample (or a ctypes array)."""
    if not isinstance(models, ctypes.Array):
        models = (nlch_model * len(models))(*models)
    if not isinstance(samples, ctypes.Array):
        samples = (nlch_sample * len(samples))(*samples)
    _check(load().nlch_solve_batch(models, len(models), samples, len(samples),
                                   int(nsteps), precision, algo, _ptr(state),
                                   _ptr(scratch), _ptr(ooi_out), _stream(stream)))


def nlch_solve_batch_energy(models, samples, nsteps: int, precision: int, algo: int,
                            state, scratch, ooi_out, energy_out, stream=None) -> None:
    """nlch_solve_batch plus the energy trace: energy_out holds
    (nsteps + 1) * len(samples) float64, row k = E_h(u^k) per sample."""
    if not isinstance(models, ctypes.Array):
        models = (nlch_model * len(models))(*models)
    if not isinstance(samples, ctypes.Array):
        samples = (nlch_sample * len(samples))(*samples)
    _check(load().nlch_solve_batch_energy(models, len(models), samples, len(samples),
                                          int(nsteps), precision, algo, _ptr(state),
                                          _ptr(scratch), _ptr(ooi_out), _ptr(energy_out),
                                          _stream(stream)))


def nlch_set_stream_shape(R=0, W=0, periods=0, B=0) -> None:
    _check(load().nlch_set_stream_shape(R, W, periods, B))


def nlch_set_stream_phases(phases=0) -> None:
    _check(load().nlch_set_stream_phases(phases))


def nlch_set_resident_shape(cols_per_lane=0, rows_per_lane=0) -> None:
    _check(load().nlch_set_resident_shape(int(cols_per_lane), int(rows_per_lane)))


def mfmc_estimate(ys, m, alpha=None, stream=None, y_stride=1) -> dict:
    """ys: K device arrays (float64) of model outputs (or raw addresses), the
    i-th output of model j at ys[j][i * y_stride]; m: K sample counts."""
    K = len(ys)
    mm = (ctypes.c_int64 * K)(*[int(v) for v in m])
    yp = (ctypes.c_void_p * K)(*[_ptr(y) for y in ys])
    al = None
    if alpha is not None:
        al = (ctypes.c_double * max(1, K - 1))(*[float(a) for a in alpha])
    res = mfmc_result()
    _check(load().mfmc_estimate(K, mm, yp, int(y_stride), al, ctypes.byref(res),
                                _stream(stream)))
    return {
        "q_mfmc": res.q_mfmc,
        "q_mc": res.q_mc,
        "mean_mj": list(res.mean_mj[:K]),
        "mean_mjm1": list(res.mean_mjm1[:K]),
        "var": list(res.var[:K]),
        "rho": list(res.rho[:K]),
        "alpha": list(res.alpha[:K]),
    }


def mfmc_select(cost, rho, cap=None):
    """Feasible model subsets sorted by V: list of (models tuple, V, Bmin/C1),
    and the number of candidates."""
    K = len(cost)
    c = (ctypes.c_double * K)(*[float(v) for v in cost])
    r = (ctypes.c_double * K)(*[float(v) for v in rho])
    cap = (1 << (K - 1)) if cap is None else cap
    out = (mfmc_subset * max(1, cap))()
    ncand = ctypes.c_int32()
    n = load().mfmc_select(K, c, r, out, cap, ctypes.byref(ncand))
    if n < 0:
        _check(n)
    res = [(tuple(out[i].models[:out[i].size]), out[i].V, out[i].bmin_over_c1)
           for i in range(min(n, cap))]
    return res, ncand.value


def mfmc_allocate(subset, cost, rho, budget):
    """(m_real list, m_int list, m1_star) for a subset of pool indices."""
    S = len(subset)
    sub = (ctypes.c_int32 * S)(*[int(v) for v in subset])
    c = (ctypes.c_double * len(cost))(*[float(v) for v in cost])
    r = (ctypes.c_double * len(rho))(*[float(v) for v in rho])
    mr = (ctypes.c_double * S)()
    mi = (ctypes.c_int64 * S)()
    m1 = ctypes.c_double()
    _check(load().mfmc_allocate(S, sub, c, r, float(budget), mr, mi, ctypes.byref(m1)))
    return list(mr), list(mi), m1.value


# ----------------------------------------------------------- marshalling --

def structs_for(workload):
    """nlch_model / nlch_sample arrays for a synth.Workload, states packed
    contiguously in sample order.  Returns (models, samples, total_elements)."""
    from .synth import state_side
    models = (nlch_model * len(workload.models))(*[
        make_model(m.n, m.delta, m.kernel, m.amp, m.sigma, m.c_F, m.beta1, m.beta2,
                   m.tau, getattr(m, "boundary", 0)) for m in workload.models])
    samples = (nlch_sample * len(workload.samples))()
    off = 0
    for i, s in enumerate(workload.samples):
        side = state_side(workload.models[s.model])
        samples[i] = nlch_sample(s.model, 0, float(s.c_F), float(s.amp), off)
        off += side * side
    return models, samples, off
