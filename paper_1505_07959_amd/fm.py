"""ctypes binding of libfm (include/fm.h): same names, argument marshalling only.

Matrices are torch FP64 CUDA (HIP) tensors; the binding passes their device
pointers and the current HIP stream.  Every computation runs in the library.
Importing this module loads libfm.so and raises if it is missing.
"""

import ctypes
import os

import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libfm.so")

FM_OK = 0
FM_WARN_NOT_CONVERGED = 1
FM_ERR_INVALID = -1
FM_ERR_NOMEM = -2
FM_ERR_DEVICE = -3
FM_ERR_NONFINITE = -4
FM_ERR_UNSUPPORTED = -5

FM_FLOW_INV_HOMOTOPY = 1
FM_FLOW_INV_STEADY = 2
FM_FLOW_SQRT_STEADY = 3
FM_FLOW_EXP = 4
FM_FLOW_INV_LINEAR = 5

FM_F64, FM_F32, FM_BF16, FM_F16, FM_BF16X3 = 0, 1, 2, 3, 4
FM_COARSE_EULER, FM_COARSE_LEARNED, FM_COARSE_CN = 0, 1, 2
FM_FINE_RK4, FM_FINE_EULER, FM_FINE_CN = 0, 1, 2
FM_PARAREAL_CLASSICAL, FM_PARAREAL_MODIFIED = 0, 1

DTYPES = {"f64": FM_F64, "f32": FM_F32, "bf16": FM_BF16, "f16": FM_F16, "bf16x3": FM_BF16X3}


class FmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("libfm status %d: %s" % (status, msg))
        self.status = status


class fm_problem(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("reserved", ctypes.c_int32), ("n", ctypes.c_int64),
                ("A", ctypes.c_void_p), ("lda", ctypes.c_int64)]


class fm_params(ctypes.Structure):
    _fields_ = [("T", ctypes.c_double), ("N", ctypes.c_int32), ("coarse_steps", ctypes.c_int32),
                ("fine_steps", ctypes.c_int32), ("max_iter", ctypes.c_int32), ("coarse", ctypes.c_int32),
                ("max_refine", ctypes.c_int32), ("tol", ctypes.c_double), ("refine_tol", ctypes.c_double),
                ("fine_method", ctypes.c_int32), ("variant", ctypes.c_int32)]


class fm_stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("refine_steps", ctypes.c_int32), ("learned_slices", ctypes.c_int32),
                ("status", ctypes.c_int32), ("increment", ctypes.c_double), ("residual_before", ctypes.c_double),
                ("residual", ctypes.c_double), ("hist", ctypes.c_double * 64),
                ("fine_launches", ctypes.c_int32), ("learned_restarts", ctypes.c_int32), ("fine_ms", ctypes.c_double),
                ("fine_flops", ctypes.c_double), ("fine_phase_ms", ctypes.c_double),
                ("basis_size", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {"iters": self.iters, "refine_steps": self.refine_steps, "learned_slices": self.learned_slices,
                "status": self.status, "increment": self.increment, "residual_before": self.residual_before,
                "residual": self.residual, "hist": list(self.hist[:max(0, min(self.iters, 64))]),
                "fine_launches": self.fine_launches, "learned_restarts": self.learned_restarts,
                "fine_ms": self.fine_ms, "fine_flops": self.fine_flops, "fine_phase_ms": self.fine_phase_ms,
                "basis_size": self.basis_size}


def _load():
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError("libfm.so not found at %s; build it with `python -m paper_1505_07959_amd.build_lib`"
                           % _LIB_PATH)
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    PP = ctypes.POINTER(ctypes.c_void_p)
    lib.fm_flow_create.argtypes = [ctypes.POINTER(P), ctypes.POINTER(fm_problem), ctypes.c_int32, ctypes.c_int32,
                                   ctypes.c_char_p, P]
    lib.fm_parareal_solve.argtypes = [P, PP, PP, ctypes.POINTER(fm_params), ctypes.POINTER(fm_stats), P]
    lib.fm_aima.argtypes = [P, PP, PP, ctypes.c_double, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, PP,
                            ctypes.POINTER(ctypes.c_double), P]
    lib.fm_aima.restype = ctypes.c_int
    lib.fm_cos.argtypes = [P, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(fm_params), P,
                           ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(fm_stats), ctypes.c_char_p, P]
    lib.fm_cos.restype = ctypes.c_int
    lib.fm_fine_propagate.argtypes = [P, ctypes.c_double, ctypes.c_double, ctypes.c_int32, PP, PP, P]
    lib.fm_fine_propagate_noalloc.argtypes = [P, ctypes.c_double, ctypes.c_double, ctypes.c_int32, PP, PP, P]
    lib.fm_coarse_propagate.argtypes = [P, ctypes.c_double, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                        PP, PP, P]
    lib.fm_destroy.argtypes = [P]
    lib.fm_destroy.restype = None
    lib.fm_last_error.restype = ctypes.c_char_p
    for f in ("fm_flow_create", "fm_parareal_solve", "fm_fine_propagate", "fm_fine_propagate_noalloc",
              "fm_coarse_propagate"):
        getattr(lib, f).restype = ctypes.c_int32
    I64, F32, F64, I32 = ctypes.c_int64, ctypes.c_float, ctypes.c_double, ctypes.c_int32
    lib.fm_mlp_param_count.restype = I32
    lib.fm_mlp_forward.argtypes = [P, P, P, I64, P, P, P]
    lib.fm_mlp_loss.argtypes = [P, P, P, P, P, P, F32, I64, P, P, P, P]
    lib.fm_mlp_backward.argtypes = [P, P, P, P, P, I64, P, P, P]
    lib.fm_mlp_adam.argtypes = [P, P, P, P, I64, I32, F32, P]
    lib.fm_learned_features.argtypes = [P, F64, PP, PP, P, P, P, P, I64, P]
    lib.fm_trace_moments.argtypes = [P, ctypes.POINTER(F64), P]
    lib.fm_flow_set_coarse_model.argtypes = [P, I32, ctypes.POINTER(F64), ctypes.POINTER(F64)]
    for f in ("fm_mlp_forward", "fm_mlp_loss", "fm_mlp_backward", "fm_mlp_adam", "fm_learned_features",
              "fm_trace_moments", "fm_flow_set_coarse_model"):
        getattr(lib, f).restype = I32
    return lib


lib = _load()


def fm_last_error():
    return lib.fm_last_error().decode()


def _check(status):
    if status < 0:
        raise FmError(status, fm_last_error())
    return status


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptrs(tensors):
    if tensors is None:
        return None
    arr = (ctypes.c_void_p * len(tensors))()
    for i, t in enumerate(tensors):
        if t is None:
            arr[i] = None
            continue
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
            raise ValueError("matrices must be contiguous float64 device tensors")
        arr[i] = t.data_ptr()
    return arr


def fm_flow_create(problems, dtype, options=None, stream=None):
    """problems: list of (kind, A) with A an n x n float64 device tensor.  Returns the handle."""
    arr = (fm_problem * len(problems))()
    for i, (kind, A) in enumerate(problems):
        if A.dtype != torch.float64 or not A.is_cuda or A.dim() != 2 or A.stride(1) != 1:
            raise ValueError("A must be a row-major float64 device matrix")
        arr[i] = fm_problem(int(kind), 0, int(A.shape[0]), A.data_ptr(), int(A.stride(0)))
    h = ctypes.c_void_p()
    dt = DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
    _check(lib.fm_flow_create(ctypes.byref(h), arr, len(problems), dt,
                              options.encode() if options else None, _stream(stream)))
    return h


def fm_parareal_solve(flow, X0, X_out, params, stream=None):
    """params: list of dicts with the fm_params fields (one per problem).  Returns (status, stats list)."""
    n = len(X_out)
    prm = (fm_params * n)()
    for i, p in enumerate(params):
        prm[i] = fm_params(float(p["T"]), int(p["N"]), int(p.get("coarse_steps", 1)), int(p["fine_steps"]),
                           int(p.get("max_iter", p["N"])), int(p.get("coarse", FM_COARSE_EULER)),
                           int(p.get("max_refine", 0)), float(p.get("tol", 0.0)), float(p.get("refine_tol", 0.0)),
                           int(p.get("fine_method", FM_FINE_RK4)), int(p.get("variant", FM_PARAREAL_CLASSICAL)))
    stats = (fm_stats * n)()
    x0 = _ptrs(X0)
    st = _check(lib.fm_parareal_solve(flow, x0, _ptrs(X_out), prm, stats, _stream(stream)))
    return st, [s.as_dict() for s in stats]


def fm_aima(flow, X0, E, dt, steps, X_out, accel_steps=None, every=0, stream=None):
    """Alg. 8; X0 / E: list of tensors or None (zero).  Returns the residual
    history (list per problem) when every > 0, else None."""
    n = len(X_out)
    nh = steps // every + 1 if every > 0 else 0
    hist = (ctypes.c_double * max(1, n * nh))() if every > 0 else None
    _check(lib.fm_aima(flow, _ptrs(X0), _ptrs(E), float(dt), int(steps),
                       int(steps if accel_steps is None else accel_steps), int(every), _ptrs(X_out),
                       hist, _stream(stream)))
    if hist is None:
        return None
    return [list(hist[i * nh:(i + 1) * nh]) for i in range(n)]


def fm_cos(A, C_out, params, dtype="f64", options=None, stream=None):
    """Alg. 5: cos(A) into C_out.  params: dict of fm_params fields (T = 1).
    Returns (status, m, stats)."""
    if A.dtype != torch.float64 or not A.is_cuda or not A.is_contiguous():
        raise FmError(FM_ERR_INVALID, "A must be a contiguous FP64 device tensor")
    n = A.shape[0]
    p = params
    prm = fm_params(float(p.get("T", 1.0)), int(p["N"]), int(p.get("coarse_steps", 1)), int(p["fine_steps"]),
                    int(p.get("max_iter", p["N"])), int(p.get("coarse", FM_COARSE_EULER)), int(p.get("max_refine", 0)),
                    float(p.get("tol", 0.0)), float(p.get("refine_tol", 0.0)), int(p.get("fine_method", FM_FINE_RK4)),
                    int(p.get("variant", FM_PARAREAL_CLASSICAL)))
    m = ctypes.c_int32(0)
    stats = fm_stats()
    st = _check(lib.fm_cos(ctypes.c_void_p(A.data_ptr()), n, n, DTYPES[dtype] if isinstance(dtype, str) else dtype,
                           ctypes.byref(prm), ctypes.c_void_p(C_out.data_ptr()), ctypes.byref(m),
                           ctypes.byref(stats), options.encode() if options else None, _stream(stream)))
    return st, m.value, stats.as_dict()


def fm_fine_propagate(flow, t_next, t_cur, steps, X_in, X_out, stream=None):
    return _check(lib.fm_fine_propagate(flow, float(t_next), float(t_cur), int(steps), _ptrs(X_in), _ptrs(X_out),
                                        _stream(stream)))


def fm_fine_propagate_noalloc(flow, t_next, t_cur, steps, X_in, X_out, stream=None):
    return _check(lib.fm_fine_propagate_noalloc(flow, float(t_next), float(t_cur), int(steps), _ptrs(X_in),
                                                _ptrs(X_out), _stream(stream)))


FM_NOALLOC_SCRATCH_BYTES = 64 << 20


def fm_coarse_propagate(flow, t_next, t_cur, steps, coarse, X_in, X_out, stream=None):
    return _check(lib.fm_coarse_propagate(flow, float(t_next), float(t_cur), int(steps), int(coarse), _ptrs(X_in),
                                          _ptrs(X_out), _stream(stream)))


def fm_destroy(flow):
    if flow is not None and flow.value:
        lib.fm_destroy(flow)


# ---------------------------------------------------------------- training
def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def fm_mlp_param_count():
    return int(lib.fm_mlp_param_count())


def fm_mlp_forward(theta, norm, X, Y, acts=None, stream=None):
    return _check(lib.fm_mlp_forward(_p(theta), _p(norm), _p(X), int(X.shape[0]), _p(Y), _p(acts), _stream(stream)))


def fm_mlp_loss(Y, cbase, G, bD, fD, fn, rho, dY, Ls, Lsum=None, stream=None):
    return _check(lib.fm_mlp_loss(_p(Y), _p(cbase), _p(G), _p(bD), _p(fD), _p(fn), float(rho), int(Y.shape[0]),
                                  _p(dY), _p(Ls), _p(Lsum), _stream(stream)))


def fm_mlp_backward(theta, norm, X, acts, dY, deltas, grad, stream=None):
    return _check(lib.fm_mlp_backward(_p(theta), _p(norm), _p(X), _p(acts), _p(dY), int(X.shape[0]), _p(deltas),
                                      _p(grad), _stream(stream)))


def fm_mlp_adam(theta, grad, m, v, t, lr, stream=None):
    return _check(lib.fm_mlp_adam(_p(theta), _p(grad), _p(m), _p(v), int(theta.numel()), int(t), float(lr),
                                  _stream(stream)))


def fm_learned_features(flow, h, X, FX, G, bD, fD, fn, row0=0, stream=None):
    return _check(lib.fm_learned_features(flow, float(h), _ptrs(X), _ptrs(FX), _p(G), _p(bD), _p(fD), _p(fn),
                                          int(row0), _stream(stream)))


def fm_trace_moments(flow, batch, stream=None):
    out = (ctypes.c_double * (4 * batch))()
    _check(lib.fm_trace_moments(flow, out, _stream(stream)))
    return [list(out[4 * i:4 * i + 4]) for i in range(batch)]


def fm_flow_set_coarse_model(flow, kind, theta, norm):
    th = (ctypes.c_double * len(theta))(*[float(x) for x in theta])
    nm = (ctypes.c_double * 12)(*[float(x) for x in norm])
    return _check(lib.fm_flow_set_coarse_model(flow, int(kind), th, nm))
