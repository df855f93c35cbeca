"""Python binding of the libhdmr C ABI (include/hdmr.h).

Argument marshalling only: every step of the evaluation and of the build's
hierarchisation runs in the library's HIP kernels.  Device arrays are torch
CUDA (HIP) tensors, float64, contiguous; the stream is torch's current stream
unless one is given.  There is no CPU fallback: if libhdmr.so is missing or
the library reports an error, a HdmrError is raised.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhdmr.so")

HDMR_OK = 0
HDMR_EINVAL = -1
HDMR_ENOMEM = -2
HDMR_EDEVICE = -3
HDMR_ECALLBACK = -4
HDMR_EUNSUPPORTED = -5
PLAIN_FP64 = 0
MIXED = 1

# every function the header declares (checked by the tests)
EXPORTS = (
    "hdmr_init", "asg_build_components", "hdmr_model_from_surpluses", "hdmr_eval", "hdmr_eval_grad",
    "hdmr_get_info", "hdmr_export_component", "hdmr_free", "hdmr_last_error", "hdmr_eval_stats",
    "hdmr_timing_enable", "hdmr_timing_read", "hdmr_model_save", "hdmr_model_load", "hdmr_eval_batched",
    "hdmr_eval_noalloc", "hdmr_model_naive", "hdmr_build_report", "hdmr_quadrature",
    # include/hdmr_irbc.h
    "irbc_residuals", "irbc_solve", "irbc_euler_errors", "irbc_time_step",
    # include/hdmr_surrogate.h
    "mlp_param_count", "mlp_create", "mlp_get_params", "mlp_set_standardization", "mlp_fit_standardization",
    "mlp_get_standardization", "mlp_forward", "mlp_loss_grads", "mlp_train", "mlp_free", "hdmr_model_select",
    "mlp_route_create", "mlp_route_info", "mlp_eval_routed", "mlp_route_free", "mlp_route_set_gate", "mlp_route_gated",
)

_LOCK = threading.Lock()
_LIB = None


class HdmrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("libhdmr error %d: %s" % (code, msg))
        self.code = code


class _BuildParams(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("m", ctypes.c_int32), ("max_order", ctypes.c_int32),
                ("max_level", ctypes.c_int32), ("level_rule", ctypes.c_int32), ("refine_rule", ctypes.c_int32),
                ("eps_gamma", ctypes.c_double), ("anchor", ctypes.c_void_p), ("n_components", ctypes.c_int32),
                ("comp_offsets", ctypes.c_void_p), ("comp_dims", ctypes.c_void_p), ("form", ctypes.c_int32),
                ("eps_eta", ctypes.c_double), ("eps_rho", ctypes.c_double)]


class _Info(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("m", ctypes.c_int32), ("n_components", ctypes.c_int32),
                ("n_tuples", ctypes.c_int32), ("n_rows", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("max_level", ctypes.c_int32), ("max_k", ctypes.c_int32), ("n_passes", ctypes.c_int32),
                ("pass_key_dims", ctypes.c_int32)]


CALLBACK_T = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                              ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p)


def lib():
    """Load libhdmr.so (raises if it has not been built)."""
    global _LIB
    with _LOCK:
        if _LIB is None:
            if not os.path.exists(LIB_PATH):
                raise HdmrError(HDMR_EUNSUPPORTED, "libhdmr.so not built (run __graft_entry__.build())")
            L = ctypes.CDLL(LIB_PATH)
            vp, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
            sig = {
                "hdmr_init": [i32],
                "asg_build_components": [vp, vp, vp, vp],
                "hdmr_model_from_surpluses": [i32, i32, vp, i32, vp, vp, vp, vp, vp, vp, vp, vp],
                "hdmr_eval": [vp, vp, i64, vp, i32, i32, vp],
                "hdmr_eval_noalloc": [vp, vp, i64, vp, i32, i32, vp],
                "hdmr_model_naive": [vp, vp, vp],
                "hdmr_build_report": [vp, vp, vp, vp, vp, vp, vp, vp],
                "hdmr_quadrature": [vp, vp, vp],
                "hdmr_eval_grad": [vp, vp, i64, vp, vp, i32, vp],
                "hdmr_get_info": [vp, vp],
                "hdmr_eval_stats": [vp, vp, i64, vp, vp, vp],
                "hdmr_export_component": [vp, i32, vp, vp, vp, vp, vp, vp, vp],
                "hdmr_timing_enable": [i32],
                "hdmr_timing_read": [ctypes.c_char_p, vp, vp],
                "hdmr_model_save": [vp, ctypes.c_char_p],
                "hdmr_model_load": [ctypes.c_char_p, vp],
                "hdmr_eval_batched": [vp, vp, vp, vp, i32, i32, vp, vp],
                "mlp_param_count": [i32, i32, i32, vp],
                "mlp_create": [i32, i32, i32, vp, vp],
                "mlp_get_params": [vp, vp],
                "mlp_set_standardization": [vp, vp, vp],
                "mlp_fit_standardization": [vp, vp, i64, vp],
                "mlp_get_standardization": [vp, vp, vp],
                "mlp_forward": [vp, vp, i64, vp, vp],
                "mlp_loss_grads": [vp, vp, vp, vp, i32, vp, vp, vp],
                "mlp_train": [vp, vp, vp, vp, i64, i32, ctypes.c_float, vp, vp],
                "hdmr_model_select": [vp, i32, vp, i32, vp, i32, vp],
                "mlp_route_create": [vp, vp, vp, i64, f64, vp],
                "mlp_route_info": [vp, vp, vp, vp],
                "mlp_eval_routed": [vp, vp, i64, vp, i32, vp],
            }
            for name, args in sig.items():
                fn = getattr(L, name)
                fn.restype = ctypes.c_int
                fn.argtypes = args
            for name in ("hdmr_free", "mlp_free", "mlp_route_free"):
                getattr(L, name).restype = None
                getattr(L, name).argtypes = [vp]
            L.hdmr_last_error.restype = ctypes.c_char_p
            L.hdmr_last_error.argtypes = []
            _LIB = L
    return _LIB


def hdmr_last_error() -> str:
    return lib().hdmr_last_error().decode()


def _check(rc):
    if rc != HDMR_OK:
        raise HdmrError(rc, hdmr_last_error())


def hdmr_init(device: int = 0):
    _check(lib().hdmr_init(int(device)))


class Model:
    """Owns an hdmr_model* (freed with hdmr_free)."""

    def __init__(self, handle):
        self._h = ctypes.c_void_p(handle)

    @property
    def handle(self):
        return self._h

    def __del__(self):
        try:
            if self._h and self._h.value and _LIB is not None:
                _LIB.hdmr_free(self._h)
                self._h = ctypes.c_void_p(0)
        except Exception:
            pass

    def info(self):
        return hdmr_get_info(self)


def hdmr_free(model: Model):
    if model._h and model._h.value:
        lib().hdmr_free(model._h)
        model._h = ctypes.c_void_p(0)


def hdmr_model_from_surpluses(model) -> Model:
    """Upload a model dict (d, m, c0, comps, weights, levels, indices, alpha)."""
    d, m = int(model["d"]), int(model["m"])
    comps = [tuple(int(q) for q in S) for S in model["comps"]]
    off = np.zeros(len(comps) + 1, np.int32)
    off[1:] = np.cumsum([len(S) for S in comps])
    dims = np.ascontiguousarray(np.concatenate([np.asarray(S, np.int32) for S in comps]) if comps
                                else np.zeros(1, np.int32), dtype=np.int32)
    npts = np.asarray([np.asarray(a).shape[0] for a in model["alpha"]], np.int64)
    cat = lambda xs, dt: (np.ascontiguousarray(np.concatenate([np.asarray(x, dt).ravel() for x in xs]))
                          if len(xs) else np.zeros(1, dt))
    lv, ix, al = cat(model["levels"], np.uint8), cat(model["indices"], np.uint32), cat(model["alpha"], np.float64)
    c0 = np.ascontiguousarray(model["c0"], dtype=np.float64)
    w = np.ascontiguousarray(model["weights"], dtype=np.float64)
    out = ctypes.c_void_p()
    _check(lib().hdmr_model_from_surpluses(d, m, c0.ctypes.data, len(comps), off.ctypes.data, dims.ctypes.data,
                                           npts.ctypes.data, lv.ctypes.data, ix.ctypes.data, al.ctypes.data,
                                           w.ctypes.data, ctypes.byref(out)))
    return Model(out.value)


def asg_build_components(d, m, anchor, fn, comps=None, max_order=2, max_level=7, level_rule=0, refine_rule=0,
                         eps_gamma=1e-4, form=0, eps_eta=0.0, eps_rho=0.0) -> Model:
    """Build a model on the device.  ``fn`` is a Python callable f(X)->Y or a
    (c_function_address, user_pointer) pair with the hdmr_fn signature.
    eps_eta / eps_rho > 0 apply the Alg. 2 criteria (hdmr_build_report)."""
    p = _BuildParams()
    p.d, p.m, p.max_order, p.max_level = int(d), int(m), int(max_order), int(max_level)
    p.level_rule, p.refine_rule, p.eps_gamma, p.form = int(level_rule), int(refine_rule), float(eps_gamma), int(form)
    p.eps_eta, p.eps_rho = float(eps_eta), float(eps_rho)
    anc = np.ascontiguousarray(anchor, dtype=np.float64)
    p.anchor = anc.ctypes.data
    keep = [anc]
    if comps is not None:
        comps = [tuple(int(q) for q in S) for S in comps]
        off = np.zeros(len(comps) + 1, np.int32)
        off[1:] = np.cumsum([len(S) for S in comps])
        dims = np.ascontiguousarray(np.concatenate([np.asarray(S, np.int32) for S in comps]), dtype=np.int32)
        p.n_components, p.comp_offsets, p.comp_dims = len(comps), off.ctypes.data, dims.ctypes.data
        keep += [off, dims]
    if callable(fn):
        def _cb(Xp, n, dd, Yp, mm, _user):
            try:
                Xa = np.ctypeslib.as_array(ctypes.cast(Xp, ctypes.POINTER(ctypes.c_double)), shape=(n, dd))
                Ya = np.ctypeslib.as_array(ctypes.cast(Yp, ctypes.POINTER(ctypes.c_double)), shape=(n, mm))
                Ya[...] = fn(Xa.copy())
                return 0
            except Exception:
                return -1
        cb = CALLBACK_T(_cb)
        keep.append(cb)
        fptr, uptr = ctypes.cast(cb, ctypes.c_void_p).value, None
    else:
        fptr, uptr = fn
    out = ctypes.c_void_p()
    _check(lib().asg_build_components(ctypes.byref(p), fptr, uptr, ctypes.byref(out)))
    return Model(out.value)


def _stream_ptr(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dev(t, name, shape=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise HdmrError(HDMR_EINVAL, "%s must be a device tensor" % name)
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise HdmrError(HDMR_EINVAL, "%s must be contiguous float64" % name)
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise HdmrError(HDMR_EINVAL, "%s has shape %s, expected %s" % (name, tuple(t.shape), tuple(shape)))
    return ctypes.c_void_p(t.data_ptr())


def hdmr_eval(model: Model, points, values=None, precision=PLAIN_FP64, stream=None):
    """values (n, m) = F(points (n, d)) on the device; returns ``values``."""
    import torch
    inf = hdmr_get_info(model)
    n = points.shape[0]
    if values is None:
        values = torch.empty((n, inf["m"]), dtype=torch.float64, device=points.device)
    _check(lib().hdmr_eval(model.handle, _dev(points, "points", (n, inf["d"])), n,
                           _dev(values, "values", (n, inf["m"])), inf["m"], int(precision), _stream_ptr(stream)))
    return values


def hdmr_model_naive(model: Model, f_anchor) -> Model:
    """The eq (3.16) term-by-term model of an eq (4.2)-form model (f_anchor =
    f(xbar), m values)."""
    import numpy as np
    fa = np.ascontiguousarray(f_anchor, dtype=np.float64)
    h = ctypes.c_void_p()
    _check(lib().hdmr_model_naive(model.handle, fa.ctypes.data, ctypes.byref(h)))
    return Model(h.value)


def hdmr_build_report(model: Model):
    """Alg. 2 report of an adaptive build: dict with 'candidates' (index-set
    tuples in build order), 'eta' (NaN where not tested), 'kept' (bool) and
    'rho' (one per expansion order built)."""
    import numpy as np
    nc, no = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().hdmr_build_report(model.handle, ctypes.byref(nc), ctypes.byref(no), None, None, None, None, None))
    k = np.zeros(nc.value, np.int32)
    dims = np.zeros((nc.value, 4), np.int32)
    eta = np.zeros(nc.value)
    kept = np.zeros(nc.value, np.uint8)
    rho = np.zeros(no.value)
    _check(lib().hdmr_build_report(model.handle, ctypes.byref(nc), ctypes.byref(no), k.ctypes.data, dims.ctypes.data,
                                   eta.ctypes.data, kept.ctypes.data, rho.ctypes.data))
    cands = [tuple(int(v) for v in dims[j, :k[j]]) for j in range(nc.value)]
    return {"candidates": cands, "eta": eta, "kept": kept.astype(bool), "rho": rho}


def hdmr_quadrature(model: Model):
    """(per-component quadratures (ncomp, m) of eq (3.7), total c0 + sum w_S Q u_S (m,))."""
    import numpy as np
    inf = hdmr_get_info(model)
    q = np.zeros((max(inf["n_components"], 1), inf["m"]))
    t = np.zeros(inf["m"])
    _check(lib().hdmr_quadrature(model.handle, q.ctypes.data, t.ctypes.data))
    return q[:inf["n_components"]], t


def hdmr_eval_noalloc(model: Model, points, values, precision=PLAIN_FP64, stream=None):
    """hdmr_eval into the caller's ``values`` (n, m) without device allocation
    (static library workspace); returns ``values``."""
    inf = hdmr_get_info(model)
    n = points.shape[0]
    _check(lib().hdmr_eval_noalloc(model.handle, _dev(points, "points", (n, inf["d"])), n,
                                   _dev(values, "values", (n, inf["m"])), inf["m"], int(precision),
                                   _stream_ptr(stream)))
    return values


def hdmr_eval_grad(model: Model, points, values=None, grad=None, stream=None):
    """Returns (values (n, m), grad (n, d, m))."""
    import torch
    inf = hdmr_get_info(model)
    n, d, m = points.shape[0], inf["d"], inf["m"]
    if values is None:
        values = torch.empty((n, m), dtype=torch.float64, device=points.device)
    if grad is None:
        grad = torch.empty((n, d, m), dtype=torch.float64, device=points.device)
    _check(lib().hdmr_eval_grad(model.handle, _dev(points, "points", (n, d)), n, _dev(values, "values", (n, m)),
                                _dev(grad, "grad", (n, d, m)), m, _stream_ptr(stream)))
    return values, grad


def hdmr_eval_batched(models, points, values=None, precision=PLAIN_FP64, stream=None):
    """Evaluate models[i] at points[i] (device tensors) in one batched call.
    Returns (values list, per-model path array: -1 none, 0 persistent gather,
    1 cell-sorted, 2 cell-sorted with the smaller row batch)."""
    import torch
    k = len(models)
    if len(points) != k or (values is not None and len(values) != k):
        raise HdmrError(HDMR_EINVAL, "models, points and values need the same length")
    infos = [hdmr_get_info(mo) for mo in models]
    if values is None:
        values = [torch.empty((p.shape[0], inf["m"]), dtype=torch.float64, device=p.device)
                  for p, inf in zip(points, infos)]
    mp = (ctypes.c_void_p * max(k, 1))(*[mo.handle.value for mo in models])
    pp = (ctypes.c_void_p * max(k, 1))(*[_dev(p, "points", (p.shape[0], inf["d"])).value
                                         for p, inf in zip(points, infos)])
    vp_ = (ctypes.c_void_p * max(k, 1))(*[_dev(v, "values", (p.shape[0], inf["m"])).value
                                          for v, p, inf in zip(values, points, infos)])
    nn = (ctypes.c_int64 * max(k, 1))(*[p.shape[0] for p in points])
    paths = np.full(max(k, 1), -1, np.int32)
    _check(lib().hdmr_eval_batched(mp, pp, nn, vp_, k, int(precision), paths.ctypes.data, _stream_ptr(stream)))
    return values, paths[:k]


def hdmr_eval_stats(model: Model, points, stream=None):
    """(hits, probes): nonzero basis products and directory lookups of an evaluation."""
    inf = hdmr_get_info(model)
    n = points.shape[0]
    h, p = ctypes.c_int64(), ctypes.c_int64()
    _check(lib().hdmr_eval_stats(model.handle, _dev(points, "points", (n, inf["d"])), n, ctypes.byref(h),
                                 ctypes.byref(p), _stream_ptr(stream)))
    return h.value, p.value


def hdmr_model_save(model: Model, path: str):
    """Write the model to a file (see include/hdmr.h for the layout)."""
    _check(lib().hdmr_model_save(model.handle, os.fsencode(path)))


def hdmr_model_load(path: str) -> Model:
    """Read a model file and build the model on the current device."""
    h = ctypes.c_void_p()
    _check(lib().hdmr_model_load(os.fsencode(path), ctypes.byref(h)))
    return Model(h.value)


def hdmr_timing_enable(on: bool = True):
    """Start (and reset) or stop the device timing of evaluation stages."""
    _check(lib().hdmr_timing_enable(1 if on else 0))


def hdmr_timing_read(stage: str):
    """(total_ms, launches) of a stage ('sort', 'rows', 'contract') since enabling."""
    t, c = ctypes.c_double(), ctypes.c_int64()
    _check(lib().hdmr_timing_read(stage.encode(), ctypes.byref(t), ctypes.byref(c)))
    return t.value, c.value


def hdmr_get_info(model: Model):
    s = _Info()
    _check(lib().hdmr_get_info(model.handle, ctypes.byref(s)))
    return {k: getattr(s, k) for k, _ in _Info._fields_}


def hdmr_export_component(model: Model, comp: int):
    """(dims, levels (N,k) uint8, indices (N,k) uint32, surpluses (N,m) float64, weight)
    of one component, rows in the model's internal order."""
    inf = hdmr_get_info(model)
    n, k = ctypes.c_int64(), ctypes.c_int32()
    _check(lib().hdmr_export_component(model.handle, int(comp), ctypes.byref(n), ctypes.byref(k), None, None, None,
                                       None, None))
    N, K = n.value, k.value
    dims = np.zeros(K, np.int32)
    lv = np.zeros((max(N, 1), K), np.uint8)
    ix = np.zeros((max(N, 1), K), np.uint32)
    al = np.zeros((max(N, 1), inf["m"]), np.float64)
    w = ctypes.c_double()
    _check(lib().hdmr_export_component(model.handle, int(comp), ctypes.byref(n), ctypes.byref(k), dims.ctypes.data,
                                       lv.ctypes.data, ix.ctypes.data, al.ctypes.data, ctypes.byref(w)))
    return tuple(int(q) for q in dims), lv[:N], ix[:N], al[:N], w.value
