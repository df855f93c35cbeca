"""ctypes binding of include/hdmr_irbc.h (argument marshalling only): the
smooth IRBC model's expectation operator and first-order-condition residuals
with the previous policy held as an HDMR model."""
from __future__ import annotations

import ctypes

from .hdmr import HdmrError, HDMR_EINVAL, Model, _check, _dev, _stream_ptr, hdmr_get_info, lib


class IrbcParams(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("beta", ctypes.c_double), ("alpha", ctypes.c_double),
                ("delta", ctypes.c_double), ("sigma", ctypes.c_double), ("rho", ctypes.c_double),
                ("phi", ctypes.c_double), ("gamma_lo", ctypes.c_double), ("gamma_span", ctypes.c_double),
                ("a_lo", ctypes.c_double), ("a_hi", ctypes.c_double), ("k_lo", ctypes.c_double),
                ("k_hi", ctypes.c_double)]


def params(p: dict) -> IrbcParams:
    return IrbcParams(**{name: p[name] for name, _ in IrbcParams._fields_})


def _fn():
    f = lib().irbc_residuals
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    return f


def irbc_residuals(policy: Model, p: dict, states, choice, residuals=None, expect=None, stream=None):
    """(residuals (n, N+1), expectations (n, N) or None) on the device."""
    import torch
    N = int(p["N"])
    n = states.shape[0]
    inf = hdmr_get_info(policy)
    if inf["d"] != 2 * N or inf["m"] != N + 1:
        raise HdmrError(HDMR_EINVAL, "policy model shape does not match N")
    if residuals is None:
        residuals = torch.empty((n, N + 1), dtype=torch.float64, device=states.device)
    prm = params(p)
    _check(_fn()(policy.handle, ctypes.byref(prm), _dev(states, "states", (n, 2 * N)),
                 _dev(choice, "choice", (n, N + 1)), n, _dev(residuals, "residuals", (n, N + 1)),
                 _dev(expect, "expect", (n, N)) if expect is not None else None, _stream_ptr(stream)))
    return residuals, expect


def irbc_solve(policy: Model, p: dict, states, x, max_iter=20, tol=1e-11, stream=None):
    """Newton solve of the FOCs in place on x (n, N+1); returns (x, iters, max |residual|)."""
    N = int(p["N"])
    n = states.shape[0]
    f = lib().irbc_solve
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                  ctypes.c_int32, ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    prm = params(p)
    it, worst = ctypes.c_int32(), ctypes.c_double()
    _check(f(policy.handle, ctypes.byref(prm), _dev(states, "states", (n, 2 * N)), _dev(x, "x", (n, N + 1)), n,
             int(max_iter), float(tol), ctypes.byref(it), ctypes.byref(worst), _stream_ptr(stream)))
    return x, it.value, worst.value


def irbc_euler_errors(policy: Model, p: dict, states, errors=None, stream=None):
    import torch
    N = int(p["N"])
    n = states.shape[0]
    if errors is None:
        errors = torch.empty((n, N + 1), dtype=torch.float64, device=states.device)
    f = lib().irbc_euler_errors
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                  ctypes.c_void_p]
    prm = params(p)
    _check(f(policy.handle, ctypes.byref(prm), _dev(states, "states", (n, 2 * N)), n,
             _dev(errors, "errors", (n, N + 1)), _stream_ptr(stream)))
    return errors


def irbc_time_step(prev: Model, p: dict, comps, max_level=5, eps_gamma=1e-4, level_rule=0, max_iter=20, tol=1e-11):
    """One time-iteration step: (new policy Model, largest Newton iterations, largest final residual)."""
    import numpy as np
    from .hdmr import _BuildParams
    N = int(p["N"])
    d, m = 2 * N, N + 1
    bp = _BuildParams()
    bp.d, bp.m, bp.max_order, bp.max_level = d, m, 2, int(max_level)
    bp.level_rule, bp.refine_rule, bp.eps_gamma, bp.form = int(level_rule), 0, float(eps_gamma), 0
    anc = np.full(d, 0.5)
    bp.anchor = anc.ctypes.data
    comps = [tuple(int(q) for q in S) for S in comps]
    off = np.zeros(len(comps) + 1, np.int32)
    off[1:] = np.cumsum([len(S) for S in comps])
    dims = np.ascontiguousarray(np.concatenate([np.asarray(S, np.int32) for S in comps]), dtype=np.int32)
    bp.n_components, bp.comp_offsets, bp.comp_dims = len(comps), off.ctypes.data, dims.ctypes.data
    f = lib().irbc_time_step
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_double,
                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    prm = params(p)
    out, it, worst = ctypes.c_void_p(), ctypes.c_int32(), ctypes.c_double()
    _check(f(prev.handle, ctypes.byref(prm), ctypes.byref(bp), int(max_iter), float(tol), ctypes.byref(out),
             ctypes.byref(it), ctypes.byref(worst)))
    return Model(out.value), it.value, worst.value
