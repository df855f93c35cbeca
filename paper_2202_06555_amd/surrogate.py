"""ctypes binding of include/hdmr_surrogate.h (same names; argument
marshalling only -- training and inference run in the library's kernels)."""
from __future__ import annotations

import ctypes

import numpy as np

from .hdmr import HDMR_EINVAL, HdmrError, Model, PLAIN_FP64, _check, _dev, _stream_ptr, lib


def _dev_i64(t, name, n):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.int64 or not t.is_contiguous():
        raise HdmrError(HDMR_EINVAL, "%s must be a contiguous int64 device tensor" % name)
    if t.numel() < n:
        raise HdmrError(HDMR_EINVAL, "%s holds %d indices, %d needed" % (name, t.numel(), n))
    return ctypes.c_void_p(t.data_ptr())


class Mlp:
    """Owns an mlp_model* (freed with mlp_free)."""

    def __init__(self, handle, d, width, m):
        self._h = ctypes.c_void_p(handle)
        self.d, self.width, self.m = d, width, m

    @property
    def handle(self):
        if not self._h or not self._h.value:
            raise HdmrError(HDMR_EINVAL, "network already freed")
        return self._h

    def __del__(self):
        try:
            mlp_free(self)
        except Exception:
            pass


class Route:
    """Owns an mlp_route* (freed with mlp_route_free); keeps its network alive."""

    def __init__(self, handle, net, m):
        self._h = ctypes.c_void_p(handle)
        self.net, self.m = net, m

    @property
    def handle(self):
        if not self._h or not self._h.value:
            raise HdmrError(HDMR_EINVAL, "route already freed")
        return self._h

    def __del__(self):
        try:
            mlp_route_free(self)
        except Exception:
            pass


def mlp_param_count(d, width, m) -> int:
    c = ctypes.c_int64()
    _check(lib().mlp_param_count(int(d), int(width), int(m), ctypes.byref(c)))
    return c.value


def mlp_create(d, width, m, params) -> Mlp:
    p = np.ascontiguousarray(params, dtype=np.float32)
    if p.size != mlp_param_count(d, width, m):
        raise HdmrError(HDMR_EINVAL, "expected %d parameters, got %d" % (mlp_param_count(d, width, m), p.size))
    h = ctypes.c_void_p()
    _check(lib().mlp_create(int(d), int(width), int(m), p.ctypes.data, ctypes.byref(h)))
    return Mlp(h.value, int(d), int(width), int(m))


def mlp_get_params(net: Mlp):
    out = np.empty(mlp_param_count(net.d, net.width, net.m), np.float32)
    _check(lib().mlp_get_params(net.handle, out.ctypes.data))
    return out


def mlp_set_standardization(net: Mlp, mean, stdev):
    mu = np.ascontiguousarray(mean, dtype=np.float32)
    sd = np.ascontiguousarray(stdev, dtype=np.float32)
    if mu.size != net.m or sd.size != net.m:
        raise HdmrError(HDMR_EINVAL, "mean and stdev need m values")
    _check(lib().mlp_set_standardization(net.handle, mu.ctypes.data, sd.ctypes.data))


def mlp_fit_standardization(net: Mlp, Y, stream=None):
    _check(lib().mlp_fit_standardization(net.handle, _dev(Y, "Y", (Y.shape[0], net.m)), Y.shape[0],
                                         _stream_ptr(stream)))


def mlp_get_standardization(net: Mlp):
    mu, sd = np.empty(net.m, np.float32), np.empty(net.m, np.float32)
    _check(lib().mlp_get_standardization(net.handle, mu.ctypes.data, sd.ctypes.data))
    return mu, sd


def mlp_forward(net: Mlp, X, Y=None, stream=None):
    import torch
    n = X.shape[0]
    if Y is None:
        Y = torch.empty((n, net.m), dtype=torch.float64, device=X.device)
    _check(lib().mlp_forward(net.handle, _dev(X, "X", (n, net.d)), n, _dev(Y, "Y", (n, net.m)), _stream_ptr(stream)))
    return Y


def mlp_loss_grads(net: Mlp, X, Y, idx, stream=None):
    """(loss, packed gradient) of the batch rows idx (int64 device tensor)."""
    n = X.shape[0]
    b = idx.numel()
    g = np.empty(mlp_param_count(net.d, net.width, net.m), np.float32)
    loss = ctypes.c_float()
    _check(lib().mlp_loss_grads(net.handle, _dev(X, "X", (n, net.d)), _dev(Y, "Y", (n, net.m)),
                                _dev_i64(idx, "idx", b), b, g.ctypes.data, ctypes.byref(loss), _stream_ptr(stream)))
    return loss.value, g


def mlp_train(net: Mlp, X, Y, order, steps, batch, lr0, return_losses=True, stream=None):
    n = X.shape[0]
    losses = np.empty(int(steps), np.float32) if return_losses else None
    _check(lib().mlp_train(net.handle, _dev(X, "X", (n, net.d)), _dev(Y, "Y", (n, net.m)),
                           _dev_i64(order, "order", int(steps) * int(batch)), int(steps), int(batch),
                           ctypes.c_float(lr0), losses.ctypes.data if losses is not None else None,
                           _stream_ptr(stream)))
    return losses


def mlp_free(net: Mlp):
    if net._h and net._h.value:
        lib().mlp_free(net._h)
        net._h = ctypes.c_void_p(0)


def hdmr_model_select(model: Model, comps=None, outs=None, with_c0=True) -> Model:
    c = None if comps is None else np.ascontiguousarray(comps, dtype=np.int32)
    o = None if outs is None else np.ascontiguousarray(outs, dtype=np.int32)
    h = ctypes.c_void_p()
    _check(lib().hdmr_model_select(model.handle, 0 if c is None else c.size, None if c is None else c.ctypes.data,
                                   0 if o is None else o.size, None if o is None else o.ctypes.data,
                                   1 if with_c0 else 0, ctypes.byref(h)))
    return Model(h.value)


def mlp_route_create(net: Mlp, full: Model, Xval, threshold) -> Route:
    n = Xval.shape[0]
    h = ctypes.c_void_p()
    _check(lib().mlp_route_create(net.handle, full.handle, _dev(Xval, "Xval", (n, net.d)), n, float(threshold),
                                  ctypes.byref(h)))
    return Route(h.value, net, net.m)


def mlp_route_info(route: Route):
    """(n_mlp, per-output validated max-abs error, per-output use-network flags)."""
    k = ctypes.c_int32()
    err = np.empty(route.m, np.float64)
    use = np.empty(route.m, np.int32)
    _check(lib().mlp_route_info(route.handle, ctypes.byref(k), err.ctypes.data, use.ctypes.data))
    return k.value, err, use.astype(bool)


def mlp_eval_routed(route: Route, X, Y=None, precision=PLAIN_FP64, stream=None):
    import torch
    n = X.shape[0]
    if Y is None:
        Y = torch.empty((n, route.m), dtype=torch.float64, device=X.device)
    _check(lib().mlp_eval_routed(route.handle, _dev(X, "X", (n, route.net.d)), n, _dev(Y, "Y", (n, route.m)),
                                 int(precision), _stream_ptr(stream)))
    return Y


def mlp_route_free(route: Route):
    if route._h and route._h.value:
        lib().mlp_route_free(route._h)
        route._h = ctypes.c_void_p(0)


def mlp_route_set_gate(route: Route, second, full: Model, tau):
    """Per-point ensemble gate (second network or None to switch it off)."""
    f = lib().mlp_route_set_gate
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double]
    _check(f(route.handle, second.handle if second is not None else None, full.handle, float(tau)))
    route._second = second     # the route borrows the network


def mlp_route_gated(route: Route) -> int:
    f = lib().mlp_route_gated
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    n = ctypes.c_int64()
    _check(f(route.handle, ctypes.byref(n)))
    return n.value
