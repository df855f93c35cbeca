"""FP64 CPU oracle for cut-HDMR expansions with sparse-grid components.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the GPU library (``paper_2202_06555_amd``) and never imports it; the
two meet only through the seeded inputs of ``workloads``.

Paper: Eftekhari & Scheidegger, "High-Dimensional Dynamic Stochastic Model
Representation", arXiv 2202.06555.  The arithmetic lives in ``orc.c`` (plain
C, FP64, Neumaier-compensated sums); this module marshals numpy arrays and
adds the small combinatorial pieces (eq (4.2) coefficients, exact cut-HDMR of
an analytic function) in plain Python.

Pinned functions and their pins (tests/test_oracle_*.py):
  hat / dhat            eq (3.1) closed-form values, golden table
  regular_grid          eq (3.5) sizes, Table 2 SG* column
  hierarchize           interpolation property, stencil route, surplus recovery
  eval (both modes)     brute force == level-wise, hat-span reproduction,
                        additive recovery, cut-HDMR telescoping at nodes
  grad                  central differences inside cells, hand cases
  build_model           regular limit == regular_grid, anchor-line zeros
  paper_coefficients    constant reproduction, closed form, Fig. 4 example
  evaluate_naive        equals the eq (4.2) regrouping a(x)^T b; telescoping at
                        HDMR nodes (eq (2.2.6))
  quadrature            exact integral of the piecewise-(bi)linear interpolant
                        by a midpoint rule finer than the finest level
  build_ddsg            eta / rho / Z against closed forms for functions whose
                        component functions lie in the hat span
  cut_hdmr_exact        Fig. 3 truncation exactness
"""
from __future__ import annotations

import ctypes
import itertools
import math
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liborc.so")
_LOCK = threading.Lock()
_LIB = None


def build_library(force: bool = True) -> str:
    """Compile orc.c with gcc (-O2, OpenMP) into oracle/liborc.so."""
    src = os.path.join(_HERE, "orc.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-o", tmp, src, "-lm"])
        os.replace(tmp, _SO)
    return _SO


class _Model(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("m", ctypes.c_int32), ("ncomp", ctypes.c_int32),
                ("pad_", ctypes.c_int32),
                ("c0", ctypes.c_void_p), ("comp_off", ctypes.c_void_p), ("comp_dims", ctypes.c_void_p),
                ("comp_npts", ctypes.c_void_p), ("levels", ctypes.c_void_p), ("indices", ctypes.c_void_p),
                ("alpha", ctypes.c_void_p), ("weights", ctypes.c_void_p)]


class _BuildArgs(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("d", ctypes.c_int32), ("m", ctypes.c_int32),
                ("max_level", ctypes.c_int32), ("level_rule", ctypes.c_int32),
                ("refine_rule", ctypes.c_int32), ("eps_gamma", ctypes.c_double),
                ("dims", ctypes.c_void_p), ("anchor", ctypes.c_void_p)]


class _Grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("cap", ctypes.c_int64), ("lv", ctypes.c_void_p),
                ("ix", ctypes.c_void_p), ("ag", ctypes.c_void_p), ("au", ctypes.c_void_p),
                ("acc", ctypes.c_void_p)]


CALLBACK_T = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                              ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p)


def lib():
    global _LIB
    with _LOCK:
        if _LIB is None:
            if not os.path.exists(_SO):
                build_library(force=False)
            L = ctypes.CDLL(_SO)
            vp, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
            L.orc_hat.restype = f64
            L.orc_hat.argtypes = [i32, i64, f64]
            L.orc_dhat.restype = f64
            L.orc_dhat.argtypes = [i32, i64, f64]
            L.orc_eval_brute.restype = ctypes.c_int
            L.orc_eval_brute.argtypes = [vp, vp, i64, vp, vp]
            L.orc_grad_brute.restype = ctypes.c_int
            L.orc_grad_brute.argtypes = [vp, vp, i64, vp, vp]
            L.orc_eval_levelwise.restype = ctypes.c_int
            L.orc_eval_levelwise.argtypes = [vp, vp, i64, vp, vp, vp]
            L.orc_regular_grid.restype = i64
            L.orc_regular_grid.argtypes = [i32, i32, i32, vp, vp, i64]
            L.orc_hierarchize.restype = ctypes.c_int
            L.orc_hierarchize.argtypes = [i32, i64, vp, vp, vp, i32, vp]
            L.orc_hierarchize_stencil.restype = ctypes.c_int
            L.orc_hierarchize_stencil.argtypes = [i32, i64, vp, vp, vp, i32, vp]
            L.orc_build_components.restype = ctypes.c_int
            L.orc_build_components.argtypes = [i32, vp, vp, vp, vp, vp, vp]
            L.orc_grid_free.restype = None
            L.orc_grid_free.argtypes = [vp]
            L.orc_num_threads.restype = ctypes.c_int
            L.orc_num_threads.argtypes = []
            L.orc_set_num_threads.restype = None
            L.orc_set_num_threads.argtypes = [ctypes.c_int]
            _LIB = L
    return _LIB


def num_threads() -> int:
    return lib().orc_num_threads()


def set_num_threads(n: int) -> None:
    """Threads of the oracle's parallel loops from now on (timing only)."""
    lib().orc_set_num_threads(int(n))


# ---------------------------------------------------------------------------
# basis (eq (3.1))
# ---------------------------------------------------------------------------

def hat(l, i, x):
    """phi_{l,i}(x) = max(1 - |x - i 2^-l| / 2^-l, 0), eq (3.1)."""
    return lib().orc_hat(int(l), int(i), float(x))


def dhat(l, i, x):
    """Right derivative of eq (3.1) in [0,1), left derivative at 1, 0 outside."""
    return lib().orc_dhat(int(l), int(i), float(x))


# ---------------------------------------------------------------------------
# model marshalling
# ---------------------------------------------------------------------------

class _Flat:
    """Keeps the flattened numpy arrays alive while C reads them."""

    def __init__(self, model):
        d, m = int(model["d"]), int(model["m"])
        comps = [tuple(int(q) for q in S) for S in model["comps"]]
        self.c0 = np.ascontiguousarray(model["c0"], dtype=np.float64).reshape(m)
        off = np.zeros(len(comps) + 1, dtype=np.int32)
        off[1:] = np.cumsum([len(S) for S in comps])
        self.off = off
        self.dims = np.ascontiguousarray(np.concatenate([np.asarray(S, np.int32) for S in comps])
                                         if comps else np.zeros(1, np.int32), dtype=np.int32)
        self.npts = np.asarray([np.asarray(a).shape[0] for a in model["alpha"]], dtype=np.int64)
        cat = lambda xs, dt: (np.ascontiguousarray(np.concatenate([np.asarray(x, dt).ravel() for x in xs]))
                              if len(xs) else np.zeros(1, dt))
        self.lv = cat(model["levels"], np.uint8)
        self.ix = cat(model["indices"], np.uint32)
        self.al = cat(model["alpha"], np.float64)
        self.w = np.ascontiguousarray(model["weights"], dtype=np.float64)
        s = _Model()
        s.d, s.m, s.ncomp = d, m, len(comps)
        s.c0, s.comp_off, s.comp_dims = self.c0.ctypes.data, self.off.ctypes.data, self.dims.ctypes.data
        s.comp_npts, s.levels, s.indices = self.npts.ctypes.data, self.lv.ctypes.data, self.ix.ctypes.data
        s.alpha, s.weights = self.al.ctypes.data, self.w.ctypes.data
        self.s = s
        self.d, self.m = d, m


def _points(X, d):
    X = np.ascontiguousarray(X, dtype=np.float64)
    if X.ndim != 2 or X.shape[1] != d:
        raise ValueError("points must be (n, %d)" % d)
    return X


def evaluate(model, X, mode="levelwise", with_abs=False):
    """F(x) = c0 + sum_S w_S sum_j alpha_j prod_q phi(x_{S_q}) at every row of X.

    mode 'brute' sums over every stored row (the plain definition, eq (3.6)
    and eq (3.16) per component); 'levelwise' visits one candidate row per
    stored level multi-index (disjoint supports, eq (3.3)).  Returns Y (n, m)
    and, with ``with_abs``, the sum of |terms| (n, m) for error bounds."""
    fl = _Flat(model)
    X = _points(X, fl.d)
    n = X.shape[0]
    Y = np.empty((n, fl.m))
    A = np.empty((n, fl.m)) if with_abs else None
    if mode == "brute":
        rc = lib().orc_eval_brute(ctypes.byref(fl.s), X.ctypes.data, n, Y.ctypes.data,
                                  A.ctypes.data if A is not None else None)
    elif mode == "levelwise":
        rc = lib().orc_eval_levelwise(ctypes.byref(fl.s), X.ctypes.data, n, Y.ctypes.data,
                                      A.ctypes.data if A is not None else None, None)
    else:
        raise ValueError(mode)
    if rc != 0:
        raise RuntimeError("oracle eval failed (%d)" % rc)
    return (Y, A) if with_abs else Y


def gradient(model, X, mode="levelwise"):
    """Values (n, m) and right partial derivatives (n, d, m); left derivative
    at a coordinate equal to 1, zero outside [0,1]."""
    fl = _Flat(model)
    X = _points(X, fl.d)
    n = X.shape[0]
    Y = np.empty((n, fl.m))
    G = np.empty((n, fl.d, fl.m))
    if mode == "brute":
        rc = lib().orc_grad_brute(ctypes.byref(fl.s), X.ctypes.data, n, Y.ctypes.data, G.ctypes.data)
    else:
        rc = lib().orc_eval_levelwise(ctypes.byref(fl.s), X.ctypes.data, n, Y.ctypes.data, None,
                                      G.ctypes.data)
    if rc != 0:
        raise RuntimeError("oracle grad failed (%d)" % rc)
    return Y, G


# ---------------------------------------------------------------------------
# grids and hierarchisation
# ---------------------------------------------------------------------------

def regular_grid(k, ell, rule=1):
    """Points of a k-dimensional regular sparse grid of level ell (rule 1,
    eq (3.5): |l|_1 <= ell + k - 1) or full grid (rule 0, eq (3.4)).
    Returns (levels (N,k) uint8, indices (N,k) uint32)."""
    L = lib()
    n = L.orc_regular_grid(k, ell, rule, None, None, 0)
    if n < 0:
        raise ValueError("bad regular grid arguments")
    lv = np.empty((n, k), np.uint8)
    ix = np.empty((n, k), np.uint32)
    L.orc_regular_grid(k, ell, rule, lv.ctypes.data, ix.ctypes.data, n)
    return lv, ix


def regular_grid_size(k, ell, rule=1):
    return int(lib().orc_regular_grid(k, ell, rule, None, None, 0))


def hierarchize(levels, indices, values, method="triangular"):
    """Surpluses alpha (N, m) whose interpolant equals ``values`` at every node."""
    lv = np.ascontiguousarray(levels, dtype=np.uint8)
    ix = np.ascontiguousarray(indices, dtype=np.uint32)
    Yv = np.ascontiguousarray(values, dtype=np.float64)
    n, k = lv.shape
    m = Yv.shape[1]
    al = np.empty((n, m))
    fn = lib().orc_hierarchize if method == "triangular" else lib().orc_hierarchize_stencil
    rc = fn(k, n, lv.ctypes.data, ix.ctypes.data, Yv.ctypes.data, m, al.ctypes.data)
    if rc != 0:
        raise RuntimeError("hierarchize failed (%d)" % rc)
    return al


def node_coordinates(levels, indices):
    """x_{l,i} = i 2^-l per dimension (exact in FP64)."""
    return np.ldexp(np.asarray(indices, dtype=np.float64), -np.asarray(levels, dtype=np.int64))


# ---------------------------------------------------------------------------
# build (Sec. 3.1 refinement + eq (2.2.6) components + Alg. 2 structure)
# ---------------------------------------------------------------------------

def build_model(comps, d, m, anchor, fn, user=None, max_level=7, level_rule=0, eps_gamma=1e-4,
          refine_rule=0, form="component"):
    """Build one adaptive sparse grid per index set in ``comps``.

    ``fn`` is either a Python callable f(X) -> Y or a pair (c_function_address,
    user_pointer) following ``int f(const double*, int64, int32, double*, int32, void*)``.

    Each grid is refined on the cut function g_S = f(xbar \\ x_S) (Alg. 2) with
    the surplus criterion of eq (3.8).  ``form='component'`` stores the
    surpluses of the cut-HDMR component u_S (eq (2.2.6)) with weight 1 and
    c0 = f(xbar); ``form='paper'`` stores those of g_S with the eq (4.2)
    weights b_S, c0 = b_empty f(xbar).  Returns (model, info) where info holds
    per-component accepted flags."""
    L = lib()
    comps = [tuple(int(q) for q in S) for S in comps]
    anchor = np.ascontiguousarray(anchor, dtype=np.float64)
    off = np.zeros(len(comps) + 1, np.int32)
    off[1:] = np.cumsum([len(S) for S in comps])
    dims = np.ascontiguousarray(np.concatenate([np.asarray(S, np.int32) for S in comps]), dtype=np.int32)
    args = _BuildArgs()
    args.k, args.d, args.m = 0, d, m
    args.max_level, args.level_rule, args.refine_rule = max_level, level_rule, refine_rule
    args.eps_gamma = eps_gamma
    args.dims, args.anchor = None, anchor.ctypes.data
    keep = None
    if callable(fn):
        def _cb(Xp, n, dd, Yp, mm, _user):
            try:
                Xa = np.ctypeslib.as_array(ctypes.cast(Xp, ctypes.POINTER(ctypes.c_double)), shape=(n, dd))
                Ya = np.ctypeslib.as_array(ctypes.cast(Yp, ctypes.POINTER(ctypes.c_double)), shape=(n, mm))
                Ya[...] = fn(Xa.copy())
                return 0
            except Exception:
                return -1
        keep = CALLBACK_T(_cb)
        fptr, uptr = ctypes.cast(keep, ctypes.c_void_p).value, None
    else:
        fptr, uptr = fn
    grids = (_Grid * len(comps))()
    rc = L.orc_build_components(len(comps), off.ctypes.data, dims.ctypes.data, ctypes.byref(args),
                                fptr, uptr, ctypes.cast(grids, ctypes.c_void_p))
    try:
        if rc != 0:
            raise RuntimeError("oracle build failed (%d)" % rc)
        levels, indices, au, ag, acc = [], [], [], [], []
        for s, S in enumerate(comps):
            g = grids[s]
            k, n = len(S), g.n
            levels.append(np.ctypeslib.as_array(ctypes.cast(g.lv, ctypes.POINTER(ctypes.c_uint8)),
                                                shape=(n * k,)).reshape(n, k).copy())
            indices.append(np.ctypeslib.as_array(ctypes.cast(g.ix, ctypes.POINTER(ctypes.c_uint32)),
                                                 shape=(n * k,)).reshape(n, k).copy())
            au.append(np.ctypeslib.as_array(ctypes.cast(g.au, ctypes.POINTER(ctypes.c_double)),
                                            shape=(n * m,)).reshape(n, m).copy())
            ag.append(np.ctypeslib.as_array(ctypes.cast(g.ag, ctypes.POINTER(ctypes.c_double)),
                                            shape=(n * m,)).reshape(n, m).copy())
            acc.append(np.ctypeslib.as_array(ctypes.cast(g.acc, ctypes.POINTER(ctypes.c_uint8)),
                                             shape=(n,)).copy().astype(bool))
    finally:
        for s in range(len(comps)):
            L.orc_grid_free(ctypes.byref(grids[s]))
    f_anchor = _call(fn, anchor[None, :], d, m)[0]
    if form == "component":
        model = {"d": d, "m": m, "c0": f_anchor, "comps": comps, "weights": np.ones(len(comps)),
                 "levels": levels, "indices": indices, "alpha": au}
    elif form == "paper":
        b = paper_coefficients([()] + comps, d)
        model = {"d": d, "m": m, "c0": b[()] * f_anchor, "comps": comps,
                 "weights": np.asarray([float(b[S]) for S in comps]),
                 "levels": levels, "indices": indices, "alpha": ag}
    else:
        raise ValueError(form)
    return model, {"accepted": acc, "alpha_cut": ag, "alpha_component": au, "f_anchor": f_anchor}


def quadrature(model):
    """eq (3.7) per component: Q u_S = sum_j alpha_j prod_q int phi_{l_jq,i_jq}
    = sum_j alpha_j 2^(-|l_j|_1) (the integral of a zero-boundary hat of level
    l over [0,1] is its support's half-width 2^-l).  Returns (ncomp, m)."""
    out = np.zeros((len(model["comps"]), model["m"]))
    for s, (lv, al) in enumerate(zip(model["levels"], model["alpha"])):
        if lv.shape[0]:
            w = np.ldexp(1.0, -lv.astype(np.int64).sum(axis=1))
            out[s] = (w[:, None] * al).sum(axis=0)
    return out


def build_ddsg(d, m, anchor, fn, max_order, eps_eta, eps_rho, comps=None, max_level=7, level_rule=0,
               eps_gamma=1e-4, refine_rule=0, form="component"):
    """Alg. 2: the adaptive DDSG build with the active-dimension criterion
    (eq (3.19)) and the expansion criterion (eq (3.18)).

    Expansion orders k = 1, 2, ... max_order in turn.  The candidates of order
    k are the index sets of size k (all of them, or those of ``comps``) that
    contain no rejected set of Z.  Each candidate's grid is grown on its cut
    function (build_model).  With Q f_u the quadrature (eq (3.7)) of the
    component function's interpolant and Q f_empty = f(xbar), the order's
    denominator is D_k = || sum over retained u with |u| <= k-1 of Q f_u ||_2
    (2-norm over the m outputs).  A candidate of order k >= 2 is kept when
    eta_u = ||Q f_u||_2 / D_k > eps_eta, else it joins Z (order-1 candidates
    are always kept); with eps_eta <= 0 every candidate is kept.  After the
    order, rho_k = || sum over the kept candidates of Q f_u ||_2 / D_k, and the
    build proceeds to order k+1 only if rho_k > eps_rho (eps_rho <= 0: always,
    up to max_order).  Returns (model, report) with the kept components in
    build order, ``form`` as in build_model (the eq (4.2) coefficients over
    the kept family), and the report's candidates, eta, Z and rho."""
    f_anchor = _call(fn, np.asarray(anchor, dtype=np.float64)[None, :], d, m)[0]
    allowed = None if comps is None else {tuple(sorted(S)) for S in comps}
    Z, kept, rho, cands, eta = [], [], [], [], {}
    Qf = {(): f_anchor}
    parts = {"levels": [], "indices": [], "alpha_u": [], "alpha_g": []}
    for k in range(1, max_order + 1):
        C = [c for c in itertools.combinations(range(d), k)
             if (allowed is None or c in allowed) and not any(set(z) <= set(c) for z in Z)]
        if not C:
            break
        model_k, info_k = build_model(C, d, m, anchor, fn, max_level=max_level, level_rule=level_rule,
                                      eps_gamma=eps_gamma, refine_rule=refine_rule, form="component")
        Qk = quadrature(model_k)
        denom = np.linalg.norm(sum(Qf[v] for v in kept + [()] if len(v) <= k - 1))
        keep_k = []
        for s, c in enumerate(C):
            cands.append(c)
            if k >= 2 and eps_eta > 0:
                eta[c] = float(np.linalg.norm(Qk[s]) / denom)
                if not eta[c] > eps_eta:
                    Z.append(c)
                    continue
            keep_k.append(s)
        for s in keep_k:
            Qf[C[s]] = Qk[s]
            kept.append(C[s])
            parts["levels"].append(model_k["levels"][s])
            parts["indices"].append(model_k["indices"][s])
            parts["alpha_u"].append(info_k["alpha_component"][s])
            parts["alpha_g"].append(info_k["alpha_cut"][s])
        r = float(np.linalg.norm(sum((Qk[s] for s in keep_k), np.zeros(m))) / denom)
        rho.append(r)
        if eps_rho > 0 and not r > eps_rho:
            break
    if form == "component":
        model = {"d": d, "m": m, "c0": f_anchor, "comps": kept, "weights": np.ones(len(kept)),
                 "levels": parts["levels"], "indices": parts["indices"], "alpha": parts["alpha_u"]}
    else:
        b = paper_coefficients([()] + kept, d)
        model = {"d": d, "m": m, "c0": b[()] * f_anchor, "comps": kept,
                 "weights": np.asarray([float(b[S]) for S in kept]),
                 "levels": parts["levels"], "indices": parts["indices"], "alpha": parts["alpha_g"]}
    return model, {"candidates": cands, "eta": eta, "Z": Z, "rho": rho, "f_anchor": f_anchor}


def _call(fn, X, d, m):
    if callable(fn):
        return np.asarray(fn(np.ascontiguousarray(X)), dtype=np.float64).reshape(X.shape[0], m)
    f = CALLBACK_T(fn[0])
    X = np.ascontiguousarray(X, dtype=np.float64)
    Y = np.empty((X.shape[0], m))
    if f(X.ctypes.data, X.shape[0], d, Y.ctypes.data, m, fn[1]) != 0:
        raise RuntimeError("callback failed")
    return Y


# ---------------------------------------------------------------------------
# combinatorics of the expansion
# ---------------------------------------------------------------------------

def paper_coefficients(index_sets, d=None):
    """eq (4.2): b_i = sum over retained u containing i of (-1)^(|u|-|i|).

    ``index_sets`` is the retained family (include () for the constant term).
    Returns a dict index-set -> integer coefficient.  Plain double loop over
    the family."""
    fam = [tuple(sorted(S)) for S in index_sets]
    sets = [frozenset(S) for S in fam]
    out = {}
    for S, fs in zip(fam, sets):
        b = 0
        for U, fu in zip(fam, sets):
            if fs <= fu:
                b += (-1) ** (len(fu) - len(fs))
        out[S] = b
    return out


def evaluate_naive(model, X, f_anchor):
    r"""eq (3.16) term by term: sum over the retained index sets u (the
    model's components, plus the empty set) and every v subset u of
    (-1)^(|u|-|v|) times the sparse-grid interpolant of the cut function
    g_v = f(xbar \ x_v), with g_empty = f(xbar) = ``f_anchor`` (m values).
    The model must hold the surpluses of the cut functions g_v (the eq (4.2)
    form of a build) for a family closed under subsets; its weights and c0 are
    not used.  Each g_v is re-evaluated for every u that contains it, as the
    direct implementation of eq (3.16) does."""
    X = np.asarray(X, dtype=np.float64)
    comps = [tuple(S) for S in model["comps"]]
    where = {S: s for s, S in enumerate(comps)}
    f_anchor = np.asarray(f_anchor, dtype=np.float64)

    def g(v):
        if not v:
            return np.broadcast_to(f_anchor, (X.shape[0], model["m"]))
        s = where[v]
        sub = {"d": model["d"], "m": model["m"], "c0": np.zeros(model["m"]), "comps": [v],
               "weights": np.ones(1), "levels": [model["levels"][s]], "indices": [model["indices"][s]],
               "alpha": [model["alpha"][s]]}
        return evaluate(sub, X)

    total = np.zeros((X.shape[0], model["m"]))
    for u in [()] + comps:
        for r in range(len(u) + 1):
            for v in itertools.combinations(u, r):
                if v not in where and v:
                    raise ValueError("index set %r of %r is not retained" % (v, u))
                total = total + ((-1) ** (len(u) - r)) * g(v)
    return total


def cut_hdmr_exact(f, xbar, order, X):
    """Order-K cut-HDMR with exact component functions (eq (2.2.6) inside
    eq (2.2.2) truncated at |u| <= K):
    F_K(x) = sum_{|u|<=K} sum_{v subset u} (-1)^{|u|-|v|} f(xbar \\ x_v).
    Plain loops over index sets; f is vectorised over points."""
    X = np.asarray(X, dtype=np.float64)
    n, d = X.shape
    xbar = np.asarray(xbar, dtype=np.float64)
    total = None
    for k in range(0, order + 1):
        for u in itertools.combinations(range(d), k):
            for r in range(0, k + 1):
                for v in itertools.combinations(u, r):
                    Z = np.tile(xbar, (n, 1))
                    if v:
                        Z[:, list(v)] = X[:, list(v)]
                    term = ((-1) ** (k - r)) * np.asarray(f(Z), dtype=np.float64)
                    total = term if total is None else total + term
    return total


def regular_grid_count(k, ell):
    """|V_{ell,k}| of eq (3.5) for any k: the number of (l, i) with l_q >= 1,
    |l|_1 <= ell + k - 1 and |I_l| = prod 2^(l_q - 1) (eq (3.3)), counted by a
    recursion over the last dimension, N(k, s) = sum_l 2^(l-1) N(k-1, s-l)."""
    top = ell + k - 1
    # N[s] = number of points of a j-dimensional grid with level sum exactly s
    N = [0] * (top + 1)
    for l in range(1, top + 1):
        N[l] = 2 ** (l - 1)
    for _ in range(2, k + 1):
        M = [0] * (top + 1)
        for s in range(top + 1):
            if N[s] == 0:
                continue
            for l in range(1, top - s + 1):
                M[s + l] += N[s] * 2 ** (l - 1)
        N = M
    return sum(N)


def ddsg_point_count(d, ell, order):
    """Number of DDSG grid points sum_{k=1}^{K} |V_{ell,k}| C(d,k) (Sec. 3.3)."""
    return sum(regular_grid_count(k, ell) * math.comb(d, k) for k in range(1, order + 1))
