"""Seeded input generators shared by the CPU oracle and the GPU path.

Everything here is input: evaluation points, the shapes and random surpluses
of synthetic models, and the synthetic test function that the builds
approximate.  Random streams are numpy ``default_rng`` (PCG64) with fixed
seeds and a fixed draw order, stated per generator.

Model interchange format (a plain dict, consumed independently by the oracle
and by the GPU binding):

    d, m      : input dimension and number of outputs
    c0        : (m,) float64 constant term
    comps     : list of tuples of distinct input dimensions (the index set S
                of each component function)
    weights   : (ncomp,) float64 weight of each component in the sum
    levels    : list of (N_S, |S|) uint8 level multi-indices, l >= 1
    indices   : list of (N_S, |S|) uint32 odd index multi-indices, 0 < i < 2^l
    alpha     : list of (N_S, m) float64 coefficient rows
"""
from __future__ import annotations

import ctypes
import itertools
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libtestfn.so")
_LOCK = threading.Lock()
_LIB = None


def build_testfn(force: bool = True) -> str:
    """Compile the C test function with gcc (OpenMP) into workloads/libtestfn.so."""
    srcs = [os.path.join(_HERE, "testfn.c"), os.path.join(_HERE, "gridgen.c")]
    if force or not os.path.exists(_SO) or any(os.path.getmtime(_SO) < os.path.getmtime(s) for s in srcs):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-o", tmp] + srcs + ["-lm"])
        os.replace(tmp, _SO)
    return _SO


def _lib():
    global _LIB
    with _LOCK:
        if _LIB is None:
            if not os.path.exists(_SO):
                build_testfn(force=False)
            lib = ctypes.CDLL(_SO)
            lib.tf_prepare.restype = ctypes.c_int
            lib.tf_prepare.argtypes = [ctypes.c_void_p]
            lib.tf_release.restype = None
            lib.tf_release.argtypes = [ctypes.c_void_p]
            lib.gg_closed_grid.restype = ctypes.c_int64
            lib.gg_closed_grid.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64,
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]
            for nm in ("tf_eval", "tf_eval_direct"):
                fn = getattr(lib, nm)
                fn.restype = ctypes.c_int
                fn.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                               ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]
            _LIB = lib
    return _LIB


class _TFParams(ctypes.Structure):
    _fields_ = [
        ("d", ctypes.c_int32), ("m", ctypes.c_int32), ("npairs", ctypes.c_int32),
        ("kink_a", ctypes.c_int32), ("kink_b", ctypes.c_int32),
        ("ref", ctypes.c_void_p), ("c", ctypes.c_void_p), ("a", ctypes.c_void_p),
        ("theta", ctypes.c_void_p), ("pairs", ctypes.c_void_p), ("b", ctypes.c_void_p),
        ("mu", ctypes.c_void_p), ("nu", ctypes.c_void_p), ("kappa", ctypes.c_void_p),
        ("f_ref", ctypes.c_void_p), ("dp_off", ctypes.c_void_p), ("dp_idx", ctypes.c_void_p),
    ]


# C signature shared by every host callback in this project:
#   int f(const double* X, int64 n, int32 d, double* Y, int32 m, void* user)
CALLBACK_T = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                              ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p)


class TestFunction:
    """Seeded smooth-plus-kink test function f : [0,1]^d -> R^m (see testfn.c).

    Each term vanishes on the boundary and on the lines through ``ref``, so
    f(ref) = c and the cut-HDMR components anchored at ``ref`` are the terms.

    Draw order from ``default_rng(seed)``: c (m), a (m x d), theta (m x d),
    b (m x P), mu (m x P), nu (m x P), kappa (m).  Distributions: c ~ U[0.5,1.5],
    a ~ N(0, 0.5^2), theta ~ U[0, 2 pi], b ~ N(0, 0.3^2), mu, nu ~ U[0,1],
    kappa ~ U[0.5, 1]; ``pair_scale`` multiplies b and kappa after the draws
    (order-2 terms smaller than order-1 terms).  ``pairs`` is the interaction
    pair set; the kink sits on dimensions (0, 1).  ``ref`` is the reference point of the incremental path
    (the anchor of the cut-HDMR builds).
    """

    __test__ = False  # not a pytest class

    def __init__(self, d, m, pairs, seed, ref=None, kink=(0, 1), pair_scale=1.0):
        rng = np.random.default_rng(seed)
        self.d, self.m = int(d), int(m)
        self.pairs = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
        P = self.pairs.shape[0]
        self.c = rng.uniform(0.5, 1.5, size=m)
        self.a = rng.normal(0.0, 0.5, size=(m, d))
        self.theta = rng.uniform(0.0, 2 * np.pi, size=(m, d))
        self.b = rng.normal(0.0, 0.3, size=(m, P))
        self.mu = rng.uniform(0.0, 1.0, size=(m, P))
        self.nu = rng.uniform(0.0, 1.0, size=(m, P))
        self.kappa = rng.uniform(0.5, 1.0, size=m)
        # optional scale of every order-2 term (pairs and kink), after the draws
        self.b *= pair_scale
        self.kappa *= pair_scale
        self.ref = np.full(d, 0.5) if ref is None else np.ascontiguousarray(ref, dtype=np.float64)
        self.kink = tuple(int(k) for k in kink)
        p = _TFParams()
        p.d, p.m, p.npairs = self.d, self.m, P
        p.kink_a, p.kink_b = self.kink
        for nm in ("ref", "c", "a", "theta", "b", "mu", "nu", "kappa"):
            arr = np.ascontiguousarray(getattr(self, nm), dtype=np.float64)
            setattr(self, nm, arr)
            setattr(p, nm, arr.ctypes.data)
        p.pairs = self.pairs.ctypes.data
        self._p = p
        rc = _lib().tf_prepare(ctypes.byref(p))
        if rc != 0:
            raise RuntimeError("tf_prepare failed (%d)" % rc)

    def __del__(self):
        try:
            if _LIB is not None:
                _LIB.tf_release(ctypes.byref(self._p))
        except Exception:
            pass

    # -- C entry points for native builds (no Python in the callback loop) --
    @property
    def c_fn(self) -> int:
        """Address of the C evaluator ``tf_eval`` (callback signature above)."""
        return ctypes.cast(_lib().tf_eval, ctypes.c_void_p).value

    @property
    def c_user(self) -> int:
        """``user`` pointer to pass alongside :pyattr:`c_fn`."""
        return ctypes.addressof(self._p)

    def _call(self, fn, X):
        X = np.ascontiguousarray(X, dtype=np.float64)
        if X.ndim != 2 or X.shape[1] != self.d:
            raise ValueError("X must be (n, %d)" % self.d)
        Y = np.empty((X.shape[0], self.m))
        rc = fn(X.ctypes.data, X.shape[0], self.d, Y.ctypes.data, self.m, ctypes.addressof(self._p))
        if rc != 0:
            raise RuntimeError("test function failed (%d)" % rc)
        return Y

    def __call__(self, X):
        return self._call(_lib().tf_eval, X)

    def direct(self, X):
        """Evaluation without the incremental path."""
        return self._call(_lib().tf_eval_direct, X)


# --------------------------------------------------------------------------
# evaluation points
# --------------------------------------------------------------------------

def uniform_points(n, d, seed):
    """n points uniform on [0,1]^d from default_rng(seed), row-major (n, d)."""
    return np.random.default_rng(seed).random((n, d))


def next_state_points(n, d, seed):
    """Quadrature next-state points x' = clip(0.9 x + 0.1 eps, 0, 1) with
    x ~ U[0,1]^d from default_rng(seed) and eps ~ N(0, I) from
    default_rng(seed + 1)."""
    x = np.random.default_rng(seed).random((n, d))
    eps = np.random.default_rng(seed + 1).standard_normal((n, d))
    return np.clip(0.9 * x + 0.1 * eps, 0.0, 1.0)


def random_pairs(d, npairs, seed, include=(0, 1)):
    """``npairs`` distinct pairs (i < j) of range(d): ``include`` first, the rest
    drawn without replacement from default_rng(seed) in lexicographic-pair
    numbering, then sorted lexicographically."""
    allp = [(i, j) for i in range(d) for j in range(i + 1, d)]
    inc = tuple(sorted(include))
    rest = [p for p in allp if p != inc]
    rng = np.random.default_rng(seed)
    pick = rng.choice(len(rest), size=npairs - 1, replace=False)
    out = sorted([inc] + [rest[i] for i in pick])
    return out


# --------------------------------------------------------------------------
# synthetic models with random coefficients
# --------------------------------------------------------------------------

def regular_levels(k, ell):
    """Level multi-indices of a k-dimensional regular sparse grid of level ell
    (|l|_1 <= ell + k - 1, every l_q >= 1), ordered by |l|_1 then
    lexicographically, with the odd index multi-indices of each level in
    lexicographic order.  Returns (levels (N,k) uint8, indices (N,k) uint32)."""
    lv, ix = [], []
    top = ell + k - 1
    for s in range(k, top + 1):
        tuples = [t for t in itertools.product(range(1, s + 1), repeat=k) if sum(t) == s]
        for t in sorted(tuples):
            ranges = [range(1, 2 ** lq, 2) for lq in t]
            for ii in itertools.product(*ranges):
                lv.append(t)
                ix.append(ii)
    return np.asarray(lv, dtype=np.uint8).reshape(-1, k), np.asarray(ix, dtype=np.uint32).reshape(-1, k)


def all_components(d, order):
    """All index sets 1 <= |S| <= order of range(d), ordered by |S| then lexicographically."""
    out = []
    for k in range(1, order + 1):
        out.extend(itertools.combinations(range(d), k))
    return out


def synthetic_regular_model(d, m, order, ell, seed):
    """Model with regular sparse-grid components of level ``ell`` for all index
    sets of size <= order and random coefficients alpha ~ N(0,1) 2^(-2|l|_1).

    Draw order from default_rng(seed): c0 (m values), then per component in
    (|S|, lexicographic) order, per grid point in (|l|_1, l, i) order, m values.
    All weights are 1."""
    rng = np.random.default_rng(seed)
    c0 = rng.standard_normal(m)
    comps = all_components(d, order)
    levels, indices, alpha = [], [], []
    for S in comps:
        lv, ix = regular_levels(len(S), ell)
        z = rng.standard_normal((lv.shape[0], m))
        scale = np.ldexp(1.0, -2 * lv.astype(np.int64).sum(axis=1))
        levels.append(lv)
        indices.append(ix)
        alpha.append(z * scale[:, None])
    return {"d": d, "m": m, "c0": c0, "comps": comps, "weights": np.ones(len(comps)),
            "levels": levels, "indices": indices, "alpha": alpha}


def mlp_init_params(d, width, m, seed):
    """Initial parameters of the surrogate network, packed [W0, b0, ..., W3, b3]
    in FP32 with W_l (out x in) row-major: W ~ U(-1/sqrt(in), 1/sqrt(in)) drawn
    from default_rng(seed) in layer order, biases zero."""
    rng = np.random.default_rng(seed)
    dims = [d, width, width, width, m]
    parts = []
    for l in range(4):
        a = 1.0 / np.sqrt(dims[l])
        parts.append(rng.uniform(-a, a, size=(dims[l + 1], dims[l])).astype(np.float32).ravel())
        parts.append(np.zeros(dims[l + 1], np.float32))
    return np.concatenate(parts)


_REGULAR_CACHE = {}


def _regular_cached(k, ell):
    key = (k, ell)
    if key not in _REGULAR_CACHE:
        _REGULAR_CACHE[key] = regular_levels(k, ell)
    return _REGULAR_CACHE[key]


def regular_grid_size(k, ell):
    """Points of a k-dimensional regular sparse grid of level ell."""
    return _regular_cached(k, ell)[0].shape[0]


# --------------------------------------------------------------------------
# named workload configurations
# --------------------------------------------------------------------------

CONFIGS = {
    # d=4, order 2, regular level-4 grids, random surpluses, m=3, 1e4 uniform points
    "c1": dict(kind="random_regular", d=4, m=3, order=2, ell=4, n=10_000, seed=0, points="uniform"),
    # d=20, all 20+190 components, adaptive L=7 eps=1e-4, m=11, 1e6 next-state points
    "c2": dict(kind="testfn", d=20, m=11, npairs="all", max_level=7, eps_gamma=1e-4,
               n=1_000_000, seed=0, points="next_state"),
    # d=100, 100 one-dim + 500 two-dim components, adaptive L=8 eps=1e-4, m=51, 4e6 points
    "c3": dict(kind="testfn", d=100, m=51, npairs=500, max_level=8, eps_gamma=1e-4,
               n=4_000_000, seed=0, points="next_state"),
    # d=300, 300 one-dim + 300 two-dim components, adaptive L=7 eps=1e-4, m=151
    "c5": dict(kind="testfn", d=300, m=151, npairs=300, max_level=7, eps_gamma=1e-4,
               n=10_000_000, seed=0, points="next_state"),
}


def config(name, **over):
    """Return a resolved configuration: points generator, component list, test
    function (for adaptive configs) or synthetic model (for random ones)."""
    cfg = dict(CONFIGS[name])
    cfg.update(over)
    d, m = cfg["d"], cfg["m"]
    if cfg["kind"] == "testfn":
        if cfg["npairs"] == "all":
            pairs = [(i, j) for i in range(d) for j in range(i + 1, d)]
        else:
            pairs = random_pairs(d, int(cfg["npairs"]), cfg["seed"])
        cfg["pairs"] = pairs
        cfg["comps"] = [(i,) for i in range(d)] + [tuple(p) for p in pairs]
        cfg["anchor"] = np.full(d, 0.5)
    return cfg


def points_for(cfg, n=None, seed=None):
    n = cfg["n"] if n is None else n
    seed = cfg["seed"] if seed is None else seed
    if cfg["points"] == "uniform":
        return uniform_points(n, cfg["d"], seed)
    return next_state_points(n, cfg["d"], seed)


def test_function_for(cfg):
    return TestFunction(cfg["d"], cfg["m"], cfg["pairs"], cfg["seed"], ref=cfg["anchor"])


# --------------------------------------------------------------------------
# smooth IRBC workload (Sec. 2.1, Table 1)
# --------------------------------------------------------------------------

def irbc_params(N, sigma=0.01, gamma_span=0.75):
    """Table 1 of the paper for N countries, with the readings used here:
    gamma_j = 0.25 + 0.75 (j - 1) / (N - 1) (the table's lower end is garbled;
    0.25 gives the usual range [0.25, 1]) and the state box
    a in [0.8, 1.2]^N, k in [0.8, 1.2]^N."""
    return dict(N=int(N), beta=0.99, alpha=0.36, delta=0.01, sigma=float(sigma), rho=0.95, phi=0.5,
                gamma_lo=0.25, gamma_span=float(gamma_span), a_lo=0.8, a_hi=1.2, k_lo=0.8, k_hi=1.2)


class IrbcGuess:
    """A smooth synthetic policy (k_{t+1}, lambda_t) over the normalised state
    box, the stand-in for a previous time-iteration iterate (the paper
    publishes no policies):
      k'_j   = k_j (1 - 0.01) + 0.01 + 0.05 (a_j - 1) + 0.02 (a_j - 1)(k_j - 1)
      lambda = 1.2 (1 - 0.3 mean_j (a_j - 1) + 0.2 mean_j (k_j - 1)),
    with a_j, k_j the box coordinates of x (a = 0.8 + 0.4 x_j, k = 0.8 + 0.4
    x_{N+j}).  Its cut-HDMR components are the one-dimensional ones and the
    pairs (j, N + j)."""

    def __init__(self, N):
        self.N = int(N)
        self.d, self.m = 2 * self.N, self.N + 1
        self.anchor = np.full(self.d, 0.5)

    def components(self):
        return [(q,) for q in range(self.d)] + [(j, self.N + j) for j in range(self.N)]

    def __call__(self, X):
        X = np.atleast_2d(np.asarray(X, dtype=np.float64))
        N = self.N
        a = 0.8 + 0.4 * X[:, :N]
        k = 0.8 + 0.4 * X[:, N:]
        Y = np.empty((X.shape[0], N + 1))
        Y[:, :N] = k * 0.99 + 0.01 + 0.05 * (a - 1.0) + 0.02 * (a - 1.0) * (k - 1.0)
        Y[:, N] = 1.2 * (1.0 - 0.3 * (a - 1.0).mean(axis=1) + 0.2 * (k - 1.0).mean(axis=1))
        return Y


def irbc_states(n, N, seed):
    """n states uniform on the normalised box [0,1]^{2N} and choices near the
    synthetic policy there (k' and lambda scaled by 1 + 0.02 u, u ~ U[-1,1])."""
    rng = np.random.default_rng(seed)
    X = rng.random((n, 2 * N))
    C = IrbcGuess(N)(X) * (1.0 + 0.02 * rng.uniform(-1.0, 1.0, size=(n, N + 1)))
    return X, C


# --------------------------------------------------------------------------
# batched workload at its stated shape
# --------------------------------------------------------------------------

def closed_grid(k, target, seed, lcap=16):
    """A random downward-closed grid of a k-dimensional component with at
    least ``target`` points (gridgen.c): (levels (n x k) uint8, indices
    (n x k) uint32) in the order the points were added."""
    cap = int(target)
    lv = np.zeros((cap, k), np.uint8)
    ix = np.zeros((cap, k), np.uint32)
    n = _lib().gg_closed_grid(int(k), int(target), int(lcap), int(seed) & ((1 << 64) - 1), lv.ctypes.data,
                              ix.ctypes.data, cap)
    if n < 0:
        raise RuntimeError("grid generation failed")
    return lv[:n].copy(), ix[:n].copy()


def c4_model(i, seed=0, d_range=(10, 100), size_range=(50, 20000), n_range=(10_000, 1_000_000), max_d=None):
    """Model i of the batched workload: draws from default_rng(seed + i)
    d ~ U{d_range} (capped at max_d if given), m = d // 2 + 1, c0 ~ N(0,1)^m;
    then per component (all d one-dimensional and all C(d,2) two-dimensional
    index sets, in (|S|, lexicographic) order) a target size
    N ~ logU(size_range), a random downward-closed grid of at least N points
    (closed_grid with a seed drawn from the same generator, levels <= 16) and
    alpha ~ N(0,1) 2^(-2|l|_1) per grid point; then n ~ logU(n_range) points
    uniform on [0,1]^d.  Returns (model, points)."""
    rng = np.random.default_rng(seed + i)
    d = int(rng.integers(d_range[0], d_range[1] + 1))
    if max_d is not None:
        d = min(d, int(max_d))
    m = d // 2 + 1
    c0 = rng.standard_normal(m)
    comps = all_components(d, 2)
    levels, indices, alpha = [], [], []
    for S in comps:
        k = len(S)
        target = int(np.ceil(np.exp(rng.uniform(np.log(size_range[0]), np.log(size_range[1])))))
        lv, ix = closed_grid(k, target, int(rng.integers(0, 2 ** 63)))
        z = rng.standard_normal((lv.shape[0], m))
        levels.append(lv)
        indices.append(ix)
        alpha.append(z * np.ldexp(1.0, -2 * lv.astype(np.int64).sum(axis=1))[:, None])
    n = int(np.exp(rng.uniform(np.log(n_range[0]), np.log(n_range[1]))))
    model = {"d": d, "m": m, "c0": c0, "comps": comps, "weights": np.ones(len(comps)),
             "levels": levels, "indices": indices, "alpha": alpha}
    return model, rng.random((n, d))
