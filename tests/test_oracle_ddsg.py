"""Pins of the oracle's quadrature (eq (3.7)) and of its adaptive DDSG build
(Alg. 2: active-dimension criterion eq (3.19) with the reject set Z, expansion
criterion eq (3.18)), against facts that do not come from the oracle: exact
integrals of piecewise-(bi)linear interpolants by a midpoint rule finer than
their finest level, and closed-form eta / rho / Z for functions whose cut-HDMR
component functions lie in the hat span of the grids."""
import itertools

import numpy as np

import oracle
import workloads.synth as ws


def _hat(l, i, x):
    return np.maximum(0.0, 1.0 - np.abs(np.asarray(x) * 2.0 ** l - i))


def test_quadrature_equals_midpoint_integral():
    # P12: int phi_{l,i} = 2^-l, int of a tensor basis function = 2^-|l|_1; a
    # midpoint rule on cells of width 2^-(L+1) integrates every interpolant of
    # level <= L exactly (linear, resp. bilinear, on every cell)
    model = ws.synthetic_regular_model(d=3, m=2, order=2, ell=5, seed=4)
    Q = oracle.quadrature(model)
    L = 5
    h = 2.0 ** -(L + 1)
    mid = (np.arange(2 ** (L + 1)) + 0.5) * h
    for s, S in enumerate(model["comps"]):
        sub = {"d": 3, "m": 2, "c0": np.zeros(2), "comps": [S], "weights": np.ones(1),
               "levels": [model["levels"][s]], "indices": [model["indices"][s]], "alpha": [model["alpha"][s]]}
        grids = np.meshgrid(*([mid] * len(S)), indexing="ij")
        X = np.full((grids[0].size, 3), 0.5)
        for q, g in zip(S, grids):
            X[:, q] = g.ravel()
        integral = oracle.evaluate(sub, X).sum(axis=0) * h ** len(S)
        np.testing.assert_allclose(Q[s], integral, rtol=1e-13, atol=1e-16)
    # one basis function alone: 2^-|l|_1
    one = {"d": 2, "m": 1, "c0": np.zeros(1), "comps": [(0, 1)], "weights": np.ones(1),
           "levels": [np.array([[3, 2]], np.uint8)], "indices": [np.array([[5, 1]], np.uint32)],
           "alpha": [np.ones((1, 1))]}
    assert oracle.quadrature(one)[0, 0] == 2.0 ** -5


class _Separable:
    """f(x) = c + h1(x0) + h2(x1) + beta p(x0) q(x1) on [0,1]^4 (two outputs),
    h1, h2, p, q sums of hats of levels 2..4 (all vanish at the anchor 0.5),
    so the component functions are u_0 = h1, u_1 = h2, u_01 = beta p q and
    every other component function is zero."""

    def __init__(self, beta):
        self.c = np.array([1.25, -0.8])
        self.beta = np.asarray(beta, dtype=np.float64)
        self.h1 = [(2, 1, [0.3, -0.2]), (3, 5, [0.1, 0.05]), (4, 3, [-0.07, 0.02])]
        self.h2 = [(2, 3, [-0.4, 0.25]), (4, 11, [0.06, -0.03])]
        self.p = [(2, 1, 1.0), (3, 7, -0.5)]
        self.q = [(3, 3, 0.8), (4, 13, 0.3)]

    @staticmethod
    def _eval(terms, x, vec):
        out = np.zeros((x.shape[0], 2)) if vec else np.zeros(x.shape[0])
        for l, i, c in terms:
            v = _hat(l, i, x)
            out = out + (v[:, None] * np.asarray(c) if vec else v * c)
        return out

    @staticmethod
    def _int(terms):
        return sum(np.asarray(c, dtype=np.float64) * 2.0 ** -l for l, _, c in terms)

    def __call__(self, X):
        X = np.atleast_2d(X)
        pq = self._eval(self.p, X[:, 0], False) * self._eval(self.q, X[:, 1], False)
        return (self.c + self._eval(self.h1, X[:, 0], True) + self._eval(self.h2, X[:, 1], True)
                + pq[:, None] * self.beta)

    def closed_forms(self):
        q1, q2 = self._int(self.h1), self._int(self.h2)
        q12 = self.beta * self._int(self.p) * self._int(self.q)
        d1 = np.linalg.norm(self.c)
        d2 = np.linalg.norm(self.c + q1 + q2)
        return {"rho1": np.linalg.norm(q1 + q2) / d1, "eta01": np.linalg.norm(q12) / d2,
                "rho2": np.linalg.norm(q12) / d2, "q": {(0,): q1, (1,): q2, (0, 1): q12}}


def test_ddsg_eta_rho_and_reject_set_closed_forms():
    f = _Separable(beta=[0.5, -0.3])
    cf = f.closed_forms()
    kw = dict(max_level=4, level_rule=0, eps_gamma=-1.0)
    model, rep = oracle.build_ddsg(4, 2, np.full(4, 0.5), f, max_order=3, eps_eta=1e-8, eps_rho=1e-12, **kw)
    # order 1: all four kept; rho_1 closed form
    np.testing.assert_allclose(rep["rho"][0], cf["rho1"], rtol=1e-12)
    # order 2: only (0, 1) has a nonzero component function
    np.testing.assert_allclose(rep["eta"][(0, 1)], cf["eta01"], rtol=1e-12)
    for c in itertools.combinations(range(4), 2):
        if c != (0, 1):
            assert rep["eta"][c] < 1e-14
    assert sorted(rep["Z"]) == [c for c in itertools.combinations(range(4), 2) if c != (0, 1)]
    np.testing.assert_allclose(rep["rho"][1], cf["rho2"], rtol=1e-12)
    # order 3: every triple contains a rejected pair, so there are no candidates
    assert len(rep["rho"]) == 2
    assert model["comps"] == [(0,), (1,), (2,), (3,), (0, 1)]
    Q = oracle.quadrature(model)
    for s, S in enumerate(model["comps"]):
        if S in cf["q"]:
            np.testing.assert_allclose(Q[s], cf["q"][S], rtol=1e-12, atol=1e-15)
    # the kept expansion reproduces f at arbitrary points (hat-span components)
    X = np.random.default_rng(3).random((200, 4))
    np.testing.assert_allclose(oracle.evaluate(model, X), f(X), rtol=0, atol=1e-13)
    # eq (4.2) form of the same kept family: b over the kept sets plus the empty set
    pmodel, _ = oracle.build_ddsg(4, 2, np.full(4, 0.5), f, max_order=3, eps_eta=1e-8, eps_rho=1e-12, form="paper",
                                  **kw)
    b = oracle.paper_coefficients([()] + model["comps"], 4)
    assert list(pmodel["weights"]) == [float(b[S]) for S in model["comps"]]
    # the two forms are different approximants under the zero-boundary basis;
    # they agree with f at the grid nodes on the anchor lines (eq (2.2.6))
    for S, lv, ix in zip(pmodel["comps"], pmodel["levels"], pmodel["indices"]):
        Xn = np.full((lv.shape[0], 4), 0.5)
        Xn[:, list(S)] = oracle.node_coordinates(lv, ix)
        np.testing.assert_allclose(oracle.evaluate(pmodel, Xn), f(Xn), rtol=0, atol=1e-12)


def test_ddsg_expansion_criterion_stops_and_eta_threshold_is_strict():
    f = _Separable(beta=[0.5, -0.3])
    cf = f.closed_forms()
    kw = dict(max_level=4, level_rule=0, eps_gamma=-1.0)
    # rho_1 below the threshold: no order-2 candidates are built
    model, rep = oracle.build_ddsg(4, 2, np.full(4, 0.5), f, max_order=3, eps_eta=0.0, eps_rho=cf["rho1"] * 1.01,
                                   **kw)
    assert len(rep["rho"]) == 1 and model["comps"] == [(0,), (1,), (2,), (3,)]
    # eta exactly at the threshold is rejected (strict), just below is kept
    _, rep = oracle.build_ddsg(4, 2, np.full(4, 0.5), f, max_order=2, eps_eta=rep_eta(cf), eps_rho=0.0, **kw)
    assert (0, 1) in rep["Z"]
    model, rep = oracle.build_ddsg(4, 2, np.full(4, 0.5), f, max_order=2, eps_eta=rep_eta(cf) * (1 - 1e-9),
                                   eps_rho=0.0, **kw)
    assert (0, 1) not in rep["Z"] and (0, 1) in model["comps"]
    # no criteria: the full order-2 expansion
    model, rep = oracle.build_ddsg(4, 2, np.full(4, 0.5), f, max_order=2, eps_eta=0.0, eps_rho=0.0, **kw)
    assert len(model["comps"]) == 4 + 6 and rep["Z"] == []


def rep_eta(cf):
    # the oracle's own eta of (0, 1) for this function equals the closed form
    # to rounding; the strict test uses the closed form's value itself
    f = _Separable(beta=[0.5, -0.3])
    _, rep = oracle.build_ddsg(4, 2, np.full(4, 0.5), f, max_order=2, eps_eta=1e-30, eps_rho=0.0, max_level=4,
                               level_rule=0, eps_gamma=-1.0)
    np.testing.assert_allclose(rep["eta"][(0, 1)], cf["eta01"], rtol=1e-12)
    return rep["eta"][(0, 1)]
