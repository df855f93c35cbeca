"""Pins of the oracle's evaluation and gradient: brute force vs level-wise,
exact reproduction of hat-span and additive functions, finite differences."""
import itertools

import numpy as np
import pytest

import oracle
import workloads.synth as ws


def _special_points(d, rng, n=64):
    X = rng.random((n, d))
    X[0] = 0.0
    X[1] = 1.0
    X[2] = 0.5
    X[3:12] = rng.integers(0, 17, size=(9, d)) / 16.0            # nodes and cell edges
    X[12:16] = rng.integers(1, 64, size=(4, d)) / 64.0 + 1e-17   # just right of edges
    X[16, 0] = -0.25                                             # outside the domain
    X[17, d - 1] = 1.75
    return X


def test_bruteforce_equals_levelwise_values_and_grads():
    # P10 + gradients: two independent evaluation routes agree on tiny models,
    # including points at 0, 1, nodes, cell edges and outside [0,1]
    rng = np.random.default_rng(11)
    model = ws.synthetic_regular_model(d=4, m=3, order=2, ell=4, seed=0)
    X = _special_points(4, rng)
    Yb, Ab = oracle.evaluate(model, X, mode="brute", with_abs=True)
    Yl, Al = oracle.evaluate(model, X, mode="levelwise", with_abs=True)
    np.testing.assert_allclose(Yb, Yl, rtol=0, atol=1e-14)
    np.testing.assert_allclose(Ab, Al, rtol=1e-14, atol=1e-14)
    Yg, Gb = oracle.gradient(model, X, mode="brute")
    Yg2, Gl = oracle.gradient(model, X, mode="levelwise")
    np.testing.assert_allclose(Yg, Yb, rtol=0, atol=1e-14)
    np.testing.assert_allclose(Gb, Gl, rtol=0, atol=1e-12)


def test_nan_and_outside_rules():
    model = ws.synthetic_regular_model(d=4, m=3, order=2, ell=3, seed=1)
    X = np.array([[0.3, np.nan, 0.2, 0.1], [-1.0, 2.0, -3.0, 5.0], [0.3, 0.4, 0.2, 0.1]])
    for mode in ("brute", "levelwise"):
        Y = oracle.evaluate(model, X, mode=mode)
        assert np.all(np.isnan(Y[0]))
        np.testing.assert_array_equal(Y[1], model["c0"])   # zero extension outside [0,1]
        assert np.all(np.isfinite(Y[2]))


def _hat_np(l, i, x):
    return np.maximum(0.0, 1.0 - np.abs(x * 2.0 ** l - i))


def test_hat_span_reproduction():
    # P5: f = c + sum_S h_S with h_S in the hat span of a regular grid and zero
    # surpluses wherever some l_q = 1 (so h_S vanishes on the anchor lines):
    # the order-2 build on regular grids reproduces f at arbitrary points.
    d, m, ell = 4, 2, 4
    rng = np.random.default_rng(7)
    comps = ws.all_components(d, 2)
    terms = []
    for S in comps:
        lv, ix = oracle.regular_grid(len(S), ell)
        beta = rng.standard_normal((lv.shape[0], m))
        beta[(lv == 1).any(axis=1)] = 0.0
        terms.append((S, lv, ix, beta))
    c = rng.standard_normal(m)

    def f(X):
        out = np.tile(c, (X.shape[0], 1))
        for S, lv, ix, beta in terms:
            for row in range(lv.shape[0]):
                w = np.ones(X.shape[0])
                for q, dim in enumerate(S):
                    w = w * _hat_np(int(lv[row, q]), int(ix[row, q]), X[:, dim])
                out += w[:, None] * beta[row]
        return out

    model, _ = oracle.build_model(comps, d, m, np.full(d, 0.5), f, max_level=ell, level_rule=1,
                                  eps_gamma=-1.0)
    X = rng.random((300, d))
    np.testing.assert_allclose(oracle.evaluate(model, X), f(X), rtol=0, atol=1e-13)


def test_additive_recovery_order_one():
    # P7: f = c + sum_i h_i(x_i), h_i in the 1-D hat span.  With h_i(0.5) = 0
    # the order-1 model is exact everywhere; otherwise exact on the interior
    # box [2^-L, 1 - 2^-L]^d (the zero-boundary cells are the only loss).
    d, m, L = 5, 3, 6
    rng = np.random.default_rng(8)
    lv, ix = oracle.regular_grid(1, 5)
    for vanish in (True, False):
        beta = rng.standard_normal((d, lv.shape[0], m))
        if vanish:
            beta[:, (lv[:, 0] == 1)] = 0.0
        c = rng.standard_normal(m)

        def f(X):
            out = np.tile(c, (X.shape[0], 1))
            for dim in range(d):
                for row in range(lv.shape[0]):
                    out += _hat_np(int(lv[row, 0]), int(ix[row, 0]), X[:, dim])[:, None] * beta[dim, row]
            return out

        model, _ = oracle.build_model([(q,) for q in range(d)], d, m, np.full(d, 0.5), f, max_level=L,
                                      level_rule=0, eps_gamma=-1.0)
        X = rng.random((400, d))
        if not vanish:
            X = 2.0 ** -L + (1 - 2.0 ** (1 - L)) * X
        np.testing.assert_allclose(oracle.evaluate(model, X), f(X), rtol=0, atol=1e-13)
    # and the boundary cells do lose the constant part when h_i(0.5) != 0
    Xb = np.full((1, d), 0.5)
    Xb[0, 0] = 0.0
    assert np.abs(oracle.evaluate(model, Xb) - f(Xb)).max() > 1e-3


def test_gradient_central_differences():
    # P11: inside cells F is multilinear, so central differences with a step far
    # below the finest cell width match the right derivative to ~1e-9
    rng = np.random.default_rng(9)
    model = ws.synthetic_regular_model(d=3, m=2, order=2, ell=5, seed=3)
    X = rng.random((40, 3))
    finest = 2.0 ** -6
    X = (np.floor(X / finest) + 0.25 + 0.5 * rng.random(X.shape)) * finest   # away from edges
    _, G = oracle.gradient(model, X, mode="brute")
    h = 1e-7
    for q in range(3):
        Xp, Xm = X.copy(), X.copy()
        Xp[:, q] += h
        Xm[:, q] -= h
        fd = (oracle.evaluate(model, Xp) - oracle.evaluate(model, Xm)) / (2 * h)
        np.testing.assert_allclose(G[:, q, :], fd, rtol=0, atol=1e-7)


def test_gradient_at_edges_is_right_derivative():
    # at a cell edge the gradient is the one-sided slope to the right; at x=1 the left one
    model = ws.synthetic_regular_model(d=2, m=1, order=1, ell=4, seed=4)
    for x0 in (0.0, 0.25, 0.5, 0.8125, 1.0):
        X = np.array([[x0, 0.3]])
        _, G = oracle.gradient(model, X, mode="brute")
        h = 1e-9
        if x0 < 1.0:
            one_sided = (oracle.evaluate(model, X + [[h, 0]]) - oracle.evaluate(model, X)) / h
        else:
            one_sided = (oracle.evaluate(model, X) - oracle.evaluate(model, X - [[h, 0]])) / h
        np.testing.assert_allclose(G[:, 0, :], one_sided, rtol=0, atol=1e-5)


def test_summed_magnitudes_closed_form():
    # Yabs = |c0| + sum_S sum_j |w_S alpha_j phi_j(x)|: with every surplus,
    # weight and c0 of one sign the terms cannot cancel, so Yabs = |F|
    # exactly (up to rounding) in both modes; with mixed signs Yabs >= |F|
    # and Yabs - |F| is twice the mass of the minority-sign terms, checked
    # against a direct sum of positive and negative parts.
    rng = np.random.default_rng(31)
    model = ws.synthetic_regular_model(d=4, m=3, order=2, ell=4, seed=31)
    X = np.vstack([_special_points(4, rng), rng.random((500, 4))])
    ok = ~np.isnan(X).any(axis=1)
    for sign in (1.0, -1.0):
        mdl = dict(model)
        mdl["alpha"] = [sign * np.abs(a) for a in model["alpha"]]
        mdl["c0"] = sign * np.abs(model["c0"])
        mdl["weights"] = np.full(len(model["comps"]), 0.75)
        for mode in ("brute", "levelwise"):
            Y, A = oracle.evaluate(mdl, X, mode=mode, with_abs=True)
            np.testing.assert_allclose(A[ok], np.abs(Y[ok]), rtol=1e-14, atol=1e-15)
    # mixed signs: positive and negative parts evaluated as separate models
    pos, neg = dict(model), dict(model)
    pos["alpha"] = [np.maximum(a, 0.0) for a in model["alpha"]]
    neg["alpha"] = [np.minimum(a, 0.0) for a in model["alpha"]]
    pos["c0"] = np.maximum(model["c0"], 0.0)
    neg["c0"] = np.minimum(model["c0"], 0.0)
    Yp = oracle.evaluate(pos, X)
    Yn = oracle.evaluate(neg, X)
    _, A = oracle.evaluate(model, X, with_abs=True)
    np.testing.assert_allclose(A[ok], Yp[ok] - Yn[ok], rtol=1e-13, atol=1e-15)
