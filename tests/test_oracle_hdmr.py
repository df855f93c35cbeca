"""Pins of the oracle's cut-HDMR composition (eq (2.2.6), eq (3.16), eq (4.2),
Fig. 3) and of its adaptive build (eq (3.8))."""
import itertools
import math

import numpy as np
import pytest

import oracle
import workloads.synth as ws


def test_fig3_truncation_exact_for_k_at_least_c():
    # Fig. 3: f = (x1+..+x4)^c, anchor 0.5^4, 1e3 random samples: the order-K
    # cut-HDMR with exact components reaches machine precision once K >= c
    rng = np.random.default_rng(0)
    X = rng.random((1000, 4))
    xbar = np.full(4, 0.5)
    for c in (1, 2, 3):
        f = lambda Z, c=c: Z.sum(axis=1, keepdims=True) ** c
        ref = f(X)
        for K in range(1, 5):
            err = np.abs(oracle.cut_hdmr_exact(f, xbar, K, X) - ref).max() / np.abs(ref).max()
            if K >= c:
                assert err < 1e-13
            else:
                assert err > 1e-4


def test_paper_coefficients_closed_form_and_constant_reproduction():
    # eq (4.2) for the full expansion: b_v = sum_{j<=K-|v|} (-1)^j C(d-|v|, j)
    for d, K in [(4, 2), (6, 3), (8, 2)]:
        fam = [()] + [S for k in range(1, K + 1) for S in itertools.combinations(range(d), k)]
        b = oracle.paper_coefficients(fam, d)
        for S in fam:
            assert b[S] == sum((-1) ** j * math.comb(d - len(S), j) for j in range(K - len(S) + 1))
        assert sum(b.values()) == 1     # a constant f is reproduced
    b = oracle.paper_coefficients([()] + [(i,) for i in range(4)] + list(itertools.combinations(range(4), 2)))
    assert (b[()], b[(0,)], b[(0, 1)]) == (3, -2, 1)
    # a pruned family (Fig. 4: {1,2} rejected, so {1,2,3} is never formed)
    fam = [(), (0,), (1,), (2,), (0, 2), (1, 2)]
    b = oracle.paper_coefficients(fam)
    assert sum(b.values()) == 1
    assert b[(2,)] == 1 - 2 and b[(0,)] == 0 and b[()] == 1 - 3 + 2


def test_d100_paper_coefficients():
    # the conditioning figure quoted for d=100, K=2: (4851, -98, 1)
    d, K = 100, 2
    vals = [sum((-1) ** j * math.comb(d - s, j) for j in range(K - s + 1)) for s in range(3)]
    assert vals == [4851, -98, 1]


@pytest.mark.parametrize("form", ["component", "paper"])
def test_telescoping_at_projected_nodes(form):
    # P6: with regular (projection-closed) grids, F(xbar \ x_S) = f(xbar \ x_S)
    # at every node x_S of every component, in both forms (eq (2.2.6) / eq (4.2))
    d, m = 5, 3
    pairs = [(0, 1), (1, 3), (2, 4)]
    tf = ws.TestFunction(d, m, pairs, seed=3)
    comps = ws.all_components(d, 2)
    model, _ = oracle.build_model(comps, d, m, tf.ref, (tf.c_fn, tf.c_user), max_level=4, level_rule=1,
                                  eps_gamma=-1.0, form=form)
    for S, lv, ix in zip(model["comps"], model["levels"], model["indices"]):
        X = np.tile(tf.ref, (lv.shape[0], 1))
        X[:, list(S)] = oracle.node_coordinates(lv, ix)
        np.testing.assert_allclose(oracle.evaluate(model, X), tf(X), rtol=0, atol=1e-12)


def test_anchor_lines_give_exact_zero_surpluses():
    # P4(iii): u_S vanishes on the lines through the anchor, so every stored
    # component surplus with some l_q = 1 is exactly zero
    d, m = 4, 2
    tf = ws.TestFunction(d, m, [(0, 1), (2, 3)], seed=4)
    model, info = oracle.build_model(ws.all_components(d, 2), d, m, tf.ref, (tf.c_fn, tf.c_user),
                                     max_level=5, eps_gamma=1e-3)
    for lv, al in zip(model["levels"], model["alpha"]):
        assert np.all(al[(lv == 1).any(axis=1)] == 0.0)
    assert np.array_equal(model["c0"], tf.c)


def test_adaptive_build_rules():
    # eq (3.8) + Sec. 3.1 exclusion: every stored point other than the root has
    # all its parents stored and accepted (gamma > eps); rejected points have no
    # children; the regular limit (eps < 0) is the regular grid of eq (3.5)/(3.4)
    d, m, L, eps = 3, 2, 6, 2e-3
    tf = ws.TestFunction(d, m, [(0, 1), (1, 2)], seed=5)
    comps = ws.all_components(d, 2)
    model, info = oracle.build_model(comps, d, m, tf.ref, (tf.c_fn, tf.c_user), max_level=L, eps_gamma=eps)
    for S, lv, ix, acc, ag in zip(comps, model["levels"], model["indices"], info["accepted"], info["alpha_cut"]):
        np.testing.assert_array_equal(acc, np.abs(ag).max(axis=1) > eps)
        index = {(tuple(a), tuple(b)): r for r, (a, b) in enumerate(zip(lv.tolist(), ix.tolist()))}
        assert lv.max() <= L
        for (l, i), r in index.items():
            for q in range(len(S)):
                if l[q] > 1:
                    a, b = (i[q] - 1) // 2, (i[q] + 1) // 2
                    pl = list(l); pi = list(i)
                    pl[q] -= 1; pi[q] = a if a % 2 else b
                    pr = index.get((tuple(pl), tuple(pi)))
                    assert pr is not None and acc[pr]
    # regular limit
    for rule, kk in [(1, 2), (0, 2)]:
        model, _ = oracle.build_model([(0, 1)], d, m, tf.ref, (tf.c_fn, tf.c_user), max_level=4,
                                      level_rule=rule, eps_gamma=-1.0)
        lv, ix = oracle.regular_grid(2, 4, rule=rule)
        got = sorted(zip(map(tuple, model["levels"][0].tolist()), map(tuple, model["indices"][0].tolist())))
        want = sorted(zip(map(tuple, lv.tolist()), map(tuple, ix.tolist())))
        assert got == want


def test_any_parent_rule_grows_superset():
    d, m = 2, 2
    tf = ws.TestFunction(d, m, [(0, 1)], seed=6)
    a, _ = oracle.build_model([(0, 1)], d, m, tf.ref, (tf.c_fn, tf.c_user), max_level=6, eps_gamma=1e-3)
    b, _ = oracle.build_model([(0, 1)], d, m, tf.ref, (tf.c_fn, tf.c_user), max_level=6, eps_gamma=1e-3,
                              refine_rule=1)
    sa = set(zip(map(tuple, a["levels"][0].tolist()), map(tuple, a["indices"][0].tolist())))
    sb = set(zip(map(tuple, b["levels"][0].tolist()), map(tuple, b["indices"][0].tolist())))
    assert sa <= sb and len(sb) > len(sa)


def test_test_function_decomposition_recovered():
    # the synthetic function's order-2 cut-HDMR components are its own terms, so
    # the component-form model approximates f up to sparse-grid error only
    cfg = ws.config("c2", d=6, m=4, npairs="all", max_level=7)
    tf = ws.test_function_for(cfg)
    model, _ = oracle.build_model(cfg["comps"], cfg["d"], cfg["m"], cfg["anchor"], (tf.c_fn, tf.c_user),
                                  max_level=7, eps_gamma=1e-5)
    X = ws.points_for(cfg, n=500)
    err = np.abs(oracle.evaluate(model, X) - tf.direct(X)).max()
    assert err < 5e-3
    # incremental and direct evaluation of the test function agree
    Z = np.tile(tf.ref, (50, 1))
    Z[:, 1] = np.linspace(0, 1, 50)
    Z[:, 3] = np.linspace(1, 0, 50)
    np.testing.assert_allclose(tf(Z), tf.direct(Z), rtol=0, atol=1e-13)


def test_naive_eq_3_16_regroups_to_eq_4_2_and_telescopes():
    # eq (3.16) summed term by term equals its regrouping a(x)^T b of eq (4.2)
    # (the same signed terms collected per cut function), and at the nodes of
    # regular (projection-closed) grids on the anchor lines it reproduces f
    # exactly (eq (2.2.6)); a family that is not closed under subsets is refused
    d, m = 5, 3
    pairs = [(0, 1), (1, 3), (2, 4)]
    tf = ws.TestFunction(d, m, pairs, seed=4)
    comps = ws.all_components(d, 2)
    model, info = oracle.build_model(comps, d, m, tf.ref, (tf.c_fn, tf.c_user), max_level=4, level_rule=1,
                                     eps_gamma=-1.0, form="paper")
    rng = np.random.default_rng(8)
    X = rng.random((300, d))
    naive = oracle.evaluate_naive(model, X, info["f_anchor"])
    regrouped, mag = oracle.evaluate(model, X, with_abs=True)
    np.testing.assert_allclose(naive, regrouped, rtol=0, atol=1e-13 * max(1.0, np.abs(mag).max()))
    for S, lv, ix in zip(model["comps"], model["levels"], model["indices"]):
        Xn = np.tile(tf.ref, (lv.shape[0], 1))
        Xn[:, list(S)] = oracle.node_coordinates(lv, ix)
        np.testing.assert_allclose(oracle.evaluate_naive(model, Xn, info["f_anchor"]), tf(Xn), rtol=0, atol=1e-12)
    # a planted mistake: one sign flipped in the term sum breaks the equality
    bad = dict(model)
    bad["alpha"] = list(model["alpha"])
    bad["alpha"][0] = -bad["alpha"][0]
    assert np.abs(oracle.evaluate_naive(bad, X, info["f_anchor"]) - regrouped).max() > 1e-6
    sub = dict(model)
    keep = [s for s, S in enumerate(comps) if S != (1,)]
    for key in ("comps", "levels", "indices", "alpha"):
        sub[key] = [model[key][s] for s in keep]
    with pytest.raises(ValueError):
        oracle.evaluate_naive(sub, X, info["f_anchor"])
