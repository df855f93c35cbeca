"""Pins of the oracle's hierarchisation (eq (3.6) interpolation property)."""
import numpy as np

import oracle


def _random_closed_grid(k, n_target, max_level, rng):
    """Downward-closed grid: start at the root, add admissible children."""
    pts = {(tuple([1] * k), tuple([1] * k))}
    frontier = []

    def parents(l, i):
        out = []
        for q in range(k):
            if l[q] > 1:
                a, b = (i[q] - 1) // 2, (i[q] + 1) // 2
                pl = list(l); pi = list(i)
                pl[q] -= 1; pi[q] = a if a % 2 else b
                out.append((tuple(pl), tuple(pi)))
        return out

    def push_children(l, i):
        for q in range(k):
            if l[q] < max_level:
                for s in (-1, 1):
                    cl = list(l); ci = list(i)
                    cl[q] += 1; ci[q] = 2 * i[q] + s
                    frontier.append((tuple(cl), tuple(ci)))

    push_children(*next(iter(pts)))
    while len(pts) < n_target and frontier:
        j = rng.integers(len(frontier))
        c = frontier.pop(j)
        if c in pts or not all(p in pts for p in parents(*c)):
            continue
        pts.add(c)
        push_children(*c)
    lv = np.array([p[0] for p in sorted(pts)], dtype=np.uint8)
    ix = np.array([p[1] for p in sorted(pts)], dtype=np.uint32)
    return lv, ix


def _interp(lv, ix, al, X):
    k = lv.shape[1]
    model = {"d": k, "m": al.shape[1], "c0": np.zeros(al.shape[1]), "comps": [tuple(range(k))],
             "weights": np.ones(1), "levels": [lv], "indices": [ix], "alpha": [al]}
    return oracle.evaluate(model, X, mode="brute")


def test_interpolation_property_regular_and_adaptive():
    # P3: the interpolant equals the nodal values at every node (defining equations)
    rng = np.random.default_rng(1)
    for k, grid in [(1, oracle.regular_grid(1, 6)), (2, oracle.regular_grid(2, 5)),
                    (3, oracle.regular_grid(3, 4)), (2, _random_closed_grid(2, 300, 7, rng))]:
        lv, ix = grid
        Y = rng.standard_normal((lv.shape[0], 3))
        al = oracle.hierarchize(lv, ix, Y)
        X = oracle.node_coordinates(lv, ix)
        np.testing.assert_allclose(_interp(lv, ix, al, X), Y, rtol=0, atol=1e-13)


def test_stencil_route_matches_triangular_solve():
    # P4(i): classical 1-D stencil hierarchisation == unit-triangular solve
    rng = np.random.default_rng(2)
    for lv, ix in [oracle.regular_grid(2, 5), oracle.regular_grid(3, 4), _random_closed_grid(2, 400, 8, rng),
                   _random_closed_grid(3, 300, 5, rng)]:
        Y = rng.standard_normal((lv.shape[0], 4))
        a1 = oracle.hierarchize(lv, ix, Y)
        a2 = oracle.hierarchize(lv, ix, Y, method="stencil")
        np.testing.assert_allclose(a1, a2, rtol=0, atol=1e-13)


def test_surplus_recovery():
    # P4(ii): seed alpha, form nodal values through the interpolant, recover alpha
    rng = np.random.default_rng(3)
    lv, ix = _random_closed_grid(2, 500, 8, rng)
    al = rng.standard_normal((lv.shape[0], 2)) * np.ldexp(1.0, -2 * lv.astype(int).sum(1))[:, None]
    Y = _interp(lv, ix, al, oracle.node_coordinates(lv, ix))
    np.testing.assert_allclose(oracle.hierarchize(lv, ix, Y), al, rtol=0, atol=1e-14)


def test_one_dimensional_surplus_closed_form():
    # 1-D: alpha_{l,i} = y(x) - (y(x - h) + y(x + h)) / 2 with zero boundary values,
    # checked against an explicitly tabulated function on the full level-4 grid
    lv, ix = oracle.regular_grid(1, 4)
    f = lambda x: x ** 2 * (1 - x)
    Y = f(oracle.node_coordinates(lv, ix))
    al = oracle.hierarchize(lv, ix, Y)
    for (l,), (i,), a in zip(lv, ix, al[:, 0]):
        h = 2.0 ** -int(l)
        x = i * h
        left = f(x - h) if x - h > 0 else 0.0
        right = f(x + h) if x + h < 1 else 0.0
        assert abs(a - (f(x) - 0.5 * (left + right))) < 1e-15
