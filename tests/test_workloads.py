"""The seeded input recipes (workloads/synth.py) both sides evaluate on:
determinism, ranges, the component lists of the named configurations and
the clipping fractions of the next-state points stated with the recipe."""
import numpy as np

import workloads.synth as ws


def test_points_are_seeded_and_in_the_unit_cube():
    a = ws.next_state_points(20000, 7, seed=3)
    b = ws.next_state_points(20000, 7, seed=3)
    c = ws.next_state_points(20000, 7, seed=4)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    assert a.min() >= 0.0 and a.max() <= 1.0
    u = ws.uniform_points(1000, 5, seed=1)
    assert np.array_equal(u, ws.uniform_points(1000, 5, seed=1)) and u.min() >= 0.0 and u.max() < 1.0


def test_next_state_clipping_fractions():
    # x' = clip(0.9 x + 0.1 eps): P(x' = 0) = P(eps < -9x) ~ phi(0) / 9 = 0.0443 and
    # P(x' = 1) = P(eps > 10 - 9x) ~ 0.0092 for x ~ U[0,1], eps ~ N(0,1)
    x = ws.next_state_points(200000, 10, seed=0)
    assert abs((x == 0.0).mean() - 0.0443) < 0.002
    assert abs((x == 1.0).mean() - 0.0092) < 0.001


def test_named_configurations():
    c3 = ws.config("c3")
    one = [S for S in c3["comps"] if len(S) == 1]
    two = [S for S in c3["comps"] if len(S) == 2]
    assert len(one) == 100 and len(two) == 500 and len(set(two)) == 500
    assert (0, 1) in two and all(i < j for i, j in two) and two == sorted(two)
    assert np.all(c3["anchor"] == 0.5) and c3["m"] == 51 and c3["n"] == 4_000_000
    assert ws.config("c3")["comps"] == c3["comps"]          # the pair draw is seeded
    c2 = ws.config("c2")
    assert len(c2["comps"]) == 20 + 190
    c5 = ws.config("c5")
    assert len(c5["comps"]) == 600 and c5["m"] == 151


def _closed(lv, ix):
    pts = {(tuple(l), tuple(i)) for l, i in zip(lv.tolist(), ix.tolist())}
    for l, i in pts:
        for q in range(len(l)):
            if l[q] > 1:
                pl, pi = list(l), list(i)
                pl[q] -= 1
                a, b = (i[q] - 1) // 2, (i[q] + 1) // 2
                pi[q] = a if a % 2 else b
                if (tuple(pl), tuple(pi)) not in pts:
                    return False
    return len(pts) == lv.shape[0]


def test_closed_grids():
    # random downward-closed grids: at least the target size, every parent
    # present, odd indices inside their level, deterministic per seed
    for k, target in [(1, 1), (1, 300), (2, 50), (2, 4000)]:
        lv, ix = ws.closed_grid(k, target, seed=target + k)
        assert lv.shape == (target, k) and _closed(lv, ix)
        assert np.all(ix % 2 == 1) and np.all(ix < (1 << lv.astype(np.int64)))
        assert tuple(lv[0]) == (1,) * k and tuple(ix[0]) == (1,) * k
        lv2, ix2 = ws.closed_grid(k, target, seed=target + k)
        assert np.array_equal(lv, lv2) and np.array_equal(ix, ix2)
    # a 1-D grid capped at level 3 holds at most 7 points
    lv, ix = ws.closed_grid(1, 100, seed=1, lcap=3)
    assert lv.shape[0] == 7 and _closed(lv, ix)


def test_batched_workload_shapes():
    # the generator of the 64-model batched workload, d capped for speed here
    for i in (23, 27):
        mo, P = ws.c4_model(i, seed=0, n_range=(10_000, 20_000))
        mo2, P2 = ws.c4_model(i, seed=0, n_range=(10_000, 20_000))
        d, m = mo["d"], mo["m"]
        assert 10 <= d <= 100 and m == d // 2 + 1
        assert len(mo["comps"]) == d + d * (d - 1) // 2
        assert 10_000 <= P.shape[0] <= 20_000 and P.shape[1] == d
        for lv, ix, al in zip(mo["levels"], mo["indices"], mo["alpha"]):
            assert 50 <= lv.shape[0] <= 20_000 and lv.shape == ix.shape and al.shape == (lv.shape[0], m)
        assert _closed(mo["levels"][-1], mo["indices"][-1])
        assert all(np.array_equal(a, b) for a, b in zip(mo["alpha"], mo2["alpha"])) and np.array_equal(P, P2)
