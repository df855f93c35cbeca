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


def test_batched_models_shapes():
    models, points = ws.batched_models(count=3, seed=0)
    again, _ = ws.batched_models(count=3, seed=0)
    for mo, P, mo2 in zip(models, points, again):
        d, m = mo["d"], mo["m"]
        assert 10 <= d <= 30 and m == d // 2 + 1
        assert len(mo["comps"]) == d + d * (d - 1) // 2
        assert 10_000 <= P.shape[0] <= 100_000 and P.shape[1] == d
        for lv, ix, al in zip(mo["levels"], mo["indices"], mo["alpha"]):
            assert lv.shape == ix.shape and al.shape == (lv.shape[0], m)
        assert all(np.array_equal(a, b) for a, b in zip(mo["alpha"], mo2["alpha"]))
