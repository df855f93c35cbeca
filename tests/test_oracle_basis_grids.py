"""Pins of the oracle's basis and grid generators against values the paper
and the mathematics fix (eq (3.1), eq (3.3), eq (3.5), Table 2, Sec. 3.3)."""
import math

import numpy as np
import pytest

import oracle
import workloads.synth as ws
from conftest import golden


def test_hat_golden_values():
    # hand-computed eq (3.1) values and one-sided slopes, tests/golden/hat_values.txt
    for l, i, x, phi, dphi in golden("hat_values.txt"):
        assert oracle.hat(int(l), int(i), float(x)) == pytest.approx(float(phi), abs=1e-15)
        assert oracle.dhat(int(l), int(i), float(x)) == float(dphi)


def test_hat_nodes_and_disjoint_supports():
    # eq (3.1): phi_{l,i}(x_{l,i}) = 1; finer hats vanish at coarser nodes;
    # eq (3.3): at any x at most one odd i of a level is nonzero.
    rng = np.random.default_rng(5)
    for l in range(1, 9):
        for i in range(1, 2 ** l, 2):
            assert oracle.hat(l, i, i / 2 ** l) == 1.0
            for lc in range(1, l):
                for ic in range(1, 2 ** lc, 2):
                    assert oracle.hat(l, i, ic / 2 ** lc) == 0.0
        for x in rng.random(50):
            nz = [i for i in range(1, 2 ** l, 2) if oracle.hat(l, i, x) > 0]
            assert len(nz) <= 1
    assert oracle.hat(3, 3, 0.0) == 0.0 and oracle.hat(3, 7, 1.0) == 0.0


def test_regular_grid_sizes_closed_form():
    # |V_{ell,k}| = sum_{n<ell} 2^n C(n+k-1, k-1) for eq (3.5); 2-D: 1,5,17,49,...
    for k in range(1, 5):
        for ell in range(1, 8):
            cf = sum(2 ** n * math.comb(n + k - 1, k - 1) for n in range(ell))
            assert oracle.regular_grid_size(k, ell) == cf
            assert oracle.regular_grid_count(k, ell) == cf
    assert [oracle.regular_grid_size(2, l) for l in range(1, 9)] == [1, 5, 17, 49, 129, 321, 769, 1793]
    assert oracle.regular_grid_size(1, 7) == 2 ** 7 - 1
    # full grid of eq (3.4): (2^ell - 1)^k points
    assert oracle.regular_grid_size(2, 5, rule=0) == 31 ** 2


def test_table2_sg_points():
    # Table 2 (Sec. 5.3), SG* column of the smooth rows: printed with 2 digits
    for d, ell, printed in golden("table2_sg_points.txt"):
        n = oracle.regular_grid_count(int(d), int(ell))
        e = math.floor(math.log10(n)) - 1
        # the table shows two digits, rounded (1.394e6 -> 1.4e6) or cut (3.654e7 -> 3.6e7)
        assert float(printed) in (round(n / 10 ** e) * 10 ** e, math.floor(n / 10 ** e) * 10 ** e)
    assert oracle.regular_grid_count(100, 4) == 1_394_001


def test_regular_grid_point_set():
    # enumerated points: odd indices, 0 < i < 2^l, |l|_1 <= ell+k-1, no duplicates
    for k, ell in [(1, 5), (2, 4), (3, 3)]:
        lv, ix = oracle.regular_grid(k, ell)
        assert np.all(lv >= 1) and np.all(ix % 2 == 1)
        assert np.all(ix < (1 << lv.astype(np.int64)))
        assert np.all(lv.astype(int).sum(axis=1) <= ell + k - 1)
        keys = {(tuple(a), tuple(b)) for a, b in zip(lv, ix)}
        assert len(keys) == lv.shape[0]
        glv, gix = ws.regular_levels(k, ell)  # the input generator's own enumeration
        assert np.array_equal(glv, lv) and np.array_equal(gix, ix)


def test_ddsg_point_counts_fig6():
    # Sec. 3.3 count sum_k |V_{ell,k}| C(d,k); Fig. 6 ratio SG/DDSG at d=100, ell=4
    sg = oracle.regular_grid_count(100, 4)
    r = [sg / oracle.ddsg_point_count(100, 4, K) for K in (1, 2, 3)]
    assert r[0] > 1 and r[1] > 1 and r[2] < 1      # reduction up to K=2 only (Sec. 5.1.1)
    assert oracle.ddsg_point_count(100, 4, 1) == 15 * 100
    assert oracle.ddsg_point_count(100, 4, 2) == 15 * 100 + 49 * 4950
