"""Pins of the IRBC oracle (oracle/irbc.py): the monomial rule's exactness
degree against the moments of N(0, I); the deterministic steady state, where
Table 1's A makes every residual vanish in closed form; and the expectation
of a constant policy, whose integrand reduces to the rule applied to a
lognormal with a closed-form value."""
import itertools

import numpy as np

import oracle
from oracle import irbc
import workloads.synth as ws


def _gauss_moment(powers):
    # E[prod e_i^{p_i}] for iid N(0,1): prod (p_i - 1)!! for even p_i, else 0
    out = 1.0
    for p in powers:
        if p % 2:
            return 0.0
        out *= float(np.prod(np.arange(p - 1, 0, -2))) if p else 1.0
    return out


def test_monomial_rule_degree_three():
    for D in (1, 2, 4, 7):
        nodes, w = irbc.monomial_rule(D)
        assert abs(w.sum() - 1.0) < 1e-15
        for deg in range(0, 4):
            for combo in itertools.combinations_with_replacement(range(D), deg):
                powers = np.bincount(np.asarray(combo, dtype=int), minlength=D)
                val = (w * np.prod(nodes ** powers, axis=1)).sum()
                assert abs(val - _gauss_moment(powers)) < 1e-13, (D, combo)
        # not exact at degree 4 when D > 3: E[e^4] = 3, the rule gives D
        val = (w * nodes[:, 0] ** 4).sum()
        assert abs(val - D) < 1e-12


def _constant_policy(N, k1, lam):
    return {"d": 2 * N, "m": N + 1, "c0": np.concatenate([np.full(N, k1), [lam]]), "comps": [],
            "weights": np.zeros(0), "levels": [], "indices": [], "alpha": []}


def test_deterministic_steady_state_residuals_vanish():
    for N in (1, 3):
        p = ws.irbc_params(N, sigma=0.0, gamma_span=0.0)
        A, gam, _ = irbc.constants(p)
        lam = ((A - p["delta"]) / A) ** (-1.0 / gam[0])
        policy = _constant_policy(N, 1.0, lam)
        X = np.full((2, 2 * N), 0.5)             # a = k = 1
        C = np.tile(np.concatenate([np.ones(N), [lam]]), (2, 1))
        R, _ = irbc.residuals(policy, p, X, C)
        np.testing.assert_allclose(R, 0.0, atol=1e-13)


def test_constant_policy_expectation_closed_form():
    # policy constant (k'' = k' = 1, lambda' = L): g'' = 0 and
    # E_j = L (A alpha a_j^rho S + 1 - delta), S = 1 + (2/D)(cosh(sigma sqrt D) - 1)
    # is the rule applied to exp(sigma (e_j + e)) (two nonzero axes per j)
    N, L = 4, 1.7
    p = ws.irbc_params(N, sigma=0.02)
    A, _, _ = irbc.constants(p)
    policy = _constant_policy(N, 1.0, L)
    rng = np.random.default_rng(2)
    X = rng.random((5, 2 * N))
    C = np.concatenate([np.ones((5, N)), np.full((5, 1), 1.3)], axis=1)
    _, E = irbc.residuals(policy, p, X, C)
    D = N + 1
    S = 1.0 + (2.0 / D) * (np.cosh(p["sigma"] * np.sqrt(D)) - 1.0)
    a = p["a_lo"] + X[:, :N] * (p["a_hi"] - p["a_lo"])
    ref = L * (A * p["alpha"] * a ** p["rho"] * S + 1.0 - p["delta"])
    np.testing.assert_allclose(E, ref, rtol=1e-14)


def test_newton_converges_to_the_deterministic_steady_state():
    # from a perturbed start the solve reaches the closed-form steady state
    # (k' = 1, lambda = ((A - delta) / A)^(-1/gamma)) of the deterministic model
    N = 3
    p = ws.irbc_params(N, sigma=0.0, gamma_span=0.0)
    A, gam, _ = irbc.constants(p)
    lam = ((A - p["delta"]) / A) ** (-1.0 / gam[0])
    policy = _constant_policy(N, 1.0, lam)
    X = np.full((3, 2 * N), 0.5)
    x0 = np.tile(np.concatenate([np.ones(N), [lam]]), (3, 1)) * np.array([[1.01], [0.98], [1.003]])
    x, it, worst = irbc.solve(policy, p, X, x0, tol=1e-12)
    assert worst <= 1e-12 and 1 <= it <= 10
    np.testing.assert_allclose(x, np.tile(np.concatenate([np.ones(N), [lam]]), (3, 1)), rtol=1e-10)
    # the steady-state policy has zero Euler errors there
    np.testing.assert_allclose(irbc.euler_errors(policy, p, X), 0.0, atol=1e-14)
