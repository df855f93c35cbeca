"""FP64 oracle of the smooth IRBC model's expectation operator and first-order
conditions (Sec. 2.1, Table 1; eq (model1), eq (model2)), with the previous
policy evaluated by the oracle's own interpolation (``oracle.evaluate``).

TEST INFRASTRUCTURE, like the rest of ``oracle/``: only ``tests/``, the smoke
check and the benchmark's CPU leg may use it, and it shares no code with the
GPU library.

Readings (the paper is silent on them): the state box [a_lo, a_hi]^N x
[k_lo, k_hi]^N is mapped affinely to [0,1]^{2N}; next states are clipped to
the box before the policy is interpolated there, while the integrand uses the
unclipped productivity; the expectation is the degree-3 monomial rule of
Judd's Sec. 7.5 (the rule the paper cites): 2D nodes at +-sqrt(D) on each of
the D = N + 1 shock axes with equal weights."""
import numpy as np

from . import evaluate


def monomial_rule(D):
    """Nodes (2D x D) and weights (2D) of the degree-3 monomial rule for
    E[g(e)], e ~ N(0, I_D): +sqrt(D) along axis i for node i, -sqrt(D) along
    axis i for node D + i, weights 1 / (2D)."""
    r = np.sqrt(float(D))
    nodes = np.vstack([r * np.eye(D), -r * np.eye(D)])
    return nodes, np.full(2 * D, 1.0 / (2 * D))


def constants(p):
    """A (steady-state capital 1 at a = 1) and gamma_j, tau_j of Table 1."""
    N = p["N"]
    A = (1.0 - p["beta"] * (1.0 - p["delta"])) / (p["alpha"] * p["beta"])
    j = np.arange(N)
    gam = p["gamma_lo"] + (p["gamma_span"] * j / (N - 1) if N > 1 else np.zeros(N))
    tau = A ** (1.0 / gam)
    return A, gam, tau


def residuals(policy, p, X, choice):
    """Euler residuals (N) and the resource constraint at states X (n x 2N,
    normalised) for choices (n x (N+1): k_{t+1}, lambda_t); returns
    (R (n x (N+1)), E (n x N)) with E the expectations of the Euler
    conditions.  Plain loops over the quadrature nodes."""
    N = p["N"]
    X = np.asarray(X, dtype=np.float64)
    choice = np.asarray(choice, dtype=np.float64)
    n = X.shape[0]
    A, gam, tau = constants(p)
    aw, kw = p["a_hi"] - p["a_lo"], p["k_hi"] - p["k_lo"]
    a = p["a_lo"] + X[:, :N] * aw
    k = p["k_lo"] + X[:, N:] * kw
    k1 = choice[:, :N]
    lam = choice[:, N]
    g1 = k1 / k - 1.0
    nodes, w = monomial_rule(N + 1)
    E = np.zeros((n, N))
    for q in range(nodes.shape[0]):
        eps = nodes[q]
        a1 = np.exp(p["rho"] * np.log(a) + p["sigma"] * (eps[:N][None, :] + eps[N]))
        Xn = np.empty((n, 2 * N))
        Xn[:, :N] = np.clip((a1 - p["a_lo"]) / aw, 0.0, 1.0)
        Xn[:, N:] = np.clip((k1 - p["k_lo"]) / kw, 0.0, 1.0)
        Pn = evaluate(policy, Xn)
        k2, lam1 = Pn[:, :N], Pn[:, N]
        g2 = k2 / k1 - 1.0
        E += w[q] * lam1[:, None] * (a1 * A * p["alpha"] * k1 ** (p["alpha"] - 1.0) + (1.0 - p["delta"])
                                     + 0.5 * p["phi"] * g2 * (g2 + 2.0))
    R = np.empty((n, N + 1))
    R[:, :N] = lam[:, None] * (1.0 + p["phi"] * g1) - p["beta"] * E
    cons = (lam[:, None] / tau[None, :]) ** (-gam[None, :])
    R[:, N] = (a * A * k ** p["alpha"] + k * ((1.0 - p["delta"]) - 0.5 * p["phi"] * g1 ** 2) - k1 - cons).sum(axis=1)
    return R, E


def solve(policy, p, X, x0, max_iter=30, tol=1e-11, rel=1e-7):
    """Newton on the first-order conditions per state: forward-difference
    Jacobian (unknown i raised by rel max(1, |x_i|)), the linear systems solved
    by numpy.linalg.solve, states whose largest |residual| is <= tol left as
    they are.  Returns (x, updates made, largest |residual| at exit)."""
    x = np.array(x0, dtype=np.float64, copy=True)
    n, M = x.shape
    it = 0
    while True:
        R, _ = residuals(policy, p, X, x)
        worst = np.abs(R).max(axis=1)
        if np.all(worst <= tol) or it >= max_iter:
            return x, it, float(worst.max())
        J = np.empty((n, M, M))
        for i in range(M):
            h = rel * np.maximum(1.0, np.abs(x[:, i]))
            xp = x.copy()
            xp[:, i] += h
            Ri, _ = residuals(policy, p, X, xp)
            J[:, :, i] = (Ri - R) / h[:, None]
        dx = np.linalg.solve(J, -R[:, :, None])[:, :, 0]
        act = worst > tol
        x[act] += dx[act]
        it += 1


def euler_errors(policy, p, X):
    """Unit-free Euler-equation errors of a policy (its own choice at X, the
    same policy next period): |R_j| / |lambda (1 + phi g_j)| per country and
    |R_N| / sum_j c_j for the resource constraint."""
    N = p["N"]
    C = evaluate(policy, X)
    R, _ = residuals(policy, p, X, C)
    A, gam, tau = constants(p)
    k = p["k_lo"] + np.asarray(X)[:, N:] * (p["k_hi"] - p["k_lo"])
    g1 = C[:, :N] / k - 1.0
    lam = C[:, N]
    err = np.empty_like(R)
    err[:, :N] = np.abs(R[:, :N]) / np.abs(lam[:, None] * (1.0 + p["phi"] * g1))
    err[:, N] = np.abs(R[:, N]) / ((lam[:, None] / tau[None, :]) ** (-gam[None, :])).sum(axis=1)
    return err
