"""GPU parity of the smooth IRBC expectation operator and first-order
conditions (irbc_residuals, include/hdmr_irbc.h) against the FP64 oracle
(oracle/irbc.py), through the C ABI.  Both sides evaluate the previous policy
in FP64 (the GPU through hdmr_eval's kernels), so residuals and expectations
are held to 1e-12 relative to their magnitude (1e-13 absolute where the closed
form is zero)."""
import numpy as np
import pytest

import oracle
from oracle import irbc as oirbc
import workloads.synth as ws

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2202_06555_amd as hd
    from paper_2202_06555_amd import irbc
    hd.hdmr_init(0)
    return hd, irbc


def _dev(X):
    import torch
    return torch.from_numpy(np.ascontiguousarray(X)).to("cuda:0")


def _policy(hd, N, max_level, eps_gamma):
    g = ws.IrbcGuess(N)
    kw = dict(comps=g.components(), max_level=max_level, eps_gamma=eps_gamma)
    gm = hd.asg_build_components(g.d, g.m, g.anchor, g, **kw)
    model, _ = oracle.build_model(g.components(), g.d, g.m, g.anchor, g, max_level=max_level, eps_gamma=eps_gamma)
    return gm, model


def _run(env, gm, p, X, C):
    import torch
    hd, irbc = env
    N = p["N"]
    E = torch.empty((X.shape[0], N), dtype=torch.float64, device="cuda:0")
    R, E = irbc.irbc_residuals(gm, p, _dev(X), _dev(C), expect=E)
    torch.cuda.synchronize()
    return R.cpu().numpy(), E.cpu().numpy()


@pytest.mark.parametrize("N", [1, 3])
def test_residuals_match_oracle_small(env, N):
    hd, _ = env
    p = ws.irbc_params(N)
    gm, model = _policy(hd, N, max_level=6, eps_gamma=1e-6)
    X, C = ws.irbc_states(3000, N, seed=N)
    X[0] = 0.0
    X[1] = 1.0
    R, E = _run(env, gm, p, X, C)
    Ro, Eo = oirbc.residuals(model, p, X, C)
    np.testing.assert_allclose(E, Eo, rtol=1e-12, atol=0)
    np.testing.assert_allclose(R, Ro, rtol=0, atol=1e-12 * max(1.0, np.abs(Eo).max()))


def test_steady_state_closed_form(env):
    hd, _ = env
    N = 3
    p = ws.irbc_params(N, sigma=0.0, gamma_span=0.0)
    A, gam, _ = oirbc.constants(p)
    lam = ((A - p["delta"]) / A) ** (-1.0 / gam[0])
    const = {"d": 2 * N, "m": N + 1, "c0": np.concatenate([np.ones(N), [lam]]), "comps": [],
             "weights": np.zeros(0), "levels": [], "indices": [], "alpha": []}
    gm = hd.hdmr_model_from_surpluses(const)
    X = np.full((4, 2 * N), 0.5)
    C = np.tile(np.concatenate([np.ones(N), [lam]]), (4, 1))
    R, _ = _run(env, gm, p, X, C)
    np.testing.assert_allclose(R, 0.0, atol=1e-13)


def test_residuals_d100_policy_sampled(env):
    # N = 50 countries (d = 100, m = 51): 20000 states, 2.04e6 next states
    # through the cell-sorted evaluation; 100 states checked against the oracle
    hd, irbc = env
    N = 50
    p = ws.irbc_params(N)
    gm, model = _policy(hd, N, max_level=7, eps_gamma=1e-5)
    X, C = ws.irbc_states(20000, N, seed=7)
    R, E = _run(env, gm, p, X, C)
    idx = np.arange(0, 20000, 200)
    Ro, Eo = oirbc.residuals(model, p, X[idx], C[idx])
    err = np.abs(R[idx] - Ro).max()
    print("irbc N=50: max |residual err| %.3e, max |E err| %.3e" % (err, np.abs(E[idx] - Eo).max()))
    np.testing.assert_allclose(E[idx], Eo, rtol=1e-12, atol=0)
    np.testing.assert_allclose(R[idx], Ro, rtol=0, atol=1e-12 * max(1.0, np.abs(Eo).max()))


def test_shape_errors(env):
    hd, irbc = env
    gm, _ = _policy(hd, 2, max_level=3, eps_gamma=1e-3)
    X, C = ws.irbc_states(10, 2, seed=1)
    with pytest.raises(hd.HdmrError):
        irbc.irbc_residuals(gm, ws.irbc_params(3), _dev(np.zeros((10, 6))), _dev(np.zeros((10, 4))))
    bad = ws.irbc_params(2)
    bad["a_hi"] = bad["a_lo"]
    with pytest.raises(hd.HdmrError):
        irbc.irbc_residuals(gm, bad, _dev(X), _dev(C))


def test_newton_solve_matches_oracle(env):
    # the batched device Newton and the oracle's Newton reach the same roots
    hd, irbc = env
    import torch
    N = 3
    p = ws.irbc_params(N)
    gm, model = _policy(hd, N, max_level=6, eps_gamma=1e-6)
    # interior states: near the box edges k' can leave the box, where the
    # clipped interpolation has a kink and Newton stalls (on both sides alike)
    X, _ = ws.irbc_states(400, N, seed=21)
    X = 0.2 + 0.6 * X
    x0 = oracle.evaluate(model, X)
    xd = _dev(x0)
    _, it, worst = irbc.irbc_solve(gm, p, _dev(X), xd, max_iter=20, tol=1e-11)
    torch.cuda.synchronize()
    xo, ito, worsto = oirbc.solve(model, p, X, x0, max_iter=20, tol=1e-11)
    print("newton: device %d iterations (max |R| %.2e), oracle %d (%.2e)" % (it, worst, ito, worsto))
    assert worst <= 1e-11 and worsto <= 1e-11
    np.testing.assert_allclose(xd.cpu().numpy(), xo, rtol=1e-9, atol=1e-10)
    # the device iterate satisfies the oracle's residuals
    Ro, _ = oirbc.residuals(model, p, X, xd.cpu().numpy())
    assert np.abs(Ro).max() <= 1e-10


def test_steady_state_solve_closed_form(env):
    hd, irbc = env
    import torch
    N = 2
    p = ws.irbc_params(N, sigma=0.0, gamma_span=0.0)
    A, gam, _ = oirbc.constants(p)
    lam = ((A - p["delta"]) / A) ** (-1.0 / gam[0])
    const = {"d": 2 * N, "m": N + 1, "c0": np.concatenate([np.ones(N), [lam]]), "comps": [],
             "weights": np.zeros(0), "levels": [], "indices": [], "alpha": []}
    gm = hd.hdmr_model_from_surpluses(const)
    X = np.full((3, 2 * N), 0.5)
    ss = np.tile(np.concatenate([np.ones(N), [lam]]), (3, 1))
    xd = _dev(ss * np.array([[1.02], [0.97], [1.001]]))
    _, it, worst = irbc.irbc_solve(gm, p, _dev(X), xd, tol=1e-12)
    torch.cuda.synchronize()
    assert worst <= 1e-12
    np.testing.assert_allclose(xd.cpu().numpy(), ss, rtol=1e-10)


def test_time_step_and_euler_errors(env):
    # one time-iteration step (Alg. 1) from the synthetic policy, N = 2
    # (d = 4, m = 3): the device step (build whose function is the device
    # Newton) against the oracle step (oracle build whose function is the
    # oracle Newton on the oracle's previous policy); then the Euler errors of
    # the new policy on 2000 states
    hd, irbc = env
    import torch
    N = 2
    p = ws.irbc_params(N)
    g = ws.IrbcGuess(N)
    comps = g.components()
    gm_prev, model_prev = _policy(hd, N, max_level=5, eps_gamma=1e-5)
    gm_new, it, worst = irbc.irbc_time_step(gm_prev, p, comps, max_level=4, eps_gamma=1e-5, max_iter=20, tol=1e-11)
    assert worst <= 1e-11

    def oracle_solver(X):
        x, _, w = oirbc.solve(model_prev, p, X, oracle.evaluate(model_prev, X), max_iter=20, tol=1e-11)
        assert w <= 1e-11
        return x

    model_new, _ = oracle.build_model(comps, 2 * N, N + 1, g.anchor, oracle_solver, max_level=4, eps_gamma=1e-5)
    assert hd.hdmr_get_info(gm_new)["n_rows"] == sum(lv.shape[0] for lv in model_new["levels"])
    X, _ = ws.irbc_states(2000, N, seed=31)
    Y = hd.hdmr_eval(gm_new, _dev(X)).cpu().numpy()
    np.testing.assert_allclose(Y, oracle.evaluate(model_new, X), rtol=0, atol=1e-9)
    err = irbc.irbc_euler_errors(gm_new, p, _dev(X)).cpu().numpy()
    err_o = oirbc.euler_errors(model_new, p, X)
    print("time step: %d Newton iterations; Euler errors log10 mean %.2f, max %.2f" %
          (it, np.log10(err[:, :N]).mean(), np.log10(err[:, :N].max())))
    np.testing.assert_allclose(err, err_o, rtol=1e-6, atol=1e-12)
