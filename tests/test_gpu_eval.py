"""GPU parity of hdmr_eval / hdmr_eval_grad (plain FP64 path) against the FP64
oracle on the same seeded inputs, through the C ABI.  Bar: max |GPU - oracle|
<= 1e-12 on values; gradients (slopes up to 2^L) at 1e-12 relative to the
magnitude of the summed terms.  Every case runs on both evaluation kernels:
the point-per-wavefront gather kernel and the cell-sorted matrix-core path
(selected through HDMR_EVAL_PATH)."""
import os

import numpy as np
import pytest

import oracle
import workloads.synth as ws

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def hd():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2202_06555_amd as hd
    hd.hdmr_init(0)
    return hd


@pytest.fixture(autouse=True, params=["gather", "sorted"])
def eval_path(request):
    old = os.environ.get("HDMR_EVAL_PATH")
    os.environ["HDMR_EVAL_PATH"] = request.param
    yield request.param
    if old is None:
        os.environ.pop("HDMR_EVAL_PATH", None)
    else:
        os.environ["HDMR_EVAL_PATH"] = old


def _dev(X):
    import torch
    return torch.from_numpy(np.ascontiguousarray(X)).to("cuda:0")


def _special_points(d, rng, n):
    X = rng.random((n, d))
    X[0] = 0.0
    X[1] = 1.0
    X[2] = 0.5
    X[3:40] = rng.integers(0, 257, size=(37, d)) / 256.0
    X[40:60] = rng.integers(1, 256, size=(20, d)) / 256.0 + 1e-17
    X[60, 0] = -0.25
    X[61, d - 1] = 1.75
    X[62, :] = 1.0 - 1e-17
    return X


def _eval(hd, model, X, **kw):
    gm = hd.hdmr_model_from_surpluses(model)
    Y = hd.hdmr_eval(gm, _dev(X), **kw).cpu().numpy()
    return gm, Y


def test_c1_regular_random_surpluses(hd):
    # d=4, order 2, regular level-4 grids, alpha ~ N(0,1) 2^(-2|l|_1), m=3, 1e4 uniform points
    cfg = ws.config("c1")
    model = ws.synthetic_regular_model(cfg["d"], cfg["m"], cfg["order"], cfg["ell"], cfg["seed"])
    X = ws.points_for(cfg)
    gm, Y = _eval(hd, model, X)
    ref = oracle.evaluate(model, X)
    print("c1 max |err| = %.3e" % np.abs(Y - ref).max())
    assert np.abs(Y - ref).max() <= TOL
    info = hd.hdmr_get_info(gm)
    assert info["n_rows"] == 354 and info["n_components"] == 10


@pytest.mark.parametrize("m", [1, 2, 4, 5, 8, 11, 16, 17, 33, 51, 64, 65, 130, 151, 200, 256])
def test_every_output_width(hd, m):
    # each lanes-per-hit / outputs-per-lane instance, ragged m, special points
    rng = np.random.default_rng(m)
    model = ws.synthetic_regular_model(d=5, m=m, order=2, ell=5, seed=m)
    X = _special_points(5, rng, 333)
    _, Y = _eval(hd, model, X)
    np.testing.assert_allclose(Y, oracle.evaluate(model, X), rtol=0, atol=TOL)


def test_nan_outside_and_empty(hd):
    import torch
    model = ws.synthetic_regular_model(d=4, m=3, order=2, ell=3, seed=2)
    X = np.array([[0.3, np.nan, 0.2, 0.1], [-1.0, 2.0, -3.0, 5.0], [0.3, 0.4, 0.2, 0.1]])
    gm, Y = _eval(hd, model, X)
    ref = oracle.evaluate(model, X)
    assert np.all(np.isnan(Y[0]))
    np.testing.assert_allclose(Y[1:], ref[1:], rtol=0, atol=TOL)
    empty = torch.empty((0, 4), dtype=torch.float64, device="cuda:0")
    assert hd.hdmr_eval(gm, empty).shape == (0, 3)
    with pytest.raises(hd.HdmrError):
        hd.hdmr_eval(gm, _dev(X), values=torch.empty((3, 2), dtype=torch.float64, device="cuda:0"))


def test_adaptive_grids_all_directory_kinds(hd):
    # oracle-built adaptive model (kinked test function): its level multi-indices
    # are stored fully, with slot tables and with hash tables
    cfg = ws.config("c2", d=6, m=7, npairs="all", max_level=9)
    tf = ws.test_function_for(cfg)
    model, _ = oracle.build_model(cfg["comps"], cfg["d"], cfg["m"], cfg["anchor"], (tf.c_fn, tf.c_user),
                                  max_level=9, eps_gamma=1e-4)
    rng = np.random.default_rng(4)
    X = np.vstack([ws.points_for(cfg, n=3000), _special_points(6, rng, 200)])
    _, Y = _eval(hd, model, X)
    np.testing.assert_allclose(Y, oracle.evaluate(model, X), rtol=0, atol=TOL)
    # the paper's eq (4.2) form (integer weights b_S) on the same grids
    modelp, _ = oracle.build_model(cfg["comps"], cfg["d"], cfg["m"], cfg["anchor"], (tf.c_fn, tf.c_user),
                                   max_level=9, eps_gamma=1e-4, form="paper")
    _, Yp = _eval(hd, modelp, X)
    np.testing.assert_allclose(Yp, oracle.evaluate(modelp, X), rtol=0, atol=1e-11)


def test_any_parent_grids_and_three_dim_components(hd):
    cfg = ws.config("c2", d=5, m=3, npairs="all", max_level=6)
    tf = ws.test_function_for(cfg)
    comps = ws.all_components(5, 3)
    model, _ = oracle.build_model(comps, 5, 3, cfg["anchor"], (tf.c_fn, tf.c_user), max_level=6,
                                  eps_gamma=1e-3, refine_rule=1)
    X = ws.points_for(cfg, n=2000)
    _, Y = _eval(hd, model, X)
    np.testing.assert_allclose(Y, oracle.evaluate(model, X), rtol=0, atol=TOL)


def test_gradient_parity(hd):
    rng = np.random.default_rng(6)
    for m, seed in [(3, 0), (20, 1), (70, 2)]:
        model = ws.synthetic_regular_model(d=4, m=m, order=2, ell=5, seed=seed)
        X = _special_points(4, rng, 300)
        X[100, 1] = np.nan
        gm = hd.hdmr_model_from_surpluses(model)
        Y, G = hd.hdmr_eval_grad(gm, _dev(X))
        Y, G = Y.cpu().numpy(), G.cpu().numpy()
        ry, rg = oracle.gradient(model, X, mode="brute")
        ok = ~np.isnan(X).any(axis=1)
        assert np.all(np.isnan(Y[~ok])) and np.all(np.isnan(G[~ok]))
        np.testing.assert_allclose(Y[ok], ry[ok], rtol=0, atol=TOL)
        scale = max(1.0, np.abs(rg[ok]).max())
        np.testing.assert_allclose(G[ok], rg[ok], rtol=0, atol=TOL * scale)


def test_c2_full_size_all_points(hd):
    # d=20, 210 components, adaptive L=7 eps=1e-4, m=11: all 1e6 next-state
    # points against the oracle
    import torch
    import _fullsize as fs
    X = fs.c2_points()
    gm = hd.hdmr_model_from_surpluses(fs.c2_model())
    Y = hd.hdmr_eval(gm, _dev(X))
    torch.cuda.synchronize()
    err = np.abs(Y.cpu().numpy() - fs.c2_reference()).max()
    print("c2 all %d points max |err| = %.3e" % (X.shape[0], err))
    assert err <= TOL


def test_non_dyadic_weights(hd):
    # component weights that are not exact in FP32 (0.1, 1/3, -2.7, ...) on
    # 20000 points (the cell-sorted path's size range) on both kernels, and the
    # mixed path's per-output bar on the same model
    model = ws.synthetic_regular_model(d=5, m=7, order=2, ell=5, seed=9)
    wts = np.array([0.1, 1.0 / 3.0, -2.7, 1e-3, 7.25, -1.0 / 7.0, np.pi, 2.0 ** -30 + 1.0])
    model["weights"] = wts[np.arange(len(model["comps"])) % len(wts)]
    rng = np.random.default_rng(19)
    X = np.vstack([_special_points(5, rng, 200), rng.random((20000, 5))])
    gm, Y = _eval(hd, model, X)
    ref = oracle.evaluate(model, X)
    ok = ~np.isnan(X).any(axis=1)
    err = np.abs(Y[ok] - ref[ok]).max()
    print("non-dyadic weights: max |err| = %.3e" % err)
    assert err <= TOL
    import _fullsize as fs
    Ym = hd.hdmr_eval(gm, _dev(X), precision=hd.MIXED).cpu().numpy()
    rel = fs.per_output_rel(Ym[ok], ref[ok])
    print("non-dyadic weights, mixed: worst per-output %.3e" % rel)
    assert rel <= 1e-6


def test_c2_full_size_gradient_sampled(hd, eval_path):
    # values and gradients at all 1e6 next-state points; values checked at
    # every point, gradients on 1e5 sampled points
    if eval_path == "gather":
        pytest.skip("the full-size gradient runs once, on the path the library picks by size")
    import os
    import torch
    import _fullsize as fs
    os.environ.pop("HDMR_EVAL_PATH", None)
    model = fs.c2_model()
    X = fs.c2_points()
    gm = hd.hdmr_model_from_surpluses(model)
    Y, G = hd.hdmr_eval_grad(gm, _dev(X))
    torch.cuda.synchronize()
    assert np.abs(Y.cpu().numpy() - fs.c2_reference()).max() <= TOL
    idx = fs.sample_rows(X.shape[0], 100_000, 5)
    ry, rg = oracle.gradient(model, X[idx])
    np.testing.assert_allclose(Y.cpu().numpy()[idx], ry, rtol=0, atol=TOL)
    g = G.cpu().numpy()[idx]
    scale = max(1.0, np.abs(rg).max())
    err = np.abs(g - rg).max()
    print("c2 gradient on %d sampled points max |err| = %.3e (scale %.1f)" % (len(idx), err, scale))
    assert err <= TOL * scale


def test_four_dim_components(hd):
    # components of every order up to 4: passes with four key dimensions
    # (4-bit cells, several candidate rows per level multi-index)
    rng = np.random.default_rng(12)
    model = ws.synthetic_regular_model(d=5, m=6, order=4, ell=5, seed=12)
    X = np.vstack([_special_points(5, rng, 200), rng.random((20000, 5))])
    _, Y = _eval(hd, model, X)
    np.testing.assert_allclose(Y, oracle.evaluate(model, X), rtol=0, atol=TOL)
    gm = hd.hdmr_model_from_surpluses(model)
    Ym = hd.hdmr_eval(gm, _dev(X), precision=hd.MIXED).cpu().numpy()
    ref = oracle.evaluate(model, X)
    ok = ~np.isnan(X).any(axis=1)
    import _fullsize as fs
    assert fs.per_output_rel(Ym[ok], ref[ok]) <= 1e-6


@pytest.mark.parametrize("variant", [1, 2, 4, 8, 15])
def test_sorted_tile_shapes(hd, eval_path, variant, monkeypatch):
    """Every tile shape of the cell-sorted path (HDMR_SORTED_VARIANT bits: the
    smaller row batch, work items of half the points, persistent grids of three
    or two workgroups per CU) on a ragged batch with special points: plain at
    1e-12 and mixed at the per-output bar against the oracle."""
    if eval_path != "sorted":
        pytest.skip("tile shapes belong to the cell-sorted path")
    monkeypatch.setenv("HDMR_SORTED_VARIANT", str(variant))
    model = ws.synthetic_regular_model(d=6, m=37, order=2, ell=6, seed=40 + variant)
    rng = np.random.default_rng(variant)
    X = _special_points(6, rng, 20011)
    gm, Y = _eval(hd, model, X)
    ref = oracle.evaluate(model, X)
    assert np.abs(Y - ref).max() <= TOL
    Ym = hd.hdmr_eval(gm, _dev(X), precision=hd.MIXED).cpu().numpy()
    per_output = (np.abs(Ym - ref).max(axis=0) / np.abs(ref).max(axis=0)).max()
    assert per_output <= 1e-6, per_output
