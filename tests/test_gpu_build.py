"""GPU parity of asg_build_components against the oracle build (same seeded
test function, same parameters): identical grid point sets (bit-exact, they
are integer data), surpluses within 1e-12, identical weights and c0; and the
full-size metric workload (d=100, m=51, 4e6 points) evaluated in the
benchmark's launch configuration (plain and mixed precision), checked on
sampled outputs."""
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


def _sorted_rows(lv, ix, al):
    keys = [tuple(a) + tuple(b) for a, b in zip(lv.tolist(), ix.tolist())]
    order = sorted(range(len(keys)), key=lambda r: keys[r])
    return [keys[r] for r in order], al[order]


def _compare_models(hd, gm, model, tol=TOL):
    info = hd.hdmr_get_info(gm)
    assert info["n_components"] == len(model["comps"])
    np.testing.assert_array_equal(model["c0"], _c0_of(hd, gm, model))
    worst = 0.0
    for s, S in enumerate(model["comps"]):
        dims, lv, ix, al, w = hd.hdmr_export_component(gm, s)
        assert dims == tuple(S)
        assert w == model["weights"][s]
        gk, ga = _sorted_rows(lv, ix, al)
        ok, oa = _sorted_rows(model["levels"][s], model["indices"][s], model["alpha"][s])
        assert gk == ok, "grid points of component %s differ" % (S,)
        worst = max(worst, float(np.abs(ga - oa).max()) if len(ga) else 0.0)
    assert worst <= tol, worst
    return worst


def _c0_of(hd, gm, model):
    # c0 is what the model returns at a point where every basis function vanishes
    import torch
    X = torch.zeros((1, model["d"]), dtype=torch.float64, device="cuda:0")
    return hd.hdmr_eval(gm, X).cpu().numpy()[0]


@pytest.mark.parametrize("refine_rule", [0, 1])
def test_adaptive_build_matches_oracle(hd, refine_rule):
    cfg = ws.config("c2", d=6, m=5, npairs="all", max_level=8)
    tf = ws.test_function_for(cfg)
    kw = dict(max_level=8, eps_gamma=1e-4, refine_rule=refine_rule)
    model, _ = oracle.build_model(cfg["comps"], 6, 5, cfg["anchor"], (tf.c_fn, tf.c_user), **kw)
    gm = hd.asg_build_components(6, 5, cfg["anchor"], (tf.c_fn, tf.c_user), comps=cfg["comps"], **kw)
    _compare_models(hd, gm, model)


@pytest.mark.parametrize("level_rule", [0, 1])
def test_regular_limit_and_three_dim_components(hd, level_rule):
    d, m = 4, 3
    tf = ws.TestFunction(d, m, [(0, 1), (1, 2), (2, 3)], seed=7)
    comps = ws.all_components(d, 3)
    kw = dict(max_level=4, level_rule=level_rule, eps_gamma=-1.0)
    model, _ = oracle.build_model(comps, d, m, tf.ref, (tf.c_fn, tf.c_user), **kw)
    gm = hd.asg_build_components(d, m, tf.ref, (tf.c_fn, tf.c_user), max_order=3, **kw)
    _compare_models(hd, gm, model)


def test_paper_form_weights_and_values(hd):
    import torch
    d, m = 5, 4
    tf = ws.TestFunction(d, m, [(0, 1), (2, 4)], seed=8)
    comps = ws.all_components(d, 2)
    kw = dict(max_level=6, eps_gamma=1e-3)
    model, _ = oracle.build_model(comps, d, m, tf.ref, (tf.c_fn, tf.c_user), form="paper", **kw)
    gm = hd.asg_build_components(d, m, tf.ref, (tf.c_fn, tf.c_user), comps=comps, form=1, **kw)
    _compare_models(hd, gm, model)
    X = ws.uniform_points(500, d, seed=3)
    Y = hd.hdmr_eval(gm, torch.from_numpy(X).to("cuda:0")).cpu().numpy()
    np.testing.assert_allclose(Y, oracle.evaluate(model, X), rtol=0, atol=1e-11)


def test_python_callback_and_errors(hd):
    d, m = 3, 2
    tf = ws.TestFunction(d, m, [(0, 1)], seed=9)
    comps = ws.all_components(d, 2)
    model, _ = oracle.build_model(comps, d, m, tf.ref, tf, max_level=5, eps_gamma=1e-3)
    gm = hd.asg_build_components(d, m, tf.ref, tf, comps=comps, max_level=5, eps_gamma=1e-3)
    _compare_models(hd, gm, model)

    def bad(X):
        raise ValueError("boom")

    with pytest.raises(hd.HdmrError) as e:
        hd.asg_build_components(d, m, tf.ref, bad, comps=comps, max_level=3)
    assert e.value.code == hd.hdmr.HDMR_ECALLBACK
    with pytest.raises(hd.HdmrError):
        hd.asg_build_components(d, m, tf.ref, tf, comps=[(1, 0)], max_level=3)


def test_c2_full_build(hd):
    cfg = ws.config("c2")
    tf = ws.test_function_for(cfg)
    kw = dict(max_level=cfg["max_level"], eps_gamma=cfg["eps_gamma"])
    model, _ = oracle.build_model(cfg["comps"], cfg["d"], cfg["m"], cfg["anchor"], (tf.c_fn, tf.c_user), **kw)
    gm = hd.asg_build_components(cfg["d"], cfg["m"], cfg["anchor"], (tf.c_fn, tf.c_user), comps=cfg["comps"], **kw)
    w = _compare_models(hd, gm, model)
    print("c2 build: %d rows, max |surplus diff| = %.3e" % (hd.hdmr_get_info(gm)["n_rows"], w))


def test_c3_full_size_build_and_eval(hd):
    """The metric workload at full size: d=100, 100 + 500 components, L=8,
    eps=1e-4, m=51; 4e6 next-state points through the plain FP64 kernel in the
    benchmark's launch configuration; 2000 sampled points plus the first and
    last rows checked against the oracle (which builds its own model)."""
    import torch
    cfg = ws.config("c3")
    tf = ws.test_function_for(cfg)
    kw = dict(max_level=cfg["max_level"], eps_gamma=cfg["eps_gamma"])
    gm = hd.asg_build_components(cfg["d"], cfg["m"], cfg["anchor"], (tf.c_fn, tf.c_user), comps=cfg["comps"], **kw)
    model, _ = oracle.build_model(cfg["comps"], cfg["d"], cfg["m"], cfg["anchor"], (tf.c_fn, tf.c_user), **kw)
    w = _compare_models(hd, gm, model)
    X = ws.points_for(cfg)
    Xd = torch.from_numpy(X).to("cuda:0")
    Y = hd.hdmr_eval(gm, Xd)
    torch.cuda.synchronize()
    idx = np.random.default_rng(1).choice(X.shape[0], 2000, replace=False)
    idx = np.concatenate([idx, np.arange(20), np.arange(X.shape[0] - 20, X.shape[0])])
    ref = oracle.evaluate(model, X[idx])
    err = float(np.abs(Y.cpu().numpy()[idx] - ref).max())
    print("c3: %d rows, surplus diff %.3e, sampled eval max |err| %.3e" % (hd.hdmr_get_info(gm)["n_rows"], w, err))
    assert err <= TOL
    # the mixed-precision path on the same launch configuration: normwise 1e-6
    Ym = hd.hdmr_eval(gm, Xd, precision=hd.MIXED)
    torch.cuda.synchronize()
    Ym = Ym.cpu().numpy()[idx]
    nw = float(np.linalg.norm(Ym - ref) / np.linalg.norm(ref))
    print("c3 mixed: sampled normwise error %.3e" % nw)
    assert nw <= 1e-6


def test_c5_full_size_build_and_eval(hd):
    """The surrogate's interpolant at full size: d=300, 300 + 300 components
    (order-2 terms scaled 1/100), L=7, eps=1e-4, m=151; the GPU build against
    the oracle's own build, then 5e5 points through the plain FP64 and mixed
    paths, 2000 sampled points plus the first and last rows checked."""
    import torch
    cfg = ws.config("c5")
    tf = ws.TestFunction(cfg["d"], cfg["m"], cfg["pairs"], cfg["seed"], ref=cfg["anchor"], pair_scale=0.01)
    kw = dict(max_level=cfg["max_level"], eps_gamma=cfg["eps_gamma"])
    gm = hd.asg_build_components(cfg["d"], cfg["m"], cfg["anchor"], (tf.c_fn, tf.c_user), comps=cfg["comps"], **kw)
    model, _ = oracle.build_model(cfg["comps"], cfg["d"], cfg["m"], cfg["anchor"], (tf.c_fn, tf.c_user), **kw)
    w = _compare_models(hd, gm, model)
    X = ws.points_for(cfg, n=500_000, seed=2)
    Xd = torch.from_numpy(X).to("cuda:0")
    Y = hd.hdmr_eval(gm, Xd)
    Ym = hd.hdmr_eval(gm, Xd, precision=hd.MIXED)
    torch.cuda.synchronize()
    idx = np.random.default_rng(2).choice(X.shape[0], 2000, replace=False)
    idx = np.concatenate([idx, np.arange(20), np.arange(X.shape[0] - 20, X.shape[0])])
    ref = oracle.evaluate(model, X[idx])
    err = float(np.abs(Y.cpu().numpy()[idx] - ref).max())
    nw = float(np.linalg.norm(Ym.cpu().numpy()[idx] - ref) / np.linalg.norm(ref))
    print("c5: %d rows, surplus diff %.3e, sampled eval max |err| %.3e, mixed normwise %.3e" %
          (hd.hdmr_get_info(gm)["n_rows"], w, err, nw))
    assert err <= TOL
    assert nw <= 1e-6
