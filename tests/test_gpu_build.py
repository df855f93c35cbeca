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


def _export_all(hd, gm):
    info = hd.hdmr_get_info(gm)
    out = []
    for s in range(info["n_components"]):
        dims, lv, ix, al, w = hd.hdmr_export_component(gm, s)
        out.append((dims, np.asarray(lv).copy(), np.asarray(ix).copy(),
                    np.ascontiguousarray(al).view(np.uint64).copy(), w))
    return info, out


_REFINE_CASES = {
    # (d, m, pairs, comps or max_order, build keywords)
    "rule0": (8, 5, "c2", None, dict(max_level=8, eps_gamma=1e-4, refine_rule=0)),
    "rule1": (8, 5, "c2", None, dict(max_level=8, eps_gamma=1e-4, refine_rule=1)),
    "order3_level_rule0": (5, 3, [(0, 1), (1, 2), (2, 3), (3, 4)], 3, dict(max_level=5, level_rule=0, eps_gamma=1e-5)),
    "order3_level_rule1": (5, 3, [(0, 1), (1, 2), (2, 3), (3, 4)], 3, dict(max_level=7, level_rule=1, eps_gamma=1e-5)),
    "order4_regular": (4, 2, [(0, 1), (2, 3)], 4, dict(max_level=4, level_rule=1, eps_gamma=-1.0)),
    "alg2_criteria": (6, 4, [(0, 1), (2, 3), (1, 4)], 3, dict(max_level=6, eps_gamma=1e-4, eps_eta=1e-9)),
    "nothing_accepted": (6, 4, [(0, 1)], 2, dict(max_level=6, eps_gamma=1e9)),
}


@pytest.mark.parametrize("case", sorted(_REFINE_CASES))
def test_device_refinement_matches_host(hd, monkeypatch, case):
    """k_refine (the default) against the host's admission of children
    (HDMR_REFINE=host): the same grid rows in the same order and bitwise the
    same surpluses, since each step's node order depends only on the set of
    admitted children."""
    d, m, pairs, order, kw = _REFINE_CASES[case]
    if pairs == "c2":
        cfg = ws.config("c2", d=d, m=m, npairs="all", max_level=kw["max_level"])
        tf, anchor = ws.test_function_for(cfg), cfg["anchor"]
        args = dict(comps=cfg["comps"])
    else:
        tf = ws.TestFunction(d, m, pairs, seed=23)
        anchor = tf.ref
        args = dict(max_order=order)
    gms = {}
    for mode in ("host", "device"):
        if mode == "host":
            monkeypatch.setenv("HDMR_REFINE", "host")
        else:
            monkeypatch.delenv("HDMR_REFINE", raising=False)
        gms[mode] = hd.asg_build_components(d, m, anchor, (tf.c_fn, tf.c_user), **args, **kw)
    ih, ch = _export_all(hd, gms["host"])
    idv, cd = _export_all(hd, gms["device"])
    assert ih == idv
    assert len(ch) == len(cd)
    for (dh, lh, xh, ah, wh), (dd, ld, xd, ad, wd) in zip(ch, cd):
        assert dh == dd and wh == wd
        np.testing.assert_array_equal(lh, ld)
        np.testing.assert_array_equal(xh, xd)
        np.testing.assert_array_equal(ah, ad)
    if "eps_eta" in kw:
        rh, rd = hd.hdmr_build_report(gms["host"]), hd.hdmr_build_report(gms["device"])
        assert rh["candidates"] == rd["candidates"] and list(rh["kept"]) == list(rd["kept"])
    print("%s: %d rows in %d components, identical" % (case, ih["n_rows"], ih["n_components"]))


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


@pytest.mark.parametrize("path", ["gather", "sorted"])
def test_naive_eq_3_16_mode(hd, path, monkeypatch):
    """eq (3.16) term by term (hdmr_model_naive of an eq (4.2)-form build)
    against the oracle's term-by-term sum, on both kernels, at 1e-12; it
    agrees with the regrouped eq (4.2) evaluation of the same build; a family
    that is not closed under subsets is refused."""
    import torch
    monkeypatch.setenv("HDMR_EVAL_PATH", path)
    d, m = 6, 5
    tf = ws.TestFunction(d, m, [(0, 1), (2, 4), (3, 5)], seed=11)
    comps = ws.all_components(d, 2)
    kw = dict(max_level=6, eps_gamma=1e-3)
    model, info = oracle.build_model(comps, d, m, tf.ref, (tf.c_fn, tf.c_user), form="paper", **kw)
    gm = hd.asg_build_components(d, m, tf.ref, (tf.c_fn, tf.c_user), comps=comps, form=1, **kw)
    f_anchor = tf(tf.ref[None, :])[0]
    naive = hd.hdmr_model_naive(gm, f_anchor)
    info_n = hd.hdmr_get_info(naive)
    assert info_n["n_components"] == d + 3 * len([S for S in comps if len(S) == 2])
    rng = np.random.default_rng(13)
    X = np.vstack([rng.random((20000, d)), np.zeros((1, d)), np.ones((1, d))])
    Xd = torch.from_numpy(X).to("cuda:0")
    Yn = hd.hdmr_eval(naive, Xd).cpu().numpy()
    Yv = hd.hdmr_eval(gm, Xd).cpu().numpy()
    idx = np.concatenate([np.arange(2000), [X.shape[0] - 2, X.shape[0] - 1]])
    ref = oracle.evaluate_naive(model, X[idx], info["f_anchor"])
    err = np.abs(Yn[idx] - ref).max()
    print("naive eq (3.16) on %s path: max |err| vs oracle %.3e, vs regrouped %.3e" %
          (path, err, np.abs(Yn - Yv).max()))
    assert err <= TOL
    assert np.abs(Yn - Yv).max() <= 1e-11
    from paper_2202_06555_amd import surrogate as sg
    sub = sg.hdmr_model_select(gm, comps=[s for s, S in enumerate(comps) if S != (0,)])
    with pytest.raises(hd.HdmrError) as e:
        hd.hdmr_model_naive(sub, f_anchor)
    assert e.value.code == hd.hdmr.HDMR_EINVAL


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
    eps=1e-4, m=51; 4e6 next-state points through the plain FP64 and mixed
    paths in the benchmark's launch configuration; 1e5 sampled points plus the
    first and last rows checked against the oracle (which builds its own
    model): plain max-abs 1e-12, mixed 1e-6 per output."""
    import torch
    import _fullsize as fs
    cfg = ws.config("c3")
    tf = ws.test_function_for(cfg)
    kw = dict(max_level=cfg["max_level"], eps_gamma=cfg["eps_gamma"])
    gm = hd.asg_build_components(cfg["d"], cfg["m"], cfg["anchor"], (tf.c_fn, tf.c_user), comps=cfg["comps"], **kw)
    model, _ = oracle.build_model(cfg["comps"], cfg["d"], cfg["m"], cfg["anchor"], (tf.c_fn, tf.c_user), **kw)
    w = _compare_models(hd, gm, model)
    X = ws.points_for(cfg)
    Xd = torch.from_numpy(X).to("cuda:0")
    Y = hd.hdmr_eval(gm, Xd)
    Ym = hd.hdmr_eval(gm, Xd, precision=hd.MIXED)
    torch.cuda.synchronize()
    idx = fs.sample_rows(X.shape[0], 100_000, 1)
    ref = oracle.evaluate(model, X[idx])
    err = float(np.abs(Y.cpu().numpy()[idx] - ref).max())
    po = fs.per_output_rel(Ym.cpu().numpy()[idx], ref)
    print("c3: %d rows, surplus diff %.3e; %d sampled points: plain max |err| %.3e, mixed worst per-output %.3e" %
          (hd.hdmr_get_info(gm)["n_rows"], w, len(idx), err, po))
    assert err <= TOL
    assert po <= 1e-6


def test_c5_full_size_build_and_eval(hd):
    """The surrogate's interpolant at full size: d=300, 300 + 300 components
    (order-2 terms scaled 1/100), L=7, eps=1e-4, m=151; the GPU build against
    the oracle's own build, then 1e6 points through the plain FP64 and mixed
    paths, 1e5 sampled points plus the first and last rows checked."""
    import torch
    import _fullsize as fs
    cfg = ws.config("c5")
    tf = ws.TestFunction(cfg["d"], cfg["m"], cfg["pairs"], cfg["seed"], ref=cfg["anchor"], pair_scale=0.01)
    kw = dict(max_level=cfg["max_level"], eps_gamma=cfg["eps_gamma"])
    gm = hd.asg_build_components(cfg["d"], cfg["m"], cfg["anchor"], (tf.c_fn, tf.c_user), comps=cfg["comps"], **kw)
    model, _ = oracle.build_model(cfg["comps"], cfg["d"], cfg["m"], cfg["anchor"], (tf.c_fn, tf.c_user), **kw)
    w = _compare_models(hd, gm, model)
    X = ws.points_for(cfg, n=1_000_000, seed=2)
    Xd = torch.from_numpy(X).to("cuda:0")
    Y = hd.hdmr_eval(gm, Xd)
    Ym = hd.hdmr_eval(gm, Xd, precision=hd.MIXED)
    torch.cuda.synchronize()
    idx = fs.sample_rows(X.shape[0], 100_000, 2)
    ref = oracle.evaluate(model, X[idx])
    err = float(np.abs(Y.cpu().numpy()[idx] - ref).max())
    po = fs.per_output_rel(Ym.cpu().numpy()[idx], ref)
    print("c5: %d rows, surplus diff %.3e; %d sampled points: plain max |err| %.3e, mixed worst per-output %.3e" %
          (hd.hdmr_get_info(gm)["n_rows"], w, len(idx), err, po))
    assert err <= TOL
    assert po <= 1e-6
