"""GPU parity of the adaptive DDSG build (Alg. 2: quadrature eq (3.7),
active-dimension criterion eq (3.19) with the reject set Z, expansion
criterion eq (3.18)) and of hdmr_quadrature against the FP64 oracle, through
the C ABI.  Bars: the same candidates, kept sets and Z; eta and rho within
1e-12 relative (absolute 1e-14 where they vanish); quadratures within 1e-13
relative; the kept models' values within 1e-12."""
import math

import numpy as np
import pytest

import oracle
import workloads.synth as ws
from test_oracle_ddsg import _Separable

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hd():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2202_06555_amd as hd
    hd.hdmr_init(0)
    return hd


def _dev(X):
    import torch
    return torch.from_numpy(np.ascontiguousarray(X)).to("cuda:0")


def _check_report(rep_gpu, rep_orc):
    assert rep_gpu["candidates"] == rep_orc["candidates"]
    zg = [c for c, k in zip(rep_gpu["candidates"], rep_gpu["kept"]) if not k]
    assert zg == rep_orc["Z"]
    for c, e in zip(rep_gpu["candidates"], rep_gpu["eta"]):
        if c in rep_orc["eta"]:
            ref = rep_orc["eta"][c]
            assert abs(e - ref) <= max(1e-12 * abs(ref), 1e-14), (c, e, ref)
        else:
            assert math.isnan(e)
    np.testing.assert_allclose(rep_gpu["rho"], rep_orc["rho"], rtol=1e-12, atol=1e-14)


def test_quadrature_matches_oracle(hd):
    for seed, (d, m, order, ell) in enumerate([(3, 2, 2, 5), (5, 7, 3, 4), (4, 130, 2, 6)]):
        model = ws.synthetic_regular_model(d=d, m=m, order=order, ell=ell, seed=seed)
        gm = hd.hdmr_model_from_surpluses(model)
        q, total = hd.hdmr_quadrature(gm)
        ref = oracle.quadrature(model)
        np.testing.assert_allclose(q, ref, rtol=1e-13, atol=1e-16)
        np.testing.assert_allclose(total, model["c0"] + (model["weights"][:, None] * ref).sum(axis=0),
                                   rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("form", [0, 1])
def test_adaptive_build_closed_form_function(hd, form):
    f = _Separable(beta=[0.5, -0.3])
    cf = f.closed_forms()
    kw = dict(max_level=4, level_rule=0, eps_gamma=-1.0)
    gm = hd.asg_build_components(4, 2, np.full(4, 0.5), f, max_order=3, eps_eta=1e-8, eps_rho=1e-12, form=form,
                                 **kw)
    rep = hd.hdmr_build_report(gm)
    model, rep_o = oracle.build_ddsg(4, 2, np.full(4, 0.5), f, max_order=3, eps_eta=1e-8, eps_rho=1e-12,
                                     form="component" if form == 0 else "paper", **kw)
    _check_report(rep, rep_o)
    np.testing.assert_allclose(rep["rho"][0], cf["rho1"], rtol=1e-12)
    assert hd.hdmr_get_info(gm)["n_components"] == len(model["comps"]) == 5
    X = np.random.default_rng(5).random((3000, 4))
    Y = hd.hdmr_eval(gm, _dev(X)).cpu().numpy()
    np.testing.assert_allclose(Y, oracle.evaluate(model, X), rtol=0, atol=1e-12)


@pytest.mark.parametrize("eps_rho", [0.0, 0.4])
def test_adaptive_build_test_function(hd, eps_rho):
    # pairs outside the function's pair set have zero component functions and
    # are rejected; the kink pair and the other listed pairs are kept; order 3
    # has no candidate left (every triple holds a rejected pair).  With
    # eps_rho = 0.4 the expansion stops after order 1 (rho_1 is about 0.36).
    d, m = 6, 4
    pairs = [(0, 1), (2, 3), (1, 4)]
    tf = ws.TestFunction(d, m, pairs, seed=17)
    kw = dict(max_level=6, eps_gamma=1e-4)
    gm = hd.asg_build_components(d, m, tf.ref, (tf.c_fn, tf.c_user), max_order=3, eps_eta=1e-9, eps_rho=eps_rho,
                                 **kw)
    rep = hd.hdmr_build_report(gm)
    model, rep_o = oracle.build_ddsg(d, m, tf.ref, (tf.c_fn, tf.c_user), max_order=3, eps_eta=1e-9,
                                     eps_rho=eps_rho, **kw)
    _check_report(rep, rep_o)
    kept_pairs = [c for c, k in zip(rep["candidates"], rep["kept"]) if k and len(c) == 2]
    print("kept pairs", kept_pairs, "rho", rep["rho"])
    assert sorted(kept_pairs) == (sorted(pairs) if eps_rho == 0.0 else [])
    assert len(rep["rho"]) == (2 if eps_rho == 0.0 else 1)
    X = ws.next_state_points(20000, d, seed=4)
    Y = hd.hdmr_eval(gm, _dev(X)).cpu().numpy()
    np.testing.assert_allclose(Y, oracle.evaluate(model, X), rtol=0, atol=1e-12)


def test_criteria_off_report_is_empty_and_nan_rejected(hd):
    model = ws.synthetic_regular_model(d=3, m=2, order=2, ell=3, seed=1)
    gm = hd.hdmr_model_from_surpluses(model)
    rep = hd.hdmr_build_report(gm)
    assert rep["candidates"] == [] and len(rep["rho"]) == 0
    f = _Separable(beta=[0.5, -0.3])
    with pytest.raises(hd.HdmrError) as e:
        hd.asg_build_components(4, 2, np.full(4, 0.5), f, max_order=2, eps_eta=float("nan"))
    assert e.value.code == hd.hdmr.HDMR_EINVAL
