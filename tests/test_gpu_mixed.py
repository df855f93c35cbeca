"""GPU parity of the mixed-precision evaluation (FP32 basis and surpluses,
split-BF16 matrix-core products with FP32 accumulation per pass, FP64
accumulation across components and of c0) against the FP64 oracle, through
the C ABI.  Bar: normwise relative error ||Y - Y_oracle||_F / ||Y_oracle||_F
<= 1e-6 on every component-form model; eq (4.2)-form models, whose weighted
terms cancel, are held to 1e-6 relative to the norm of the summed |terms|.
NaN and out-of-domain points behave as in the plain path."""
import numpy as np
import pytest

import oracle
import workloads.synth as ws

pytestmark = pytest.mark.gpu

NORMWISE = 1e-6


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


def _mixed(hd, gm, X):
    return hd.hdmr_eval(gm, _dev(X), precision=hd.MIXED).cpu().numpy()


def _normwise(Y, ref):
    return float(np.linalg.norm(Y - ref) / max(np.linalg.norm(ref), 1e-300))


def _special_points(d, rng, n):
    X = rng.random((n, d))
    X[0] = 0.0
    X[1] = 1.0
    X[2] = 0.5
    X[3:40] = rng.integers(0, 257, size=(37, d)) / 256.0
    X[40:60] = rng.integers(1, 256, size=(20, d)) / 256.0 + 1e-17
    X[60, 0] = -0.25
    X[61, d - 1] = 1.75
    return X


def test_c1_mixed(hd):
    cfg = ws.config("c1")
    model = ws.synthetic_regular_model(cfg["d"], cfg["m"], cfg["order"], cfg["ell"], cfg["seed"])
    X = ws.points_for(cfg)
    gm = hd.hdmr_model_from_surpluses(model)
    Y = _mixed(hd, gm, X)
    ref = oracle.evaluate(model, X)
    nw = _normwise(Y, ref)
    print("c1 mixed normwise %.3e, max |err| %.3e" % (nw, np.abs(Y - ref).max()))
    assert nw <= NORMWISE


@pytest.mark.parametrize("m", [1, 3, 16, 17, 51, 64, 65, 130, 256])
def test_mixed_output_widths(hd, m):
    rng = np.random.default_rng(100 + m)
    model = ws.synthetic_regular_model(d=5, m=m, order=2, ell=5, seed=m)
    X = np.vstack([_special_points(5, rng, 300), ws.uniform_points(5000, 5, seed=m)])
    gm = hd.hdmr_model_from_surpluses(model)
    Y = _mixed(hd, gm, X)
    ref = oracle.evaluate(model, X)
    assert _normwise(Y, ref) <= NORMWISE
    # every output column on its own
    for o in range(m):
        assert _normwise(Y[:, o], ref[:, o]) <= 10 * NORMWISE


def test_mixed_nan_outside_and_empty(hd):
    import torch
    model = ws.synthetic_regular_model(d=4, m=3, order=2, ell=3, seed=2)
    X = np.array([[0.3, np.nan, 0.2, 0.1], [-1.0, 2.0, -3.0, 5.0], [0.3, 0.4, 0.2, 0.1]])
    gm = hd.hdmr_model_from_surpluses(model)
    Y = _mixed(hd, gm, X)
    ref = oracle.evaluate(model, X)
    assert np.all(np.isnan(Y[0]))
    np.testing.assert_array_equal(Y[1], ref[1])      # all basis functions vanish: exactly c0
    assert _normwise(Y[2:], ref[2:]) <= NORMWISE
    empty = torch.empty((0, 4), dtype=torch.float64, device="cuda:0")
    assert hd.hdmr_eval(gm, empty, precision=hd.MIXED).shape == (0, 3)


def test_mixed_adaptive_three_dim_and_paper_form(hd):
    """Component form (u_S surpluses, unit weights): normwise 1e-6.  The
    eq (4.2) form sums integer-weighted cut functions b_S g_S that cancel
    (|F| far below sum |b_S g_S|), and FP32 rounding error scales with the
    summed terms; its bar is 1e-6 relative to ||sum of |terms|||."""
    cfg = ws.config("c2", d=5, m=7, npairs="all", max_level=8)
    tf = ws.test_function_for(cfg)
    comps = ws.all_components(5, 3)
    X = ws.points_for(cfg, n=20000)
    for form in ("component", "paper"):
        model, _ = oracle.build_model(comps, 5, 7, cfg["anchor"], (tf.c_fn, tf.c_user), max_level=8,
                                      eps_gamma=1e-4, form=form)
        gm = hd.hdmr_model_from_surpluses(model)
        Y = _mixed(hd, gm, X)
        ref, mag = oracle.evaluate(model, X, with_abs=True)
        nw = _normwise(Y, ref)
        rel_terms = float(np.linalg.norm(Y - ref) / np.linalg.norm(mag))
        print("adaptive 3-D %s form: mixed normwise %.3e, relative to summed terms %.3e" % (form, nw, rel_terms))
        if form == "component":
            assert nw <= NORMWISE
        assert rel_terms <= NORMWISE


def test_mixed_c2_full_size_sampled(hd):
    import torch
    cfg = ws.config("c2")
    tf = ws.test_function_for(cfg)
    model, _ = oracle.build_model(cfg["comps"], cfg["d"], cfg["m"], cfg["anchor"], (tf.c_fn, tf.c_user),
                                  max_level=cfg["max_level"], eps_gamma=cfg["eps_gamma"])
    X = ws.points_for(cfg)
    gm = hd.hdmr_model_from_surpluses(model)
    Y = hd.hdmr_eval(gm, _dev(X), precision=hd.MIXED)
    torch.cuda.synchronize()
    idx = np.random.default_rng(0).choice(X.shape[0], 3000, replace=False)
    idx = np.concatenate([idx, np.arange(50), np.arange(X.shape[0] - 50, X.shape[0])])
    ref = oracle.evaluate(model, X[idx])
    nw = _normwise(Y.cpu().numpy()[idx], ref)
    print("c2 mixed sampled normwise %.3e" % nw)
    assert nw <= NORMWISE
