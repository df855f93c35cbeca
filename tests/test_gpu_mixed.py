"""GPU parity of the mixed-precision evaluation (FP32 basis and surpluses,
split-BF16 matrix-core products with FP32 accumulation per pass, FP64
accumulation across components and of c0) against the FP64 oracle, through
the C ABI.  Bar, per output o: max_p |Y_po - Y_oracle,po| / max_p |Y_oracle,po|
<= 1e-6 on every component-form model (the normwise error is printed beside
it); eq (4.2)-form models, whose weighted terms cancel, are held per output to
1e-6 relative to max_p of the summed |terms|.
NaN and out-of-domain points behave as in the plain path."""
import numpy as np
import pytest

import oracle
import workloads.synth as ws

pytestmark = pytest.mark.gpu

BAR = 1e-6


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


def _per_output(Y, ref, scale=None):
    """max over outputs of max_p |Y - ref| / max_p |scale| (scale = ref)."""
    scale = ref if scale is None else scale
    Y, ref, scale = (np.asarray(a).reshape(a.shape[0], -1) for a in (Y, ref, scale))
    return float((np.abs(Y - ref).max(axis=0) / np.maximum(np.abs(scale).max(axis=0), 1e-300)).max())


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
    nw, po = _normwise(Y, ref), _per_output(Y, ref)
    print("c1 mixed normwise %.3e, worst per-output %.3e, max |err| %.3e" % (nw, po, np.abs(Y - ref).max()))
    assert po <= BAR


@pytest.mark.parametrize("m", [1, 3, 16, 17, 51, 64, 65, 130, 256])
def test_mixed_output_widths(hd, m):
    rng = np.random.default_rng(100 + m)
    model = ws.synthetic_regular_model(d=5, m=m, order=2, ell=5, seed=m)
    X = np.vstack([_special_points(5, rng, 300), ws.uniform_points(5000, 5, seed=m)])
    gm = hd.hdmr_model_from_surpluses(model)
    Y = _mixed(hd, gm, X)
    ref = oracle.evaluate(model, X)
    po = _per_output(Y, ref)
    print("m=%d mixed worst per-output %.3e" % (m, po))
    assert po <= BAR


def test_mixed_nan_outside_and_empty(hd):
    import torch
    model = ws.synthetic_regular_model(d=4, m=3, order=2, ell=3, seed=2)
    X = np.array([[0.3, np.nan, 0.2, 0.1], [-1.0, 2.0, -3.0, 5.0], [0.3, 0.4, 0.2, 0.1]])
    gm = hd.hdmr_model_from_surpluses(model)
    Y = _mixed(hd, gm, X)
    ref = oracle.evaluate(model, X)
    assert np.all(np.isnan(Y[0]))
    np.testing.assert_array_equal(Y[1], ref[1])      # all basis functions vanish: exactly c0
    assert _per_output(Y[2:], ref[2:]) <= BAR
    empty = torch.empty((0, 4), dtype=torch.float64, device="cuda:0")
    assert hd.hdmr_eval(gm, empty, precision=hd.MIXED).shape == (0, 3)


def test_mixed_adaptive_three_dim_and_paper_form(hd):
    """Component form (u_S surpluses, unit weights): the per-output bar.  The
    eq (4.2) form sums integer-weighted cut functions b_S g_S that cancel
    (|F| far below sum |b_S g_S|), and FP32 rounding error scales with the
    summed terms; its bar is 1e-6 per output relative to the summed |terms|."""
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
        nw, po = _normwise(Y, ref), _per_output(Y, ref)
        rel_terms = _per_output(Y, ref, scale=mag)
        print("adaptive 3-D %s form: mixed normwise %.3e, worst per-output %.3e, relative to summed terms %.3e" %
              (form, nw, po, rel_terms))
        if form == "component":
            assert po <= BAR
        assert rel_terms <= BAR


def test_mixed_c2_full_size_all_points(hd):
    # all 1e6 next-state points of the d=20 workload against the oracle
    import torch
    import _fullsize as fs
    X = fs.c2_points()
    gm = hd.hdmr_model_from_surpluses(fs.c2_model())
    Y = hd.hdmr_eval(gm, _dev(X), precision=hd.MIXED)
    torch.cuda.synchronize()
    Y = Y.cpu().numpy()
    ref = fs.c2_reference()
    nw, po = _normwise(Y, ref), _per_output(Y, ref)
    print("c2 mixed, all points: normwise %.3e, worst per-output %.3e" % (nw, po))
    assert po <= BAR
