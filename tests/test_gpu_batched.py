"""GPU parity of hdmr_eval_batched (persistent multi-model launch, graph
replay, autotuned path choice) against the FP64 oracle and against
per-model hdmr_eval, through the C ABI."""
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


def _dev(X):
    import torch
    return torch.from_numpy(np.ascontiguousarray(X)).to("cuda:0")


def _batch(seed=0):
    """Models of uneven dimension, order, grid size and output width, with
    point counts from 0 to above the autotuning threshold."""
    rng = np.random.default_rng(seed)
    specs = [(4, 3, 2, 4, 1000), (7, 1, 1, 6, 63), (5, 17, 2, 5, 20000), (12, 65, 2, 3, 500), (3, 2, 3, 4, 0),
             (9, 130, 2, 3, 300), (6, 8, 2, 6, 1), (20, 11, 2, 3, 5000), (4, 3, 2, 7, 30000)]
    models, X = [], []
    for i, (d, m, order, ell, n) in enumerate(specs):
        models.append(ws.synthetic_regular_model(d=d, m=m, order=order, ell=ell, seed=100 + i))
        P = rng.random((n, d))
        if n > 3:
            P[0] = 0.0
            P[1] = 1.0
            P[2, 0] = np.nan
        X.append(P)
    # an adaptive model built from the test function
    cfg = ws.config("c2", d=6, m=5, npairs="all", max_level=7)
    tf = ws.test_function_for(cfg)
    model, _ = oracle.build_model(cfg["comps"], 6, 5, cfg["anchor"], (tf.c_fn, tf.c_user), max_level=7, eps_gamma=1e-4)
    models.append(model)
    X.append(ws.points_for(cfg, n=3000))
    return models, X


def _check_against_oracle(models, X, Y, tol=TOL):
    for mo, P, V in zip(models, X, Y):
        if P.shape[0] == 0:
            assert V.shape == (0, mo["m"])
            continue
        idx = np.arange(P.shape[0]) if P.shape[0] <= 3000 else np.r_[0:50, np.random.default_rng(0).choice(P.shape[0], 1500, replace=False)]
        ref = oracle.evaluate(mo, P[idx])
        got = V.cpu().numpy()[idx]
        nan = np.isnan(P[idx]).any(axis=1)
        assert np.all(np.isnan(got[nan]))
        np.testing.assert_allclose(got[~nan], ref[~nan], rtol=0, atol=tol)


def test_batched_matches_oracle(hd):
    models, X = _batch()
    gms = [hd.hdmr_model_from_surpluses(mo) for mo in models]
    Y, paths = hd.hdmr_eval_batched(gms, [_dev(P) for P in X])
    print("paths", paths.tolist())
    # -1 none, 0 gather, 1 + v cell-sorted with tile shape v in {0, 1, 2, 4, 6}
    assert paths[4] == -1 and all(p in (0, 1, 2, 3, 5, 7) for i, p in enumerate(paths) if i != 4)
    assert paths[1] == 0 and paths[0] == 0
    _check_against_oracle(models, X, Y)


def test_graph_replay_with_new_data(hd):
    import torch
    models, X = _batch(seed=1)
    gms = [hd.hdmr_model_from_surpluses(mo) for mo in models]
    Xd = [_dev(P) for P in X]
    Yd = [torch.empty((P.shape[0], mo["m"]), dtype=torch.float64, device="cuda:0") for P, mo in zip(X, models)]
    rng = np.random.default_rng(7)
    for rep in range(4):
        # new coordinates in place, eager work in between, then a replay
        for P in Xd:
            if P.shape[0]:
                P.copy_(torch.from_numpy(rng.random(tuple(P.shape))))
        torch.cuda.synchronize()
        _, paths = hd.hdmr_eval_batched(gms, Xd, Yd)
        torch.cuda.synchronize()
        for gm, P, V in zip(gms, Xd, Yd):
            if P.shape[0]:
                ref = hd.hdmr_eval(gm, P)
                np.testing.assert_allclose(V.cpu().numpy(), ref.cpu().numpy(), rtol=0, atol=1e-13)
    _check_against_oracle(models, [P.cpu().numpy() for P in Xd], Yd)


def test_batched_mixed_precision(hd):
    # every model with grid points takes the mixed-capable cell-sorted path
    # (the FP64 gather kernel is never used for HDMR_MIXED); per-output bar
    models, X = _batch(seed=2)
    gms = [hd.hdmr_model_from_surpluses(mo) for mo in models]
    Y, paths = hd.hdmr_eval_batched(gms, [_dev(P) for P in X], precision=hd.MIXED)
    for mo, P, V, path in zip(models, X, Y, paths):
        if P.shape[0] == 0:
            continue
        assert path >= 1, path
        ok = ~np.isnan(P).any(axis=1)
        ref = oracle.evaluate(mo, P[ok][:2000])
        got = V.cpu().numpy()[ok][:2000]
        rel = (np.abs(got - ref).max(axis=0) / np.abs(ref).max(axis=0)).max()
        assert rel <= 1e-6, rel


def test_empty_and_single(hd):
    import torch
    mo = ws.synthetic_regular_model(d=3, m=2, order=2, ell=3, seed=5)
    gm = hd.hdmr_model_from_surpluses(mo)
    Y, paths = hd.hdmr_eval_batched([gm], [torch.empty((0, 3), dtype=torch.float64, device="cuda:0")])
    assert paths.tolist() == [-1] and Y[0].shape == (0, 2)
    Y, paths = hd.hdmr_eval_batched([], [])
    assert Y == [] and len(paths) == 0


@pytest.mark.parametrize("precision", ["plain", "mixed"])
def test_c4_shaped_batch_sampled(hd, precision):
    # four models of the batched workload's generator (d = 22, 13, 10, 53; all
    # one- and two-dimensional components; random downward-closed grids of
    # log-uniform size 50..20000; m = d/2 + 1), 1e4..4e4 points each, one
    # batched call (autotuned paths), 300 sampled points per model against
    # the oracle: plain max-abs 1e-12, mixed per output 1e-6
    import torch
    prec = hd.PLAIN_FP64 if precision == "plain" else hd.MIXED
    models, X = [], []
    for i in (11, 23, 27, 1):
        mo, P = ws.c4_model(i, seed=0, n_range=(10_000, 40_000))
        models.append(mo)
        X.append(P)
    gms = [hd.hdmr_model_from_surpluses(mo) for mo in models]
    Xd = [_dev(P) for P in X]
    Y, paths = hd.hdmr_eval_batched(gms, Xd, precision=prec)        # tuning call
    Y, paths2 = hd.hdmr_eval_batched(gms, Xd, precision=prec)       # tuned call
    torch.cuda.synchronize()
    print("c4-shaped batch (%s): d %s, rows %s, n %s, paths %s" %
          (precision, [mo["d"] for mo in models], [sum(l.shape[0] for l in mo["levels"]) for mo in models],
           [P.shape[0] for P in X], paths2.tolist()))
    assert paths.tolist() == paths2.tolist()
    for mo, P, V in zip(models, X, Y):
        idx = np.random.default_rng(mo["d"]).choice(P.shape[0], 300, replace=False)
        ref = oracle.evaluate(mo, P[idx])
        got = V.cpu().numpy()[idx]
        if precision == "plain":
            assert np.abs(got - ref).max() <= TOL
        else:
            rel = (np.abs(got - ref).max(axis=0) / np.abs(ref).max(axis=0)).max()
            assert rel <= 1e-6, rel
