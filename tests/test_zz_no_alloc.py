"""hdmr_eval_noalloc (the evaluation for callers that cannot allocate device
memory: static library workspace) against hdmr_eval, through the C ABI.

Bar: the same kernels run on the same inputs, so plain FP64 results are held to
max-abs 1e-12 and mixed results to the mixed bar (per output max|err|/max|F|
<= 1e-6) against hdmr_eval's output; both are also checked against the FP64
oracle.  Two calls in a row, the second with fewer points, on the gather path,
the cell-sorted plain path and the mixed path; an oversized call is rejected
before any work is enqueued."""
import numpy as np
import pytest

import oracle
import workloads.synth as ws

pytestmark = pytest.mark.gpu

TOL = 1e-12
MIXED_BAR = 1e-6


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


def _per_output(Y, ref):
    return float((np.abs(Y - ref).max(axis=0) / np.abs(ref).max(axis=0)).max())


@pytest.mark.parametrize("sizes,prec", [((3000, 1200), "plain"), ((40000, 20000), "plain"),
                                        ((30000, 5000), "mixed")])
def test_noalloc_matches_eval(hd, sizes, prec):
    import torch
    model = ws.synthetic_regular_model(d=6, m=13, order=2, ell=6, seed=21)
    gm = hd.hdmr_model_from_surpluses(model)
    precision = hd.PLAIN_FP64 if prec == "plain" else hd.MIXED
    rng = np.random.default_rng(7)
    for n in sizes:
        X = rng.random((n, 6))
        X[0] = 0.0
        X[1] = 1.0
        Xd = _dev(X)
        Yn = torch.full((n, 13), -7.0, dtype=torch.float64, device="cuda:0")
        hd.hdmr_eval_noalloc(gm, Xd, Yn, precision=precision)
        Ye = hd.hdmr_eval(gm, Xd, precision=precision)
        torch.cuda.synchronize()
        Yn, Ye = Yn.cpu().numpy(), Ye.cpu().numpy()
        ref = oracle.evaluate(model, X[:2000])
        if prec == "plain":
            assert np.abs(Yn - Ye).max() <= TOL
            assert np.abs(Yn[:2000] - ref).max() <= TOL
        else:
            assert _per_output(Yn, Ye) <= MIXED_BAR
            assert _per_output(Yn[:2000], ref) <= MIXED_BAR


def test_noalloc_rejects_oversized_calls(hd):
    import torch
    model = ws.synthetic_regular_model(d=4, m=3, order=2, ell=4, seed=3)
    gm = hd.hdmr_model_from_surpluses(model)
    n = 4_000_000
    X = torch.rand((n, 4), dtype=torch.float64, device="cuda:0")
    Y = torch.full((n, 3), 5.0, dtype=torch.float64, device="cuda:0")
    with pytest.raises(hd.HdmrError) as ei:
        hd.hdmr_eval_noalloc(gm, X, Y)
    assert ei.value.code == hd.hdmr.HDMR_EINVAL and "static workspace" in str(ei.value)
    torch.cuda.synchronize()
    assert bool((Y == 5.0).all())   # nothing was enqueued
    # a call within the limit afterwards still works
    Xs = X[:1000].contiguous()
    Ys = torch.empty((1000, 3), dtype=torch.float64, device="cuda:0")
    hd.hdmr_eval_noalloc(gm, Xs, Ys)
    np.testing.assert_allclose(Ys.cpu().numpy(), oracle.evaluate(model, Xs.cpu().numpy()), rtol=0, atol=TOL)
