"""Error paths forced from the host: an injected device-allocation failure
(HDMR_FAIL_ALLOC=k makes the library's allocation numbered k fail, counted
from the moment the variable takes that value) gives HDMR_ENOMEM with a
message, leaves no partial model behind, and the library works as before once
the variable is cleared.  The allocation-free entry point is unaffected by
it.  No kernel is made to fail: the failure is decided on the host before the
allocation is made."""
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


def _model():
    return ws.synthetic_regular_model(d=5, m=7, order=2, ell=5, seed=31)


def test_model_upload_fails_cleanly_at_every_allocation(hd, monkeypatch):
    import torch
    model = _model()
    failed = 0
    for k in range(64):
        monkeypatch.setenv("HDMR_FAIL_ALLOC", str(k))
        try:
            gm = hd.hdmr_model_from_surpluses(model)
        except hd.HdmrError as e:
            assert e.code == hd.hdmr.HDMR_ENOMEM, str(e)
            assert "out of memory" in str(e).lower() or "alloc" in str(e).lower(), str(e)
            failed += 1
            continue
        break
    else:
        pytest.fail("64 allocations were not enough to upload a small model")
    print("model upload: allocations 0..%d fail cleanly, %d succeeds" % (failed - 1, failed))
    assert failed >= 3  # the model's tables, surpluses and anchor values are separate allocations
    monkeypatch.delenv("HDMR_FAIL_ALLOC")
    gm = hd.hdmr_model_from_surpluses(model)
    X = ws.uniform_points(3000, model["d"], seed=5)
    Y = hd.hdmr_eval(gm, torch.from_numpy(X).to("cuda:0")).cpu().numpy()
    assert np.abs(Y - oracle.evaluate(model, X)).max() <= TOL


def test_eval_allocation_failure_and_noalloc(hd, monkeypatch):
    import torch
    model = _model()
    gm = hd.hdmr_model_from_surpluses(model)
    n = 20000  # cell-sorted path: its workspace is one allocation
    X = ws.uniform_points(n, model["d"], seed=6)
    Xd = torch.from_numpy(X).to("cuda:0")
    Y = torch.full((n, model["m"]), -7.0, dtype=torch.float64, device="cuda:0")
    monkeypatch.setenv("HDMR_EVAL_PATH", "sorted")
    monkeypatch.setenv("HDMR_FAIL_ALLOC", "0")
    with pytest.raises(hd.HdmrError) as e:
        hd.hdmr_eval(gm, Xd, Y)
    assert e.value.code == hd.hdmr.HDMR_ENOMEM
    torch.cuda.synchronize()
    assert bool((Y == -7.0).all()), "a failed call wrote its output"
    # the static-workspace entry point allocates nothing, so the flag does not reach it
    Yn = torch.full((n, model["m"]), -7.0, dtype=torch.float64, device="cuda:0")
    hd.hdmr_eval_noalloc(gm, Xd, Yn)
    torch.cuda.synchronize()
    monkeypatch.delenv("HDMR_FAIL_ALLOC")
    hd.hdmr_eval(gm, Xd, Y)
    torch.cuda.synchronize()
    Y, Yn = Y.cpu().numpy(), Yn.cpu().numpy()
    idx = np.arange(0, n, 10)
    ref = oracle.evaluate(model, X[idx])
    assert np.abs(Y[idx] - ref).max() <= TOL
    assert np.abs(Yn - Y).max() <= TOL


def test_build_allocation_failure(hd, monkeypatch):
    d, m = 4, 3
    tf = ws.TestFunction(d, m, [(0, 1), (2, 3)], seed=12)
    comps = ws.all_components(d, 2)
    kw = dict(max_level=5, eps_gamma=1e-3)
    failed = 0
    for k in range(0, 400, 7):
        monkeypatch.setenv("HDMR_FAIL_ALLOC", str(k))
        try:
            hd.asg_build_components(d, m, tf.ref, (tf.c_fn, tf.c_user), comps=comps, **kw)
        except hd.HdmrError as e:
            assert e.code == hd.hdmr.HDMR_ENOMEM, str(e)
            failed += 1
            continue
        break
    print("build: %d injected allocation failures reported as HDMR_ENOMEM" % failed)
    assert failed >= 2
    monkeypatch.delenv("HDMR_FAIL_ALLOC")
    gm = hd.asg_build_components(d, m, tf.ref, (tf.c_fn, tf.c_user), comps=comps, **kw)
    model, _ = oracle.build_model(comps, d, m, tf.ref, (tf.c_fn, tf.c_user), **kw)
    X = ws.uniform_points(2000, d, seed=8)
    import torch
    Y = hd.hdmr_eval(gm, torch.from_numpy(X).to("cuda:0")).cpu().numpy()
    assert np.abs(Y - oracle.evaluate(model, X)).max() <= TOL
