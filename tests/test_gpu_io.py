"""Model files: a saved and reloaded model has the same grids, surpluses,
weights and c0 (bit-exact) and evaluates to the same values."""
import numpy as np
import pytest

import oracle
import workloads.synth as ws

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hd():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2202_06555_amd as hd
    hd.hdmr_init(0)
    return hd


def test_save_load_roundtrip(hd, tmp_path):
    import torch
    cfg = ws.config("c2", d=6, m=5, npairs="all", max_level=7)
    tf = ws.test_function_for(cfg)
    gm = hd.asg_build_components(6, 5, cfg["anchor"], (tf.c_fn, tf.c_user), comps=cfg["comps"], max_level=7,
                                 eps_gamma=1e-4, form=1)
    path = str(tmp_path / "m.hdmr")
    hd.hdmr_model_save(gm, path)
    gl = hd.hdmr_model_load(path)
    a, b = hd.hdmr_get_info(gm), hd.hdmr_get_info(gl)
    for key in ("d", "m", "n_components", "n_tuples", "n_rows", "max_level", "max_k"):
        assert a[key] == b[key], key
    for s in range(a["n_components"]):
        ea, eb = hd.hdmr_export_component(gm, s), hd.hdmr_export_component(gl, s)
        assert ea[0] == eb[0] and ea[4] == eb[4]
        for x, y in zip(ea[1:4], eb[1:4]):
            np.testing.assert_array_equal(x, y)
    X = torch.from_numpy(ws.points_for(cfg, n=3000)).to("cuda:0")
    np.testing.assert_array_equal(hd.hdmr_eval(gm, X).cpu().numpy(), hd.hdmr_eval(gl, X).cpu().numpy())
    # and the reloaded model still matches the oracle built the same way
    model, _ = oracle.build_model(cfg["comps"], 6, 5, cfg["anchor"], (tf.c_fn, tf.c_user), max_level=7,
                                  eps_gamma=1e-4, form="paper")
    Xh = X.cpu().numpy()
    np.testing.assert_allclose(hd.hdmr_eval(gl, X).cpu().numpy(), oracle.evaluate(model, Xh), rtol=0, atol=1e-11)
