"""GPU parity of the BF16 MLP surrogate against the FP64 oracle network
(oracle/mlp.py, BF16 storage emulated at the same places), through the C ABI,
and the interpolant-fallback routing.

Bars (derived from BF16 storage: one BF16 ulp is 2^-8 relative; the GPU
accumulates in FP32 and evaluates GELU in FP32, so an activation can round to
the neighbouring BF16 value where the oracle's FP64 value sits near a
rounding boundary):
  forward  : normwise error <= 4e-3, max-abs <= 2e-2 of the output scale;
  gradient : normwise error per tensor <= 2e-2, loss within 1e-3 relative;
  Adam     : the update from the GPU's own gradient to one FP32 rounding of
             the parameters (they are FP32 masters) plus 1e-6 of the step;
  routing  : network outputs = order-1 part + network prediction, fallback
             outputs = interpolant, to 1e-12; validated errors recomputed
             independently to 1e-9.
"""
import numpy as np
import pytest

import oracle
from oracle import mlp as omlp
import workloads.synth as ws

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2202_06555_amd as hd
    from paper_2202_06555_amd import surrogate as sg
    hd.hdmr_init(0)
    return hd, sg


def _dev(a, dtype=None):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _net(sg, d, w, m, seed, mean=None, std=None):
    p = ws.mlp_init_params(d, w, m, seed)
    rng = np.random.default_rng(seed + 100)
    p = p + rng.normal(0, 0.02, size=p.shape).astype(np.float32)   # non-zero biases
    net = sg.mlp_create(d, w, m, p)
    mean = rng.normal(size=m).astype(np.float32) if mean is None else mean
    std = rng.uniform(0.5, 2.0, size=m).astype(np.float32) if std is None else std
    sg.mlp_set_standardization(net, mean, std)
    return net, p.astype(np.float64), mean.astype(np.float64), std.astype(np.float64)


@pytest.mark.parametrize("d,w,m,n", [(20, 64, 7, 1000), (5, 16, 1, 65), (33, 72, 19, 300)])
def test_forward_parity(env, d, w, m, n):
    hd, sg = env
    net, p, mean, std = _net(sg, d, w, m, seed=d)
    X = np.random.default_rng(1).random((n, d))
    Y = sg.mlp_forward(net, _dev(X)).cpu().numpy()
    out, _ = omlp.forward(p, X, d, w, m, storage="bf16")
    ref = out * std + mean
    scale = np.abs(out).max() * std.max()
    nw = np.linalg.norm((Y - ref) / std) / np.linalg.norm(out)
    print("forward d=%d w=%d m=%d n=%d: normwise %.2e, max-abs %.2e (scale %.2e)" %
          (d, w, m, n, nw, np.abs(Y - ref).max(), scale))
    assert nw <= 4e-3
    assert np.abs(Y - ref).max() <= 2e-2 * scale


@pytest.mark.parametrize("d,w,m,n", [(300, 512, 151, 40000), (45, 256, 257, 70000)])
def test_forward_parity_large_tiles(env, d, w, m, n):
    # enough rows for the 128 x 128 tile kernel (ragged rows, inputs and
    # outputs), checked on sampled rows including the last tile
    hd, sg = env
    net, p, mean, std = _net(sg, d, w, m, seed=d)
    X = np.random.default_rng(3).random((n, d))
    Y = sg.mlp_forward(net, _dev(X)).cpu().numpy()
    idx = np.concatenate([np.random.default_rng(4).choice(n, 1200, replace=False), np.arange(n - 200, n)])
    out, _ = omlp.forward(p, X[idx], d, w, m, storage="bf16")
    ref = out * std + mean
    scale = np.abs(out).max() * std.max()
    nw = np.linalg.norm((Y[idx] - ref) / std) / np.linalg.norm(out)
    print("forward d=%d w=%d m=%d n=%d (sampled): normwise %.2e, max-abs %.2e" % (d, w, m, n, nw, np.abs(Y[idx] - ref).max()))
    assert nw <= 4e-3
    assert np.abs(Y[idx] - ref).max() <= 2e-2 * scale


def _check_grads(g, rg, dims):
    o = 0
    for l in range(4):
        for size in (dims[l + 1] * dims[l], dims[l + 1]):
            a, b = g[o:o + size], rg[o:o + size]
            nw = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
            print("layer %d tensor of %d: normwise %.2e" % (l, size, nw))
            assert nw <= 2e-2
            o += size


def test_gradient_parity_large_batch(env):
    # a batch large enough for the 128 x 128 tile kernel in the forward and
    # in the back-propagated products, and a deep split of the weight gradient
    hd, sg = env
    import torch
    d, w, m, B = 24, 128, 9, 131100
    net, p, mean, std = _net(sg, d, w, m, seed=6)
    rng = np.random.default_rng(7)
    X = rng.random((140000, d))
    Yraw = rng.normal(size=(140000, m)) * std + mean
    idx = rng.choice(140000, B, replace=False)
    loss, g = sg.mlp_loss_grads(net, _dev(X), _dev(Yraw), torch.from_numpy(idx.astype(np.int64)).to("cuda:0"))
    mu32, sd32 = sg.mlp_get_standardization(net)
    T = (Yraw[idx] - mu32.astype(np.float64)) / sd32.astype(np.float64)
    rl, rg = omlp.loss_and_grads(p, X[idx], T, d, w, m, storage="bf16")
    assert abs(loss - rl) <= 1e-3 * rl
    _check_grads(g, rg, [d, w, w, w, m])


def test_gradient_parity(env):
    hd, sg = env
    import torch
    d, w, m, B = 24, 64, 9, 256
    net, p, mean, std = _net(sg, d, w, m, seed=5)
    rng = np.random.default_rng(2)
    X = rng.random((1000, d))
    Yraw = rng.normal(size=(1000, m)) * std + mean
    idx = rng.choice(1000, B, replace=False)
    loss, g = sg.mlp_loss_grads(net, _dev(X), _dev(Yraw), torch.from_numpy(idx.astype(np.int64)).to("cuda:0"))
    # the GPU standardises with its FP32 mean and std
    mu32, sd32 = sg.mlp_get_standardization(net)
    T = (Yraw[idx] - mu32.astype(np.float64)) / sd32.astype(np.float64)
    rl, rg = omlp.loss_and_grads(p, X[idx], T, d, w, m, storage="bf16")
    assert abs(loss - rl) <= 1e-3 * rl
    _check_grads(g, rg, [d, w, w, w, m])


def test_adam_step_matches_textbook_update(env):
    hd, sg = env
    import torch
    d, w, m, B = 12, 32, 4, 128
    net, p, mean, std = _net(sg, d, w, m, seed=7)
    rng = np.random.default_rng(3)
    X = rng.random((B, d))
    Yraw = rng.normal(size=(B, m))
    order = torch.arange(B, dtype=torch.int64, device="cuda:0")
    _, g = sg.mlp_loss_grads(net, _dev(X), _dev(Yraw), order)
    p0 = sg.mlp_get_params(net).astype(np.float64)
    sg.mlp_train(net, _dev(X), _dev(Yraw), order, steps=1, batch=B, lr0=1e-3)
    p1 = sg.mlp_get_params(net).astype(np.float64)
    want, _, _ = omlp.adam_step(p0, g.astype(np.float64), np.zeros_like(p0), np.zeros_like(p0), 1, lr=1e-3)
    # the parameters are FP32: one FP32 rounding of the largest one, plus 1e-6 of the step
    tol = 2.0 ** -23 * np.abs(p0).max() + 1e-6 * 1e-3
    assert np.abs(p1 - want).max() <= tol, (np.abs(p1 - want).max(), tol)


def _small_problem(hd, sg, d=8, m=5, pair_scale=1.0):
    cfg = ws.config("c2", d=d, m=m, npairs="all", max_level=6)
    tf = ws.TestFunction(d, m, cfg["pairs"], seed=11, ref=cfg["anchor"], pair_scale=pair_scale)
    kw = dict(max_level=6, eps_gamma=1e-4)
    full = hd.asg_build_components(d, m, cfg["anchor"], (tf.c_fn, tf.c_user), comps=cfg["comps"], **kw)
    model, _ = oracle.build_model(cfg["comps"], d, m, cfg["anchor"], (tf.c_fn, tf.c_user), **kw)
    return cfg, full, model


def test_training_and_routing(env):
    hd, sg = env
    import torch
    d, m, w = 8, 5, 64
    cfg, full, model = _small_problem(hd, sg, d, m)
    rng = np.random.default_rng(4)
    n = 20000
    X = _dev(ws.points_for(cfg, n=n, seed=1))
    c1 = [s for s, S in enumerate(model["comps"]) if len(S) == 1]
    o1 = sg.hdmr_model_select(full, comps=c1)
    Yres = hd.hdmr_eval(full, X) - hd.hdmr_eval(o1, X)
    net = sg.mlp_create(d, w, m, ws.mlp_init_params(d, w, m, seed=3))
    sg.mlp_fit_standardization(net, Yres)
    steps, B = 400, 256
    order = torch.from_numpy(np.concatenate([rng.permutation(n) for _ in range(steps * B // n + 1)])[:steps * B]
                             .astype(np.int64)).to("cuda:0")
    losses = sg.mlp_train(net, X, Yres, order, steps=steps, batch=B, lr0=3e-3)
    print("loss first %.4f last %.4f" % (losses[:20].mean(), losses[-20:].mean()))
    assert np.all(np.isfinite(losses))
    assert losses[-20:].mean() < 0.5 * losses[:20].mean()
    # routing: validate on fresh points; threshold puts some outputs on each side
    Xv = _dev(ws.points_for(cfg, n=4000, seed=2))
    route0 = sg.mlp_route_create(net, full, Xv, 0.0)
    _, err, _ = sg.mlp_route_info(route0)
    thr = float(np.sort(err)[m // 2])
    route = sg.mlp_route_create(net, full, Xv, thr)
    k, err2, use = sg.mlp_route_info(route)
    np.testing.assert_array_equal(err, err2)
    assert 0 < k < m and k == int(use.sum())
    # the validated errors, recomputed from the oracle interpolant and the network
    Xvh = Xv.cpu().numpy()
    F = oracle.evaluate(model, Xvh)
    model1 = dict(model)
    for key in ("comps", "weights", "levels", "indices", "alpha"):
        model1[key] = [model[key][s] for s in c1]
    F1 = oracle.evaluate(model1, Xvh)
    P = sg.mlp_forward(net, Xv).cpu().numpy()
    np.testing.assert_allclose(err, np.abs(F1 + P - F).max(axis=0), rtol=0, atol=1e-9)
    # routed evaluation: composition per output
    Xt = _dev(ws.points_for(cfg, n=5000, seed=3))
    Yr = sg.mlp_eval_routed(route, Xt).cpu().numpy()
    Ff = hd.hdmr_eval(full, Xt).cpu().numpy()
    F1t = hd.hdmr_eval(o1, Xt).cpu().numpy()
    Pt = sg.mlp_forward(net, Xt).cpu().numpy()
    np.testing.assert_allclose(Yr[:, use], (F1t + Pt)[:, use], rtol=0, atol=1e-12)
    np.testing.assert_allclose(Yr[:, ~use], Ff[:, ~use], rtol=0, atol=1e-12)


def test_model_select(env):
    hd, sg = env
    d, m = 6, 4
    cfg, full, model = _small_problem(hd, sg, d, m)
    X = np.random.default_rng(9).random((700, d))
    outs = [3, 1]
    comps = [0, 2, 7, 11]
    sub = sg.hdmr_model_select(full, comps=comps, outs=outs, with_c0=False)
    msub = dict(model)
    msub["m"] = len(outs)
    msub["c0"] = np.zeros(len(outs))
    for key in ("comps", "weights", "levels", "indices"):
        msub[key] = [model[key][s] for s in comps]
    msub["alpha"] = [model["alpha"][s][:, outs] for s in comps]
    got = hd.hdmr_eval(sub, _dev(X)).cpu().numpy()
    np.testing.assert_allclose(got, oracle.evaluate(msub, X), rtol=0, atol=1e-12)


def test_surrogate_gain_over_interpolant(env):
    """What the trained network gains, at the surrogate's fixed threshold of
    1e-4 max-abs: d=20, m=11, 20 one-dim + 60 two-dim components whose
    order-2 terms are 1000x smaller than the order-1 ones (residual amplitude
    about 2.6e-4, so the order-1 part alone misses 1e-4).  The network learns
    the order-2 residual from 2e5 interpolant points; every output validates
    at <= 1e-4 on 5e4 fresh points and is routed to it; routed evaluation
    (exact order-1 part plus network) holds 1.5e-4 on 1e6 other points and
    runs faster than the interpolant alone.  With a second network as a
    per-point gate at the same threshold, gated points take the interpolant's
    values."""
    hd, sg = env
    import time
    import torch
    TAU = 1e-4
    d, m, w = 20, 11, 256
    cfg = ws.config("c2", d=d, m=m, npairs=60, max_level=6)
    tf = ws.TestFunction(d, m, cfg["pairs"], 11, ref=cfg["anchor"], pair_scale=1e-3)
    full = hd.asg_build_components(d, m, cfg["anchor"], (tf.c_fn, tf.c_user), comps=cfg["comps"], max_level=6,
                                   eps_gamma=1e-5)
    c1 = [s for s, S in enumerate(cfg["comps"]) if len(S) == 1]
    o1 = sg.hdmr_model_select(full, comps=c1)
    n, steps, B = 200_000, 6000, 1024
    X = _dev(ws.points_for(cfg, n=n, seed=1))
    Yres = hd.hdmr_eval(full, X) - hd.hdmr_eval(o1, X)
    res_max = float(Yres.abs().max())
    assert res_max > 2 * TAU            # the order-1 part alone misses the threshold

    def train(seed):
        net = sg.mlp_create(d, w, m, ws.mlp_init_params(d, w, m, seed=seed))
        sg.mlp_fit_standardization(net, Yres)
        rng = np.random.default_rng(5 + seed)
        order = torch.from_numpy(np.concatenate([rng.permutation(n) for _ in range(steps * B // n + 1)])
                                 [:steps * B].astype(np.int64)).to("cuda:0")
        sg.mlp_train(net, X, Yres, order, steps=steps, batch=B, lr0=2e-3, return_losses=False)
        return net

    net = train(0)
    Xv = _dev(ws.points_for(cfg, n=50_000, seed=3))
    route = sg.mlp_route_create(net, full, Xv, TAU)
    k, err, _ = sg.mlp_route_info(route)
    print("validated max-abs per output: max %.2e, median %.2e; residual amplitude %.2e; outputs routed %d of %d"
          % (err.max(), np.median(err), res_max, k, m))
    assert k == m
    Xs = _dev(ws.points_for(cfg, n=1_000_000, seed=2))

    def timed(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            out = fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return out, float(np.median(ts))

    Yi, t_interp = timed(lambda: hd.hdmr_eval(full, Xs))
    Yr, t_routed = timed(lambda: sg.mlp_eval_routed(route, Xs))
    fresh = float((Yr - Yi).abs().max())
    print("fresh-point max-abs %.2e; interpolant %.2f ms, routed %.2f ms: %.2fx"
          % (fresh, t_interp * 1e3, t_routed * 1e3, t_interp / t_routed))
    assert fresh <= 1.5 * TAU
    assert t_interp / t_routed >= 1.5
    # per-point gate: a second network; points where the two disagree by more
    # than TAU in an output take the interpolant's values
    net2 = train(1)
    sg.mlp_route_set_gate(route, net2, full, TAU)
    Yg = sg.mlp_eval_routed(route, Xs)
    torch.cuda.synchronize()
    ng = sg.mlp_route_gated(route)
    P1 = sg.mlp_forward(net, Xs)
    P2 = sg.mlp_forward(net2, Xs)
    gated = ((P1 - P2).abs() > TAU).any(dim=1)
    print("gate: %d of %d points take the interpolant" % (ng, Xs.shape[0]))
    assert ng == int(gated.sum())
    assert float((Yg[gated] - Yi[gated]).abs().max() if ng else 0.0) <= 1e-12
    assert float((Yg[~gated] - Yr[~gated]).abs().max()) == 0.0
    sg.mlp_route_set_gate(route, None, full, TAU)
    assert float((sg.mlp_eval_routed(route, Xs) - Yr).abs().max()) == 0.0


# ---- the GPU network against the exact FP64 network (storage='exact') -------
# Error model of the BF16 kernels, derived from the BF16 unit roundoff
# u = 2^-9 (round to nearest) and the layer widths K: the input, every weight
# and every stored activation / back-propagated gradient is rounded to BF16
# once, a relative perturbation in [-u, u] (variance u^2 / 3), independent
# between operands; products accumulate in FP32 (2^-24, negligible next to u).
# Propagating variances through the exact network (rounding errors of the K
# products of a dot product add in quadrature):
#   var(dz) = (W*W) var(dh) + (2 u^2 / 3) (W*W)(h*h)
#   var(dh') = gelu'(z)^2 var(dz) + (u^2 / 3) h'^2        (stored BF16)
# and the backward pass alike through W^T and gelu' (with gelu''(z) dz for the
# error of the stored pre-activation).  The bound is 8 standard deviations,
# about the largest of 10^6 Gaussian samples: the statistical sqrt(K) u
# analysis of floating-point dot products rather than the worst-case K u.

U = 2.0 ** -9
V = U * U / 3.0
G2 = 0.80 ** 2      # (max |gelu''|)^2
NSIG = 8.0


def _fwd_var(layers, X):
    H = np.asarray(X, np.float64)
    VH = V * H * H
    cache = []
    for l, (W, b) in enumerate(layers):
        Z = H @ W.T + b
        VZ = VH @ (W * W).T + 2.0 * V * ((H * H) @ (W * W).T)
        cache.append((H, VH, Z, VZ))
        if l < 3:
            Hn = omlp.gelu(Z)
            VH = omlp.gelu_grad(Z) ** 2 * VZ + V * Hn * Hn
            H = Hn
    return Z, VZ, cache


@pytest.mark.parametrize("d,w,m,n", [(20, 64, 7, 1000), (33, 72, 19, 300), (300, 512, 151, 40000)])
def test_forward_within_bf16_error_model_of_exact_network(env, d, w, m, n):
    hd, sg = env
    net, p, mean, std = _net(sg, d, w, m, seed=d + 1)
    X = np.random.default_rng(8).random((n, d))
    Y = sg.mlp_forward(net, _dev(X)).cpu().numpy()
    idx = np.arange(n) if n <= 2000 else np.random.default_rng(9).choice(n, 1500, replace=False)
    layers = omlp.unpack(p, d, w, m)
    out, _ = omlp.forward(p, X[idx], d, w, m, storage="exact")
    ref = out * std + mean
    _, VZ, _ = _fwd_var(layers, X[idx])
    bound = NSIG * np.sqrt(VZ) * std + 2.0 ** -23 * np.abs(ref)   # FP32 output
    ratio = np.abs(Y[idx] - ref) / bound
    print("forward d=%d w=%d m=%d vs exact network: max |err| / bound = %.3f (median %.3f), max |err| %.2e" %
          (d, w, m, ratio.max(), np.median(ratio), np.abs(Y[idx] - ref).max()))
    assert ratio.max() <= 1.0


def test_gradients_within_bf16_error_model_of_exact_network(env):
    hd, sg = env
    import torch
    d, w, m, B = 24, 64, 9, 512
    net, p, mean, std = _net(sg, d, w, m, seed=15)
    rng = np.random.default_rng(16)
    X = rng.random((2000, d))
    Yraw = rng.normal(size=(2000, m)) * std + mean
    idx = rng.choice(2000, B, replace=False)
    loss, g = sg.mlp_loss_grads(net, _dev(X), _dev(Yraw), torch.from_numpy(idx.astype(np.int64)).to("cuda:0"))
    mu32, sd32 = sg.mlp_get_standardization(net)
    T = (Yraw[idx] - mu32.astype(np.float64)) / sd32.astype(np.float64)
    rl, rg = omlp.loss_and_grads(p, X[idx], T, d, w, m, storage="exact")
    layers = omlp.unpack(p, d, w, m)
    out, VZ, cache = _fwd_var(layers, X[idx])
    # backward: D = dL/dZ of a layer and the variance of its stored value
    D = 2.0 * (out - T) / (B * m)
    VD = (2.0 / (B * m)) ** 2 * VZ + V * D * D
    vars_ = [None] * 4
    for l in range(3, -1, -1):
        H, VH, Z, _ = cache[l]
        W, _ = layers[l]
        vars_[l] = (VD.T @ (H * H) + (D * D).T @ VH, VD.sum(axis=0))
        if l > 0:
            Zp, VZp = cache[l - 1][2], cache[l - 1][3]
            dH = D @ W
            VdH = VD @ (W * W) + V * ((D * D) @ (W * W))
            Dn = dH * omlp.gelu_grad(Zp)
            VD = omlp.gelu_grad(Zp) ** 2 * VdH + G2 * dH * dH * VZp + V * Dn * Dn
            D = Dn
    bound = omlp.pack([(NSIG * np.sqrt(a), NSIG * np.sqrt(b)) for a, b in vars_]) + 2.0 ** -23 * np.abs(rg)
    ratio = np.abs(g - rg) / np.maximum(bound, 1e-300)
    print("gradients vs exact network: max |err| / bound = %.3f (median %.3f)" % (ratio.max(), np.median(ratio)))
    assert ratio.max() <= 1.0
    assert abs(loss - rl) <= 1e-2 * rl
