"""Shared, cached oracle references of the full-size workloads for the GPU
parity tests (each is computed once per test session: the FP64 oracle needs
about a minute on a 16-core host for each of them)."""
import functools

import numpy as np

import oracle
import workloads.synth as ws


@functools.lru_cache(maxsize=None)
def c2_model():
    """The oracle's own build of the d=20 workload (210 components, L=7,
    eps_gamma=1e-4, m=11)."""
    cfg = ws.config("c2")
    tf = ws.test_function_for(cfg)
    model, _ = oracle.build_model(cfg["comps"], cfg["d"], cfg["m"], cfg["anchor"], (tf.c_fn, tf.c_user),
                                  max_level=cfg["max_level"], eps_gamma=cfg["eps_gamma"])
    return model


@functools.lru_cache(maxsize=None)
def c2_points():
    return ws.points_for(ws.config("c2"))


@functools.lru_cache(maxsize=None)
def c2_reference():
    """Oracle values at all 1e6 next-state points of the d=20 workload."""
    return oracle.evaluate(c2_model(), c2_points())


def per_output_rel(Y, ref):
    """Worst over outputs of max_p |Y - ref| / max_p |ref| (the mixed bar)."""
    err = np.abs(Y - ref).max(axis=0)
    return float((err / np.maximum(np.abs(ref).max(axis=0), 1e-300)).max())


def sample_rows(n, k, seed):
    """k distinct random rows of n plus the first and last 20."""
    idx = np.random.default_rng(seed).choice(n, min(k, n), replace=False)
    return np.unique(np.concatenate([idx, np.arange(min(20, n)), np.arange(max(0, n - 20), n)]))
