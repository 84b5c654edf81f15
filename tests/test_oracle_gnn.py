"""Pins of the learned-correction oracle (oracle/gnn.py).

* bf16 rounding against hand-worked bit patterns (ties to even, carries).
* The network gradient against central finite differences of the loss in
  float64 with the bf16 rounding switched off (rounding is piecewise
  constant, so differences through it measure nothing).
* The targets: c* minimises ||e - z - sum c_p Z_p|| (random perturbations of
  c* only increase it), and the loss identity
  ||e - z'||^2 / ||e||^2 = ||e - z - sum c*_p Z_p||^2 / ||e||^2 + loss.
* Adam against its closed form on the first step (|update| = lr per weight).
"""
import numpy as np
import pytest

import oracle.gnn as G


def test_bf16_rounding_bit_patterns():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -9, -2.5, 0.0,
                  1.0 + 2 ** -7 + 2 ** -9], dtype=np.float32)
    # 1+2^-8 is a tie between 1 and 1+2^-7: even mantissa -> 1; 1+3*2^-8 ties up to 1+2^-6
    exp = np.array([1.0, 1.0, 1.0 + 2 ** -6, 1.0, -2.5, 0.0, 1.0 + 2 ** -7])
    assert np.array_equal(G.bf16(x), exp)


def _no_rounding(monkeypatch):
    monkeypatch.setattr(G, "bf16", lambda a: np.asarray(a, dtype=np.float64))


def test_gradient_matches_finite_differences(monkeypatch):
    _no_rounding(monkeypatch)
    rng = np.random.default_rng(3)
    adj = (rng.random((G.P, G.P)) < 0.08).astype(int)
    adj = np.maximum(adj, adj.T)
    ahat = G.normalized_adjacency(adj)
    X = rng.normal(size=(G.P, G.F_IN))
    cstar = rng.normal(size=G.P) + 1j * rng.normal(size=G.P)
    w = rng.random(G.P)
    th = G.init_params(1)
    th[G.N_PARAMS - G.F_OUT:] = rng.normal(size=G.F_OUT) * 0.1     # nonzero output bias
    th[-G.F_OUT + 2:] = 0.0
    loss, g = G.loss_and_grad(th, ahat, X, cstar, w)
    idx = np.concatenate([rng.choice(G.N_PARAMS - 16 * 64 - 16, 40, replace=False),
                          np.arange(G.N_PARAMS - 16 * 64 - 16, G.N_PARAMS - 16 * 64 - 16 + 2)])
    h = 1e-6
    for i in idx:
        tp, tm = th.copy(), th.copy()
        tp[i] += h
        tm[i] -= h
        fd = (G.loss_and_grad(tp, ahat, X, cstar, w)[0] - G.loss_and_grad(tm, ahat, X, cstar, w)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_targets_minimise_the_error_and_loss_identity():
    rng = np.random.default_rng(4)
    n = 3000
    sub = np.sort(rng.integers(0, G.P, size=n))
    z = rng.normal(size=n) + 1j * rng.normal(size=n)
    e = z * (1 + 0.3 * rng.normal(size=n)) + 0.2 * (rng.normal(size=n) + 1j * rng.normal(size=n))
    cs, w = G.targets(sub, z, e)

    def err(c):
        return np.linalg.norm(e - z - c[sub] * z) ** 2 / np.linalg.norm(e) ** 2

    e0 = err(cs)
    for _ in range(5):
        c = cs + 0.05 * (rng.normal(size=G.P) + 1j * rng.normal(size=G.P))
        assert err(c) > e0
        assert abs(err(c) - (e0 + np.sum(w * np.abs(c - cs) ** 2))) <= 1e-10


def test_adam_first_step():
    th = np.array([1.0, -2.0, 3.0])
    g = np.array([0.5, -1e-3, 7.0])
    t2, m, v = G.adam(th, np.zeros(3), np.zeros(3), g, 1, lr=0.01)
    assert np.allclose(t2 - th, -0.01 * np.sign(g), rtol=1e-4, atol=0)
