"""Learned coarse correction: training data from the solver, training on the
GPU with the library's own forward/backward/Adam kernels, and evaluation
against the plain preconditioner.  Every numerical step runs in the library
(eddy_gnn_pair, eddy_gnn_train_step, eddy_solve); this module only drives it.

Training pairs (r, e) with M e = r come from the solver itself: for each
right-hand side, a converged solution x* (tolerance 1e-10) and the iterates x
returned at looser tolerances give r = b - M x and e = x* - x.
"""
from __future__ import annotations

import time

import numpy as np

from . import eddy
from .eddy import GNN_FIN, GNN_P, GNN_PARAMS

_SHAPES = [(GNN_FIN, 64), (64,), (64, 64), (64,), (64, 64), (64,), (64, 16), (16,)]


def init_theta(seed: int, device="cuda"):
    """Glorot-uniform weights, zero biases, output weights scaled by 0.1 and
    only the two used output columns nonzero (float32 device tensor)."""
    import torch
    rng = np.random.default_rng(seed)
    parts = []
    for shp in _SHAPES:
        if len(shp) == 2:
            lim = np.sqrt(6.0 / (shp[0] + shp[1]))
            w = rng.uniform(-lim, lim, size=shp)
            if shp == (64, 16):
                w *= 0.1
                w[:, 2:] = 0.0
            parts.append(w.ravel())
        else:
            parts.append(np.zeros(shp))
    th = np.concatenate(parts).astype(np.float32)
    assert th.size == GNN_PARAMS
    return torch.from_numpy(th).to(device)


def collect_pairs(op, rhs, tols=(1e-1, 3e-2, 1e-2, 3e-3, 1e-3, 1e-4, 1e-5, 1e-6), restart=48, max_iter=20000,
                  precision="mixed"):
    """(X [n, 64, 16], c* [n, 64, 2], w [n, 64]) device tensors from solves of the
    right-hand sides rhs (list of complex128 device vectors)."""
    import torch
    Xs, Cs, Ws = [], [], []
    for b in rhs:
        xs, rep = op.solve(b, tol=1e-10, restart=restart, max_iter=max_iter, precision=precision)
        if not rep.converged:
            continue
        for tol in tols:
            xk, _ = op.solve(b, tol=tol, restart=restart, max_iter=max_iter, precision=precision)
            X, cs, w = op.gnn_pair(b, xk, xs)
            Xs.append(X)
            Cs.append(cs)
            Ws.append(w)
    return torch.stack(Xs), torch.stack(Cs), torch.stack(Ws)


def train(sets, steps=400, batch=32, lr=2e-3, seed=0, log_every=50):
    """Adam on batches drawn from sets = [(op, X, c*, w)], one operator per
    step (its adjacency is the graph).  Returns (theta, losses per step)."""
    import torch
    rng = np.random.default_rng(seed)
    theta = init_theta(seed, sets[0][0].device)
    m = torch.zeros_like(theta)
    v = torch.zeros_like(theta)
    hist = []
    for step in range(1, steps + 1):
        op, X, C, W = sets[int(rng.integers(len(sets)))]
        idx = torch.from_numpy(rng.choice(X.shape[0], size=min(batch, X.shape[0]), replace=False)).to(X.device)
        loss = op.gnn_train_step(theta, m, v, X[idx], C[idx], W[idx], step, lr)
        hist.append(float(loss.mean()))
        if log_every and step % log_every == 0:
            print(f"  step {step}: loss {np.mean(hist[-log_every:]):.4f}", flush=True)
    return theta, hist


def mean_loss(op, theta, X, C, W):
    """Mean loss of theta on a set (one training step with lr = 0)."""
    import torch
    m = torch.zeros_like(theta)
    v = torch.zeros_like(theta)
    return float(op.gnn_train_step(theta, m, v, X, C, W, 1, 0.0).mean())


def evaluate(op, b, theta, tol=1e-8, restart=48, max_iter=20000, precision="mixed"):
    """Plain vs learned solves of one right-hand side."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x0, r0 = op.solve(b, tol=tol, restart=restart, max_iter=max_iter, precision=precision)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    x1, r1 = op.solve(b, tol=tol, restart=restart, max_iter=max_iter, precision=precision, gnn_theta=theta)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    diff = float((torch.linalg.norm(x1 - x0) / torch.linalg.norm(x0)).item())
    return {"plain_iters": r0.iters, "plain_s": t1 - t0, "learned_iters": r1.iters, "learned_s": t2 - t1,
            "learned_cycles": r1.learned_cycles, "fell_back": r1.fell_back, "converged": r1.converged,
            "relres": r1.relres, "rel_diff": diff}
