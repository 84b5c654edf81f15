"""Oracle of the learned coarse correction (test infrastructure only: imported
by tests/ and nothing on the product path).

The correction and its network are not in the paper; they follow the
specification of the solver's learned variant.  Definitions:

* Subdomains: the block-Jacobi blocks (recursive coordinate bisection, in
  their bisection order) grouped into P consecutive runs of equal block count,
  so each subdomain is a spatially compact union of blocks.  Two subdomains
  are adjacent if a tetrahedron holds DOFs of both (its six edges, and its
  four nodes when it conducts): the structural coupling of M, whatever the
  values.
  A_hat = D^-1/2 (A + I) D^-1/2 (symmetric normalisation with self loops).
* Correction of a preconditioned residual z = B r (B the block-Jacobi apply):
  z' = z + sum_p c_p Z_p with Z_p = z restricted to subdomain p.  For a
  (residual, error) pair with A e = r, the coefficients minimising
  ||e - z'||^2 are, since the Z_p have disjoint supports,
  c*_p = <Z_p, e - z> / ||Z_p||^2, and ||e - z'||^2 = ||e - z - sum c*_p Z_p||^2
  + sum_p ||Z_p||^2 |c_p - c*_p|^2.  The training loss is the second term
  divided by ||e||^2: loss = sum_p w_p |c_p - c*_p|^2, w_p = ||Z_p||^2 / ||e||^2.
* Features per subdomain (F = 16 columns, 8 used): ||r_p|| / ||r|| sqrt(P),
  ||z_p|| / ||z|| sqrt(P), Re and Im of <z_p, r_p> / (||z_p|| ||r_p||), the
  fraction of conductor (V) DOFs, log10(omega) / 6, log10(1 + sigma_p / 1e4) / 3
  with sigma_p the subdomain mean over its DOFs of the largest conductivity
  of a tetrahedron containing the DOF, and 1.
* Network (4 layers, width 64): T0 = X W0, H1 = relu(A_hat T0 + b0);
  for l = 1, 2: H_{l+1} = relu(A_hat (H_l W_l) + b_l) + H_l;
  Y = A_hat (H_3 W3) + b3 (16 columns, the first two used): c_p = Y_p0 + i Y_p1.
* Precision: every GEMM operand is rounded to bfloat16 (round to nearest
  even), in the backward pass too (dY, dZ, dT), and accumulated in float32;
  biases, activations, the residual path and the loss stay float32.  The oracle rounds at the same points and accumulates
  in float64.  Backward passes treat the rounding as the identity.
* Adam (Kingma and Ba, 2015) on float32 master weights; the bfloat16 copies
  are the rounded masters.
"""
from __future__ import annotations

import numpy as np

P = 64
F_IN = 16
WIDTH = 64
F_OUT = 16
PARAM_SHAPES = [("W0", (F_IN, WIDTH)), ("b0", (WIDTH,)), ("W1", (WIDTH, WIDTH)), ("b1", (WIDTH,)),
                ("W2", (WIDTH, WIDTH)), ("b2", (WIDTH,)), ("W3", (WIDTH, F_OUT)), ("b3", (F_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in PARAM_SHAPES)


def bf16(x) -> np.ndarray:
    """Round float32 values to bfloat16 (nearest, ties to even), returned as float64."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(theta: np.ndarray) -> dict:
    out, k = {}, 0
    for name, shp in PARAM_SHAPES:
        n = int(np.prod(shp))
        out[name] = theta[k:k + n].reshape(shp)
        k += n
    return out


def pack(d: dict) -> np.ndarray:
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in PARAM_SHAPES])


def init_params(seed: int) -> np.ndarray:
    """Glorot-uniform weights, zero biases, the output layer scaled by 0.1."""
    rng = np.random.default_rng(seed)
    d = {}
    for name, shp in PARAM_SHAPES:
        if name.startswith("W"):
            lim = np.sqrt(6.0 / (shp[0] + shp[1]))
            d[name] = rng.uniform(-lim, lim, size=shp) * (0.1 if name == "W3" else 1.0)
        else:
            d[name] = np.zeros(shp)
    d["W3"][:, 2:] = 0.0
    return pack(d).astype(np.float32).astype(np.float64)


def normalized_adjacency(adj: np.ndarray) -> np.ndarray:
    """A_hat = D^-1/2 (A + I) D^-1/2 from a 0/1 adjacency matrix."""
    a = (np.asarray(adj) != 0).astype(np.float64)
    np.fill_diagonal(a, 1.0)
    d = 1.0 / np.sqrt(a.sum(axis=1))
    return d[:, None] * a * d[None, :]


def forward(theta: np.ndarray, ahat: np.ndarray, X: np.ndarray):
    """(Y [P, F_OUT], cache) with the rounding points of the module doc."""
    p = unpack(theta)
    Ab = bf16(ahat)
    Xb = bf16(X)
    T0 = bf16(Xb @ bf16(p["W0"]))
    Z0 = Ab @ T0 + p["b0"]
    H = [None, np.maximum(Z0, 0.0)]
    Zs = [Z0]
    Hb = [Xb]
    Ts = [T0]
    for l in (1, 2):
        hb = bf16(H[l])
        T = bf16(hb @ bf16(p[f"W{l}"]))
        Z = Ab @ T + p[f"b{l}"]
        H.append(np.maximum(Z, 0.0) + H[l])
        Zs.append(Z)
        Hb.append(hb)
        Ts.append(T)
    h3b = bf16(H[3])
    T3 = bf16(h3b @ bf16(p["W3"]))
    Y = Ab @ T3 + p["b3"]
    Hb.append(h3b)
    return Y, {"Ab": Ab, "Hb": Hb, "Z": Zs, "p": p}


def coefficients(Y: np.ndarray) -> np.ndarray:
    return Y[:, 0] + 1j * Y[:, 1]


def loss_and_grad(theta: np.ndarray, ahat: np.ndarray, X: np.ndarray, cstar: np.ndarray, w: np.ndarray):
    """loss = sum_p w_p |c_p - c*_p|^2 and its gradient (module doc)."""
    Y, c = forward(theta, ahat, X)
    diff = coefficients(Y) - cstar
    loss = float(np.sum(w * np.abs(diff) ** 2))
    dY = np.zeros_like(Y)
    dY[:, 0] = 2.0 * w * diff.real
    dY[:, 1] = 2.0 * w * diff.imag
    Ab, Hb, Z, p = c["Ab"], c["Hb"], c["Z"], c["p"]
    g = {}
    # output layer: Y = Ab T3 + b3, T3 = bf16(Hb3 W3)
    g["b3"] = dY.sum(axis=0)
    dT = bf16(Ab.T @ bf16(dY))
    g["W3"] = Hb[3].T @ dT
    dH = dT @ bf16(p["W3"]).T
    for l in (2, 1):
        dZ = dH * (Z[l] > 0)
        g[f"b{l}"] = dZ.sum(axis=0)
        dT = bf16(Ab.T @ bf16(dZ))
        g[f"W{l}"] = Hb[l].T @ dT
        dH = dH + dT @ bf16(p[f"W{l}"]).T
    dZ = dH * (Z[0] > 0)
    g["b0"] = dZ.sum(axis=0)
    dT = bf16(Ab.T @ bf16(dZ))
    g["W0"] = Hb[0].T @ dT
    g["W3"][:, 2:] = 0.0
    g["b3"][2:] = 0.0
    return loss, pack(g)


def adam(theta, m, v, grad, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (step counts from 1)."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


# ------------------------------------------------------------ data side

def subdomains(blocks: list, nparts: int = P) -> np.ndarray:
    """Subdomain of every DOF: blocks (in bisection order) grouped into nparts runs."""
    nb = len(blocks)
    n = sum(len(b) for b in blocks)
    sub = np.empty(n, dtype=np.int64)
    for k, blk in enumerate(blocks):
        sub[np.asarray(blk)] = (k * nparts) // nb
    return sub


def adjacency(topo, tet: np.ndarray, sub: np.ndarray, nparts: int = P) -> np.ndarray:
    """0/1 subdomain adjacency from the tetrahedra (module doc)."""
    a = np.zeros((nparts, nparts), dtype=np.int64)
    ne = topo.ne
    for t in range(tet.shape[0]):
        d = list(topo.tet2edge[t])
        if topo.cond_tet[t]:
            d += [ne + topo.vmap[v] for v in tet[t]]
        ss = np.unique(sub[np.asarray(d)])
        a[np.ix_(ss, ss)] = 1
    np.fill_diagonal(a, 0)
    return a


def dof_sigma(topo, tet: np.ndarray, region: np.ndarray, sigma: np.ndarray) -> np.ndarray:
    """Per DOF (edges, then conductor nodes): the largest sigma of a tetrahedron containing it."""
    st = np.asarray(sigma, dtype=np.float64)[np.asarray(region)]
    s_e = np.zeros(topo.ne)
    np.maximum.at(s_e, topo.tet2edge.ravel(), np.repeat(st, 6))
    s_n = np.zeros(topo.nv)
    np.maximum.at(s_n, np.asarray(tet).ravel(), np.repeat(st, 4))
    return np.concatenate([s_e, s_n[topo.cond_nodes]])


def static_features(sub, ne: int, dsig: np.ndarray, omega: float, nparts: int = P) -> np.ndarray:
    """Columns 4..7 of the features (module doc)."""
    n = sub.size
    cnt = np.bincount(sub, minlength=nparts).astype(np.float64)
    cond = np.bincount(sub[ne:], minlength=nparts).astype(np.float64) if n > ne else np.zeros(nparts)
    smean = np.bincount(sub, weights=dsig, minlength=nparts) / np.maximum(cnt, 1)
    out = np.zeros((nparts, 4))
    out[:, 0] = cond / np.maximum(cnt, 1)
    out[:, 1] = np.log10(omega) / 6.0
    out[:, 2] = np.log10(1.0 + smean / 1e4) / 3.0
    out[:, 3] = 1.0
    return out


def features(sub, r: np.ndarray, z: np.ndarray, static: np.ndarray, nparts: int = P) -> np.ndarray:
    nr = np.sqrt(np.bincount(sub, weights=np.abs(r) ** 2, minlength=nparts))
    nz = np.sqrt(np.bincount(sub, weights=np.abs(z) ** 2, minlength=nparts))
    zr = np.bincount(sub, weights=(np.conj(z) * r).real, minlength=nparts) \
        + 1j * np.bincount(sub, weights=(np.conj(z) * r).imag, minlength=nparts)
    X = np.zeros((nparts, F_IN))
    X[:, 0] = nr / max(np.linalg.norm(r), 1e-300) * np.sqrt(nparts)
    X[:, 1] = nz / max(np.linalg.norm(z), 1e-300) * np.sqrt(nparts)
    den = nz * nr
    ok = den > 0
    X[ok, 2] = zr.real[ok] / den[ok]
    X[ok, 3] = zr.imag[ok] / den[ok]
    X[:, 4:8] = static
    return X


def targets(sub, z: np.ndarray, e: np.ndarray, nparts: int = P):
    """(c*, w) of the module doc."""
    zz = np.bincount(sub, weights=np.abs(z) ** 2, minlength=nparts)
    d = e - z
    zd = np.bincount(sub, weights=(np.conj(z) * d).real, minlength=nparts) \
        + 1j * np.bincount(sub, weights=(np.conj(z) * d).imag, minlength=nparts)
    cstar = np.where(zz > 0, zd / np.where(zz > 0, zz, 1.0), 0.0)
    w = zz / max(np.vdot(e, e).real, 1e-300)
    return cstar, w
