"""Pins for the oracle's closed-form element integrals.

The reference values are computed by brute force, independently of the
closed forms: barycentric gradients from the 4x4 interpolation system
[x_j y_j z_j 1] g = e_i, Whitney functions evaluated pointwise, their curl by
central differences (exact for the linear Whitney fields), and a collapsed
(Duffy) tensor Gauss-Legendre rule that is exact for the polynomial degrees
involved.
"""
import numpy as np
import pytest

from oracle.elements import element_matrices, geometry
from oracle.topology import LOCAL_EDGES


def duffy_rule(n=5):
    """Points (barycentric l1..l3) and weights on the reference tet (volume 1/6)."""
    g, w = np.polynomial.legendre.leggauss(n)
    g = 0.5 * (g + 1.0)
    w = 0.5 * w
    U, V, W = np.meshgrid(g, g, g, indexing="ij")
    wu, wv, ww = np.meshgrid(w, w, w, indexing="ij")
    l1 = U
    l2 = V * (1 - U)
    l3 = W * (1 - U) * (1 - V)
    jac = (1 - U) ** 2 * (1 - V)
    return np.stack([l1.ravel(), l2.ravel(), l3.ravel()], 1), (wu * wv * ww * jac).ravel()


def random_tets(k, seed):
    rng = np.random.default_rng(seed)
    xyz = rng.normal(size=(4 * k, 3))
    tet = np.arange(4 * k).reshape(k, 4)
    return xyz, tet


def brute(xyz, tet):
    pts, wts = duffy_rule(5)
    out = []
    for t in tet:
        P = xyz[t]
        A = np.hstack([P, np.ones((4, 1))])
        coef = np.linalg.solve(A, np.eye(4))            # column i: (grad l_i, c_i)
        grads = coef[:3, :].T                           # [4, 3]
        E = P[1:] - P[0]
        vol = abs(np.linalg.det(E)) / 6.0
        X = P[0] + pts @ E                              # physical points [q, 3]

        def lam(x):
            return x @ coef[:3, :] + coef[3, :]         # [q, 4]

        def whit(x):
            L = lam(x)
            return np.stack([L[:, a, None] * grads[b] - L[:, b, None] * grads[a] for a, b in LOCAL_EDGES], 1)

        h = 1e-3
        curl = np.zeros((6, 3))
        x0 = P.mean(0, keepdims=True)
        d = [(whit(x0 + h * np.eye(3)[i]) - whit(x0 - h * np.eye(3)[i]))[0] / (2 * h) for i in range(3)]
        # d[i][l, j] = d w_l,j / d x_i
        for l in range(6):
            curl[l] = [d[1][l, 2] - d[2][l, 1], d[2][l, 0] - d[0][l, 2], d[0][l, 1] - d[1][l, 0]]
        wq = wts * 6.0 * vol                            # weights on the physical tet
        Wv = whit(X)                                    # [q, 6, 3]
        L = lam(X)
        out.append({
            "vol": vol,
            "K": vol * curl @ curl.T,
            "M": np.einsum("q,qlx,qmx->lm", wq, Wv, Wv),
            "W": np.einsum("q,qlx,kx->lk", wq, Wv, grads),
            "S": vol * grads @ grads.T,
            "N": np.einsum("q,qi,qj->ij", wq, L, L),
            "F": np.einsum("q,qlx->lx", wq, Wv),
        })
    return out


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_element_integrals_match_quadrature(seed):
    xyz, tet = random_tets(6, seed)
    el = element_matrices(xyz, tet)
    ref = brute(xyz, tet)
    for t, r in enumerate(ref):
        assert abs(el["vol"][t] - r["vol"]) <= 1e-14 * r["vol"]
        for key in ("K", "M", "W", "S", "N", "F"):
            a, b = el[key][t], r[key]
            tol = 1e-12 if key != "K" else 1e-7             # K: finite-difference curl
            assert np.max(np.abs(a - b)) <= tol * np.max(np.abs(b)), key


def test_element_orientation_independent():
    """Swapping two vertices flips det but not |K| or the symmetric forms."""
    xyz, tet = random_tets(4, 7)
    v1, g1, d1 = geometry(xyz, tet)
    v2, g2, d2 = geometry(xyz, tet[:, [1, 0, 2, 3]])
    assert np.allclose(v1, v2, rtol=1e-14) and np.all(np.sign(d1) == -np.sign(d2))
    assert np.allclose(g1[:, [1, 0, 2, 3]], g2, rtol=1e-12, atol=1e-12)


def test_whitney_tangential_moment():
    """The line integral of w_(a,b) along its own edge a->b is 1 (basis normalisation)."""
    xyz, tet = random_tets(3, 11)
    _, grad, _ = geometry(xyz, tet)
    for t in range(tet.shape[0]):
        P = xyz[tet[t]]
        for l, (a, b) in enumerate(LOCAL_EDGES):
            s = np.linspace(0, 1, 7)
            # on the edge l_a = 1 - s, l_b = s
            w = (1 - s)[:, None] * grad[t, b] - s[:, None] * grad[t, a]
            val = np.trapezoid(w @ (P[b] - P[a]), s)
            assert abs(val - 1.0) < 1e-12
