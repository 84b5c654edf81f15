"""Closed-form element integrals on one tetrahedron (oracle).

These are the element-level pieces of the variational forms L11, L12, L21,
L22 of Section 2 (Eqs. 5-7) and Section 3, for lowest-order Nedelec
(Whitney) functions w = l_a grad(l_b) - l_b grad(l_a) on the local edge
(a, b) and P1 functions l_i (barycentric coordinates).  Facts used:

* int_K l_i l_j = |K| (1 + delta_ij) / 20,  int_K l_i = |K| / 4;
* curl w_(a,b) = 2 grad(l_a) x grad(l_b);
* grad(l_1..3) are the columns of E^-1, E having rows p_i - p_0;
  grad(l_0) = -(grad l_1 + grad l_2 + grad l_3).

All quantities are for the LOCAL edge orientation (a -> b); the global
orientation sign is applied at assembly.
"""
from __future__ import annotations

import numpy as np

from .topology import LOCAL_EDGES


def geometry(xyz: np.ndarray, tet: np.ndarray):
    """Return (vol[nt], grad[nt, 4, 3], signed det[nt])."""
    p = xyz[np.asarray(tet)]
    E = p[:, 1:, :] - p[:, :1, :]
    det = np.linalg.det(E)
    Einv = np.linalg.inv(E)
    grad = np.empty((p.shape[0], 4, 3))
    grad[:, 1:, :] = np.transpose(Einv, (0, 2, 1))      # grad l_i = column i of E^-1
    grad[:, 0, :] = -grad[:, 1:, :].sum(axis=1)
    return np.abs(det) / 6.0, grad, det


def lambda_mass(vol: np.ndarray) -> np.ndarray:
    """int_K l_i l_j = |K| (1 + delta_ij)/20, shape [nt, 4, 4]."""
    return vol[:, None, None] * (np.ones((4, 4)) + np.eye(4))[None] / 20.0


def element_matrices(xyz: np.ndarray, tet: np.ndarray):
    """Per-tetrahedron element integrals (unit coefficients).

    Returns a dict of arrays:
      vol  [nt]        |K|
      grad [nt,4,3]    grad l_i
      K    [nt,6,6]    int curl w_l . curl w_m
      M    [nt,6,6]    int w_l . w_m
      W    [nt,6,4]    int w_l . grad l_k
      S    [nt,4,4]    int grad l_i . grad l_j
      N    [nt,4,4]    int l_i l_j
      F    [nt,6,3]    int w_l  (vector), so int J . w_l = J . F_l for constant J
    """
    vol, grad, _ = geometry(xyz, tet)
    a, b = LOCAL_EDGES[:, 0], LOCAL_EDGES[:, 1]
    ga, gb = grad[:, a, :], grad[:, b, :]               # [nt, 6, 3]
    curl = 2.0 * np.cross(ga, gb)
    K = vol[:, None, None] * np.einsum("tlx,tmx->tlm", curl, curl)
    G = np.einsum("tix,tjx->tij", grad, grad)           # grad l_i . grad l_j
    L = lambda_mass(vol)                                # int l_i l_j
    # int (l_a g_b - l_b g_a).(l_c g_d - l_d g_c)
    A_ = a[:, None]; B_ = b[:, None]; C_ = a[None, :]; D_ = b[None, :]
    M = (L[:, A_, C_] * G[:, B_, D_] - L[:, A_, D_] * G[:, B_, C_]
         - L[:, B_, C_] * G[:, A_, D_] + L[:, B_, D_] * G[:, A_, C_])
    F = (vol[:, None, None] / 4.0) * (gb - ga)          # int w_l
    W = np.einsum("tlx,tkx->tlk", F, grad)
    S = vol[:, None, None] * G
    return {"vol": vol, "grad": grad, "K": K, "M": M, "W": W, "S": S, "N": L, "F": F, "curl": curl}
