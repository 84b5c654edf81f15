"""Derived quantities (oracle): V gauge fixing, E, B, impedance.

* V is fixed per conductor component by removing its mean weighted by the
  lumped conductor mass (the first option of Section 4: the integral of V
  over each connected conductor component is zero).
* E = i omega A + grad V (Eq. 2); on edges of conducting tetrahedra
  E_e = i omega A_e + V_hi - V_lo.
* B = mu H = curl A (Eq. 2); per tetrahedron sum_l s_l A_e(l) curl w_l.
* Coil impedance Z_kl = -(1 / (I_k I_l)) int E_k . J_l.  The coils lie in the
  insulator where E = i omega A, hence Z_kl = -(i omega / (I_k I_l)) b_l^T A_k
  with the unconjugated product (the paper's volume formula, Eq. 12, is a
  defect-region difference of such terms).
"""
from __future__ import annotations

import numpy as np

from .assemble import System
from .elements import element_matrices


def remove_v_mean(sysm: System, x: np.ndarray) -> np.ndarray:
    topo = sysm.topo
    x = x.copy()
    if topo.nc == 0:
        return x
    V = x[topo.ne:]
    w = sysm.lumped_c
    num = np.bincount(topo.comp, weights=w * V.real, minlength=topo.ncomp) \
        + 1j * np.bincount(topo.comp, weights=w * V.imag, minlength=topo.ncomp)
    den = np.bincount(topo.comp, weights=w, minlength=topo.ncomp)
    x[topo.ne:] = V - (num / den)[topo.comp]
    return x


def edge_field(sysm: System, x: np.ndarray) -> np.ndarray:
    """E on edges: i omega A_e, plus V_hi - V_lo on edges of conducting tets."""
    topo = sysm.topo
    A = x[: topo.ne]
    V = x[topo.ne:]
    E = 1j * sysm.omega * A
    ce = np.unique(topo.tet2edge[topo.cond_tet])
    lo, hi = topo.edges[ce, 0], topo.edges[ce, 1]
    E[ce] += V[topo.vmap[hi]] - V[topo.vmap[lo]]
    return E


def curl_per_tet(sysm: System, xyz: np.ndarray, tet: np.ndarray, A: np.ndarray) -> np.ndarray:
    """B_K = curl A_h on each tetrahedron, [nt, 3] complex."""
    el = element_matrices(xyz, tet)
    coef = sysm.topo.sign * A[sysm.topo.tet2edge]        # [nt, 6]
    return np.einsum("tl,tlx->tx", coef, el["curl"])


def joule_loss(sysm: System, x: np.ndarray) -> float:
    """int sigma |E_h|^2 over the conductor, = E^H M_sigma E."""
    E = edge_field(sysm, x)
    return float(np.real(np.conj(E) @ (sysm.Msig @ E)))


def impedance(sysm: System, rhs_list, sol_list, currents) -> np.ndarray:
    """Z[k, l] = -(i omega / (I_k I_l)) b_l^T A_k."""
    ne = sysm.topo.ne
    n = len(rhs_list)
    Z = np.zeros((n, n), dtype=complex)
    for k in range(n):
        for l in range(n):
            Z[k, l] = -1j * sysm.omega / (currents[k] * currents[l]) * (rhs_list[l][:ne] @ sol_list[k][:ne])
    return Z
