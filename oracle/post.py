"""Derived quantities (oracle): V gauge fixing, E, B, impedance.

* V is fixed per conductor component by removing its mean weighted by the
  lumped conductor mass (the first option of Section 4: the integral of V
  over each connected conductor component is zero).
* E = i omega A + grad V (Eq. 2); on edges of conducting tetrahedra
  E_e = i omega A_e + V_hi - V_lo.
* B = mu H = curl A (Eq. 2); per tetrahedron sum_l s_l A_e(l) curl w_l.
* The impedance change caused by a defect (Section 2, Eq. 12) as a volume
  integral over the tetrahedra whose (nu, sigma) differ between the defect
  and the defect-free configuration.  With M_d, M_0 the two (complex
  symmetric) system matrices on one DOF space (V extended by 0 on nodes that
  conduct only in the defect configuration), b_l^T (x_k^d - x_k^0) =
  -x_l^0^T (M_d - M_0) x_k^d, and the sigma-part of x^T M y is
  (i / omega) int sigma E_x . E_y, hence
  dZ_kl = (1 / (I_k I_l)) [ i omega int dnu curl A_k^d . curl A_l^0
                            - int dsig E_k^d . E_l^0 ],
  the paper's reciprocity-type formula with the vacuum taken as sigma = 0.
* Coil impedance Z_kl = -(1 / (I_k I_l)) int E_k . J_l.  The coils lie in the
  insulator where E = i omega A, hence Z_kl = -(i omega / (I_k I_l)) b_l^T A_k
  with the unconjugated product (the paper's volume formula, Eq. 12, is a
  defect-region difference of such terms).
"""
from __future__ import annotations

import numpy as np

from .assemble import System
from .elements import element_matrices
from .topology import LOCAL_EDGES


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


def ect_signals(Z_defect, Z_free):
    """Signals of Eq. 11 from coil impedance matrices Z[p, k, l] (coil k in the
    field of coil l) with and without the defect:
    dZ = Z_defect - Z_free, Z_FA = (i/2)(dZ_11 + dZ_12), Z_F3 = (i/2)(dZ_11 - dZ_22).
    """
    dZ = np.asarray(Z_defect) - np.asarray(Z_free)
    fa = 0.5j * (dZ[:, 0, 0] + dZ[:, 0, 1])
    f3 = 0.5j * (dZ[:, 0, 0] - dZ[:, 1, 1])
    return dZ, fa, f3


def _local_fields(sysm: System, tet_d: np.ndarray, e6: np.ndarray, sg: np.ndarray, x: np.ndarray):
    """Local-orientation edge coefficients of E = i omega A + grad V and of A on
    the listed tetrahedra; V = 0 on nodes that are not conductor nodes."""
    topo = sysm.topo
    Vn = np.zeros(topo.nv, dtype=complex)
    cn = topo.vmap >= 0
    Vn[cn] = x[topo.ne + topo.vmap[cn]]
    Vt = Vn[tet_d]                                      # [nD, 4]
    A = sg * x[e6]                                      # [nD, 6]
    dV = Vt[:, LOCAL_EDGES[:, 1]] - Vt[:, LOCAL_EDGES[:, 0]]
    return 1j * sysm.omega * A + dV, A


def delta_z_volume(xyz, tet, region, sys_d: System, nu_d, sig_d, xs_d, sys_0: System, nu_0, sig_0, xs_0,
                   currents_k, currents_l) -> np.ndarray:
    """dZ[k, l] of Eq. 12 (module doc) from defect solutions xs_d[k] (DOFs of
    sys_d) and defect-free solutions xs_0[l] (DOFs of sys_0) on one mesh."""
    region = np.asarray(region)
    dnu = (np.asarray(nu_d, float) - np.asarray(nu_0, float))[region]
    dsig = (np.asarray(sig_d, float) - np.asarray(sig_0, float))[region]
    D = np.nonzero((dnu != 0) | (dsig != 0))[0]
    tet_d = np.asarray(tet, dtype=np.int64)[D]
    el = element_matrices(xyz, tet_d)
    e6 = sys_d.topo.tet2edge[D]
    sg = sys_d.topo.sign[D]
    dZ = np.zeros((len(xs_d), len(xs_0)), dtype=complex)
    for k, xd in enumerate(xs_d):
        Ed, Ad = _local_fields(sys_d, tet_d, e6, sg, xd)
        Bd = np.einsum("tl,tlx->tx", Ad, el["curl"])
        for l, x0 in enumerate(xs_0):
            E0, A0 = _local_fields(sys_0, tet_d, e6, sg, x0)
            B0 = np.einsum("tl,tlx->tx", A0, el["curl"])
            mag = np.sum(dnu[D] * el["vol"] * np.einsum("tx,tx->t", Bd, B0))
            ohm = np.sum(dsig[D] * np.einsum("ti,tij,tj->t", Ed, el["M"], E0))
            dZ[k, l] = (1j * sys_d.omega * mag - ohm) / (currents_k[k] * currents_l[l])
    return dZ
