"""Global assembly of the A-V system (oracle).

The discrete system of Section 3,

    [ M11  M12 ] [A]   [J_h]
    [ M21  M22 ] [V] = [ 0 ],

with the element forms of Eqs. 5-7 and the readings listed in the package
docstring:

    M11 = K_nu + tau * W D0^-1 W^T - i omega M_sigma
    M12 = -B_sigma,   M21 = -B_sigma^T
    M22 = (i / omega) S_sigma + delta_V N_sigma

K_nu = int nu curl w_e . curl w_f, M_sigma = int sigma w_e . w_f,
W = int w_e . grad l_n (all tetrahedra), B_sigma = int sigma w_e . grad l_n,
S_sigma = int sigma grad l_m . grad l_n, N_sigma = int sigma l_m l_n,
D0 = lumped P1 mass (|K|/4 per vertex).  The right-hand side is
int J . w_e for a current that is constant per tetrahedron.

Optional surface-conductor triangles with complex coefficients c_f (the
impedance boundary condition of Eqs. 8-10 has c_f = 1/Z, oracle/ibc.py)
add -i omega M_G, -B_G and (i/omega) S_G (coefficients included) to the
three blocks; their nodes carry V.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from .topology import Topology, build
from .elements import element_matrices
from .ibc import FACE_EDGES, face_matrices


def _coo(rows, cols, vals, shape) -> sp.csr_matrix:
    m = sp.coo_matrix((vals.ravel(), (rows.ravel(), cols.ravel())), shape=shape).tocsr()
    m.sum_duplicates()
    return m


@dataclass
class System:
    topo: Topology
    omega: float
    tau: float
    delta_v: float
    K: sp.csr_matrix        # ne x ne, real
    Msig: sp.csr_matrix     # ne x ne, real
    W: sp.csr_matrix        # ne x nv, real (all tets)
    Bsig: sp.csr_matrix     # ne x nc, real (conductor tets)
    Ssig: sp.csr_matrix     # nc x nc, real
    Nsig: sp.csr_matrix     # nc x nc, real
    D0: np.ndarray          # nv
    F: np.ndarray           # [nt, 6, 3] int w_l (global orientation)
    vol: np.ndarray
    lumped_c: np.ndarray    # nc, lumped conductor mass per conductor node (+ area/3 on surface nodes)
    Msurf: sp.csr_matrix = None   # ne x ne, complex: sum_f c_f int_f w_e . w_f
    Bsurf: sp.csr_matrix = None   # ne x nc, complex: sum_f c_f int_f w_e . grad l_n
    Ssurf: sp.csr_matrix = None   # nc x nc, complex: sum_f c_f int_f grad l_m . grad l_n

    @property
    def ndof(self) -> int:
        return self.topo.ndof

    def gauge(self) -> sp.csr_matrix:
        """tau * W D0^-1 W^T explicitly (ne x ne); only for small problems."""
        return (self.tau * (self.W @ sp.diags(1.0 / self.D0) @ self.W.T)).tocsr()

    def blocks_no_gauge(self):
        M11 = (self.K - 1j * self.omega * self.Msig).tocsr()
        M12 = (-self.Bsig).tocsr()
        M22 = ((1j / self.omega) * self.Ssig + self.delta_v * self.Nsig).tocsr()
        if self.Msurf is not None:
            M11 = (M11 - 1j * self.omega * self.Msurf).tocsr()
            M12 = (M12 - self.Bsurf).tocsr()
            M22 = (M22 + (1j / self.omega) * self.Ssurf).tocsr()
        return M11, M12, M22

    def matrix_no_gauge(self) -> sp.csr_matrix:
        """M without the factored gauge term (the stored CSR part)."""
        M11, M12, M22 = self.blocks_no_gauge()
        return sp.bmat([[M11, M12], [M12.T, M22]], format="csr")

    def matrix(self) -> sp.csr_matrix:
        """The full complex-symmetric M (gauge included explicitly)."""
        M11, M12, M22 = self.blocks_no_gauge()
        M11 = (M11 + self.gauge()).tocsr()
        return sp.bmat([[M11, M12], [M12.T, M22]], format="csr")

    def matvec(self, x: np.ndarray) -> np.ndarray:
        """y = M x with the gauge applied in factored form W (D0^-1 (W^T x_A))."""
        ne = self.topo.ne
        if not hasattr(self, "_Mng"):
            self._Mng = self.matrix_no_gauge()
        y = self._Mng @ x
        xa = x[:ne]
        y[:ne] += self.tau * (self.W @ ((self.W.T @ xa) / self.D0))
        return y

    def diag(self) -> np.ndarray:
        """diag M (complex), gauge diagonal tau sum_n W_en^2 / D0_n included."""
        ne = self.topo.ne
        d = np.empty(self.ndof, dtype=complex)
        Wsq = self.W.multiply(self.W)
        d[:ne] = self.K.diagonal() - 1j * self.omega * self.Msig.diagonal() + self.tau * (Wsq @ (1.0 / self.D0))
        d[ne:] = (1j / self.omega) * self.Ssig.diagonal() + self.delta_v * self.Nsig.diagonal()
        if self.Msurf is not None:
            d[:ne] -= 1j * self.omega * self.Msurf.diagonal()
            d[ne:] += (1j / self.omega) * self.Ssurf.diagonal()
        return d

    def rhs(self, J: np.ndarray) -> np.ndarray:
        """b = [int J . w_e ; 0] for a per-tetrahedron constant current J[nt, 3]."""
        ne = self.topo.ne
        contrib = np.einsum("tlx,tx->tl", self.F, J)
        b = np.zeros(self.ndof, dtype=complex)
        b[:ne] = np.bincount(self.topo.tet2edge.ravel(), weights=contrib.ravel(), minlength=ne)
        return b


def assemble(xyz, tet, region, nu, sigma, omega, tau=1.0, delta_v=0.0, conductor_regions=None,
             faces=None, face_coef=None) -> System:
    """Assemble the A-V system on the mesh with per-region nu (=1/mu) and
    sigma; faces [nf, 3] (node ids, any order) with complex face_coef [nf]
    are surface conductors."""
    tet = np.asarray(tet, dtype=np.int64)
    region = np.asarray(region)
    nu = np.asarray(nu, dtype=float)
    sigma = np.asarray(sigma, dtype=float)
    if conductor_regions is None:
        conductor_regions = [r for r in range(sigma.size) if sigma[r] > 0]
    if faces is not None:
        faces = np.sort(np.asarray(faces, dtype=np.int64), axis=1)
        face_coef = np.asarray(face_coef, dtype=complex)
    topo = build(tet, xyz.shape[0], region, conductor_regions, faces)
    ne, nv, nc = topo.ne, topo.nv, topo.nc
    el = element_matrices(xyz, tet)
    s = topo.sign                                       # [nt, 6]
    ss = s[:, :, None] * s[:, None, :]
    nuK = nu[region]
    sgK = sigma[region]
    e = topo.tet2edge
    er = np.broadcast_to(e[:, :, None], (tet.shape[0], 6, 6))
    ec = np.broadcast_to(e[:, None, :], (tet.shape[0], 6, 6))
    K = _coo(er, ec, nuK[:, None, None] * ss * el["K"], (ne, ne))
    Msig = _coo(er, ec, sgK[:, None, None] * ss * el["M"], (ne, ne))
    # W over all tetrahedra (gauge); B_sigma over conductor tetrahedra
    wr = np.broadcast_to(e[:, :, None], (tet.shape[0], 6, 4))
    wc = np.broadcast_to(tet[:, None, :], (tet.shape[0], 6, 4))
    Ws = s[:, :, None] * el["W"]
    W = _coo(wr, wc, Ws, (ne, nv))
    ct = topo.cond_tet
    vloc = topo.vmap[tet[ct]]                           # conductor-local node ids
    Bsig = _coo(wr[ct], np.broadcast_to(vloc[:, None, :], (vloc.shape[0], 6, 4)),
                sgK[ct][:, None, None] * Ws[ct], (ne, nc))
    vr = np.broadcast_to(vloc[:, :, None], (vloc.shape[0], 4, 4))
    vc = np.broadcast_to(vloc[:, None, :], (vloc.shape[0], 4, 4))
    Ssig = _coo(vr, vc, sgK[ct][:, None, None] * el["S"][ct], (nc, nc))
    Nsig = _coo(vr, vc, sgK[ct][:, None, None] * el["N"][ct], (nc, nc))
    D0 = np.bincount(tet.ravel(), weights=np.repeat(el["vol"] / 4.0, 4), minlength=nv)
    lumped_c = np.bincount(vloc.ravel(), weights=np.repeat(el["vol"][ct] / 4.0, 4), minlength=nc)
    F = s[:, :, None] * el["F"]
    sysm = System(topo, float(omega), float(tau), float(delta_v), K, Msig, W, Bsig, Ssig, Nsig,
                  D0, F, el["vol"], lumped_c)
    if faces is not None and faces.shape[0]:
        fm = face_matrices(xyz, faces)
        ekey = topo.edges[:, 0] * nv + topo.edges[:, 1]
        fe = faces[:, FACE_EDGES]                                   # [nf, 3, 2], lo < hi
        fkey = fe[..., 0] * nv + fe[..., 1]
        f2e = np.searchsorted(ekey, fkey)
        if np.any(f2e >= ne) or np.any(ekey[np.minimum(f2e, ne - 1)] != fkey):
            raise ValueError("a surface triangle edge is not an edge of the mesh")
        nf = faces.shape[0]
        c = face_coef[:, None, None]
        r3 = np.broadcast_to(f2e[:, :, None], (nf, 3, 3))
        c3 = np.broadcast_to(f2e[:, None, :], (nf, 3, 3))
        fv = topo.vmap[faces]
        sysm.Msurf = _coo(r3, c3, c * fm["M"], (ne, ne))
        sysm.Bsurf = _coo(r3, np.broadcast_to(fv[:, None, :], (nf, 3, 3)), c * fm["B"], (ne, nc))
        sysm.Ssurf = _coo(np.broadcast_to(fv[:, :, None], (nf, 3, 3)), np.broadcast_to(fv[:, None, :], (nf, 3, 3)),
                          c * fm["S"], (nc, nc))
        sysm.lumped_c = lumped_c + np.bincount(fv.ravel(), weights=np.repeat(fm["area"] / 3.0, 3), minlength=nc)
    return sysm
