"""Impedance boundary condition on the support plate (Section 2, Eqs. 8-10)
(oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Eq. 8 replaces the plate volume by a condition on its boundary Gamma_p:
n x (nu curl A) = -(1/Z)(i omega A_t + grad_t V), with the surface
impedance Z = (1 - i) / (delta sigma) and the skin depth
delta = sqrt(2 / (omega mu sigma)) of the plate.  Eqs. 9 and 10 are the
surface terms this adds to the weak forms of the A and V equations.

Reading (worked out here, the paper leaves the discrete form to its
references).  Take the test functions of the volume form (w_e for the A
rows; for the V rows grad l_n with the factor -1/(i omega) that makes the
volume system complex-symmetric).  The A-row surface term is
-(1/Z) int_G (i omega A_t + grad_G V) . w_e, and the V row of the plate,
whose normal current vanishes (the plate is surrounded by insulator), is
(1/Z) int_G (i omega A_t + grad_G V) . grad_G l_n = 0 (Eq. 10).  Both have
the structure of the volume conductor terms with sigma dV replaced by
(1/Z) dS on Gamma_p:

    M11 += -i omega (1/Z) M_G,   M12 = M21^T += -(1/Z) B_G,
    M22 += (i / omega) (1/Z) S_G,

M_G = int_G w_e . w_f, B_G = int_G w_e . grad_G l_n, S_G = int_G grad_G
l_m . grad_G l_n over the triangles of Gamma_p (tangential traces of the
Whitney functions, surface gradients of P1).  The normal of Eq. 8 is read
as pointing out of the computational domain, into the plate: with it the
real part of the surface term, (omega delta sigma / 2) M_G, is positive
like the magnetic energy in the skin layer it stands for, and the
imaginary part has the sign of the volume eddy-current term.  The surface
potential V lives on the nodes of Gamma_p; its constant per connected part
is removed like a conductor's, with area / 3 weights per node.

The same assembly with a real coefficient sigma * d is a conducting sheet
of thickness d (the thin-layer limit of a volume conductor), which is how
the surface terms are pinned against the volume ones.
"""
from __future__ import annotations

import numpy as np

FACE_EDGES = np.array([(0, 1), (0, 2), (1, 2)])
TET_FACES = np.array([(0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3)])


def surface_conductance(sigma, nu, omega):
    """1/Z of Eq. 8: Z = (1 - i)/(delta sigma), delta = sqrt(2 nu / (omega sigma))."""
    sigma = np.asarray(sigma, dtype=float)
    delta = np.sqrt(2.0 * np.asarray(nu, dtype=float) / (omega * sigma))
    return delta * sigma / (1.0 - 1j)


def split(xyz, tet, region, ibc_regions):
    """Remove the tetrahedra of ibc_regions and return the remaining mesh
    (nodes renumbered in increasing old id), the interface triangles
    Gamma_p (faces shared by a removed and a kept tetrahedron; node triples
    in increasing new id) with the region of the removed tetrahedron, and
    node_map[old] = new id or -1."""
    tet = np.asarray(tet, dtype=np.int64)
    region = np.asarray(region)
    gone = np.isin(region, np.asarray(list(ibc_regions)))
    keep = ~gone
    nv = xyz.shape[0]

    def faces_of(ts):
        f = np.sort(ts[:, TET_FACES].reshape(-1, 3), axis=1)
        return (f[:, 0] * nv + f[:, 1]) * nv + f[:, 2], f

    kk, _ = faces_of(tet[keep])
    gk, gf = faces_of(tet[gone])
    greg = np.repeat(region[gone], 4)
    on = np.isin(gk, kk)
    fkey, first = np.unique(gk[on], return_index=True)
    faces_old = gf[on][first]
    freg = greg[on][first]
    used = np.zeros(nv, dtype=bool)
    used[tet[keep].ravel()] = True
    node_map = -np.ones(nv, dtype=np.int64)
    node_map[used] = np.arange(int(used.sum()))
    return {"xyz": np.ascontiguousarray(xyz[used]), "tet": node_map[tet[keep]], "region": region[keep],
            "faces": node_map[faces_old], "face_region": freg, "node_map": node_map}


def face_geometry(xyz, faces):
    """Area [nf] and surface gradients of the barycentric coordinates
    [nf, 3, 3]: grad l_i = n x (p_(i+2) - p_(i+1)) / (2 area), n the unit
    normal of (p1 - p0) x (p2 - p0)."""
    p = xyz[np.asarray(faces)]
    c = np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0])
    two_a = np.linalg.norm(c, axis=1)
    n = c / two_a[:, None]
    grad = np.empty_like(p)
    for i in range(3):
        grad[:, i] = np.cross(n, p[:, (i + 2) % 3] - p[:, (i + 1) % 3]) / two_a[:, None]
    return two_a / 2.0, grad


def face_matrices(xyz, faces):
    """Per-triangle integrals with unit coefficient, for faces whose node
    ids increase (local edges (0,1), (0,2), (1,2), each oriented as the
    global edge):  M [nf,3,3] = int w_l . w_m,  B [nf,3,3] = int w_l . grad l_k,
    S [nf,3,3] = int grad l_i . grad l_j, area [nf].  Facts:
    int_T l_i l_j = |T| (1 + delta_ij) / 12, int_T l_i = |T| / 3."""
    area, grad = face_geometry(xyz, faces)
    a, b = FACE_EDGES[:, 0], FACE_EDGES[:, 1]
    G = np.einsum("fix,fjx->fij", grad, grad)
    L = area[:, None, None] * (np.ones((3, 3)) + np.eye(3))[None] / 12.0
    A_ = a[:, None]; B_ = b[:, None]; C_ = a[None, :]; D_ = b[None, :]
    M = (L[:, A_, C_] * G[:, B_, D_] - L[:, A_, D_] * G[:, B_, C_]
         - L[:, B_, C_] * G[:, A_, D_] + L[:, B_, D_] * G[:, A_, C_])
    F = (area[:, None, None] / 3.0) * (grad[:, b, :] - grad[:, a, :])     # int w_l
    B = np.einsum("flx,fkx->flk", F, grad)
    S = area[:, None, None] * G
    return {"area": area, "grad": grad, "M": M, "B": B, "S": S}
