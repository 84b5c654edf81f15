"""Mesh topology for the A-V unknowns (oracle).

A lives on the edges of the triangulation (lowest-order Nedelec), V on the
nodes of the conducting sub-mesh (P1), cf. the discrete spaces of Section 3,
and on the nodes of impedance-boundary triangles (Eqs. 8-10, oracle/ibc.py).
Edges are the sorted node pairs (lo, hi), numbered in lexicographic order and
oriented from the lower to the higher global node id.  Conductor nodes are
numbered in increasing global id.  DOF order: [A on edges ; V on conductor
nodes].
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

LOCAL_EDGES = np.array([(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)])


@dataclass
class Topology:
    nv: int
    nt: int
    edges: np.ndarray        # int64 [ne, 2]  (lo, hi)
    tet2edge: np.ndarray     # int64 [nt, 6]
    sign: np.ndarray         # float64 [nt, 6]  +1 if local (a,b) runs lo->hi
    cond_tet: np.ndarray     # bool [nt]
    cond_nodes: np.ndarray   # int64 [nc]  global ids, increasing
    vmap: np.ndarray         # int64 [nv]  conductor index or -1
    comp: np.ndarray         # int64 [nc]  conductor component id
    ncomp: int

    @property
    def ne(self) -> int:
        return int(self.edges.shape[0])

    @property
    def nc(self) -> int:
        return int(self.cond_nodes.shape[0])

    @property
    def ndof(self) -> int:
        return self.ne + self.nc


def build(tet: np.ndarray, nv: int, region: np.ndarray, conductor_regions, faces=None) -> Topology:
    """faces: optional [nf, 3] surface-conductor triangles; their nodes carry V
    and they join conductor components like conducting tetrahedra."""
    tet = np.asarray(tet, dtype=np.int64)
    nt = tet.shape[0]
    pairs = tet[:, LOCAL_EDGES]                          # [nt, 6, 2] local (a, b)
    lo = np.minimum(pairs[..., 0], pairs[..., 1])
    hi = np.maximum(pairs[..., 0], pairs[..., 1])
    key = lo * nv + hi
    uniq, inv = np.unique(key.ravel(), return_inverse=True)
    edges = np.stack([uniq // nv, uniq % nv], axis=1)
    tet2edge = inv.reshape(nt, 6)
    sign = np.where(pairs[..., 0] < pairs[..., 1], 1.0, -1.0)

    cond_tet = np.isin(region, np.asarray(list(conductor_regions)))
    faces = np.zeros((0, 3), dtype=np.int64) if faces is None else np.asarray(faces, dtype=np.int64)
    cond_nodes = np.unique(np.concatenate([tet[cond_tet].ravel(), faces.ravel()]))
    vmap = -np.ones(nv, dtype=np.int64)
    vmap[cond_nodes] = np.arange(cond_nodes.size)

    # connected components of the conducting sub-mesh (tets and surface
    # triangles sharing a node)
    ct = tet[cond_tet]
    if ct.size or faces.size:
        loc, flo = vmap[ct], vmap[faces]
        rows = np.concatenate([np.repeat(loc[:, 0], 3), np.repeat(flo[:, 0], 2)])
        cols = np.concatenate([loc[:, 1:].ravel(), flo[:, 1:].ravel()])
        g = sp.coo_matrix((np.ones(rows.size), (rows, cols)), shape=(cond_nodes.size,) * 2)
        ncomp, comp = connected_components(g, directed=False)
    else:
        ncomp, comp = 0, np.zeros(0, dtype=np.int64)
    return Topology(nv, nt, edges, tet2edge, sign, cond_tet, cond_nodes, vmap,
                    np.asarray(comp, dtype=np.int64), int(ncomp))


def gradient_matrix(topo: Topology) -> sp.csr_matrix:
    """Edge-node incidence G [ne x nv]: (G phi)_e = phi(hi) - phi(lo)."""
    ne = topo.ne
    rows = np.repeat(np.arange(ne), 2)
    cols = topo.edges.ravel()
    vals = np.tile([-1.0, 1.0], ne)
    return sp.csr_matrix((vals, (rows, cols)), shape=(ne, topo.nv))


def curl_matrix(tet: np.ndarray, topo: Topology) -> sp.csr_matrix:
    """Face-edge incidence C [nf x ne] with faces as sorted node triples.

    (C a)_f is the circulation of a around face f, oriented by its sorted
    node order (n0 -> n1 -> n2 -> n0).  Integer-valued, used for the exact
    identity C G = 0.
    """
    tet = np.asarray(tet, dtype=np.int64)
    faces = np.sort(tet[:, [[0, 1, 2], [0, 1, 3], [0, 2, 3], [1, 2, 3]]].reshape(-1, 3), axis=1)
    nv = topo.nv
    fkey = (faces[:, 0] * nv + faces[:, 1]) * nv + faces[:, 2]
    fu, fi = np.unique(fkey, return_index=True)
    f = faces[fi]
    ekey = topo.edges[:, 0] * nv + topo.edges[:, 1]

    def eid(a, b):
        return np.searchsorted(ekey, np.minimum(a, b) * nv + np.maximum(a, b))

    n0, n1, n2 = f[:, 0], f[:, 1], f[:, 2]
    # boundary n0->n1 (+, lo->hi), n1->n2 (+), n2->n0 (-, since n0 < n2)
    rows = np.repeat(np.arange(f.shape[0]), 3)
    cols = np.stack([eid(n0, n1), eid(n1, n2), eid(n0, n2)], axis=1).ravel()
    vals = np.tile([1.0, 1.0, -1.0], f.shape[0])
    return sp.csr_matrix((vals, (rows, cols)), shape=(f.shape[0], topo.ne))
