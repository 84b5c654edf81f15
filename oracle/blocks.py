"""Block partition of the DOFs for the block-Jacobi preconditioner (oracle).

The paper partitions the mesh with a graph partitioner only to distribute
assembly (Section 3); the preconditioner blocks here are this solver's own
definition, written out plainly so the GPU path's partition can be checked
against it bit for bit:

* DOF coordinates: edge midpoint (x_lo + x_hi) * 0.5 for an A DOF, node
  position for a V DOF;
* recursive coordinate bisection of a DOF set S (kept sorted by DOF id):
  nb = ceil(|S| / b); if nb <= 1 the set is one block; otherwise split along
  the axis of largest coordinate extent (lowest axis on ties) after a stable
  sort by (coordinate, DOF id), giving the first floor(|S| * floor(nb/2) / nb)
  DOFs to the left child; left child first;
* blocks are numbered in that depth-first order; inside a block DOFs are in
  increasing id.
"""
from __future__ import annotations

import numpy as np


def dof_coords(xyz: np.ndarray, edges: np.ndarray, cond_nodes: np.ndarray) -> np.ndarray:
    mid = (xyz[edges[:, 0]] + xyz[edges[:, 1]]) * 0.5
    return np.concatenate([mid, xyz[cond_nodes]], axis=0)


def rcb_blocks(coords: np.ndarray, b: int):
    """Return a list of int64 arrays (DOF ids per block)."""
    n = coords.shape[0]
    out = []
    stack = [np.arange(n, dtype=np.int64)]
    while stack:
        ids = stack.pop()
        m = ids.size
        nb = -(-m // b)
        if nb <= 1:
            out.append(ids)
            continue
        c = coords[ids]
        ext = c.max(axis=0) - c.min(axis=0)
        axis = int(np.argmax(ext))                      # first max on ties
        order = np.lexsort((ids, c[:, axis]))
        s = (m * (nb // 2)) // nb
        left = np.sort(ids[order[:s]])
        right = np.sort(ids[order[s:]])
        stack.append(right)                             # popped after left
        stack.append(left)
    return out
