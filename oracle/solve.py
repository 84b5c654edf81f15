"""Solvers for the A-V system (oracle).

* ``direct``: sparse LU (SuperLU through scipy, the solver family the paper
  factors its global matrix with, Section 4) or a dense solve for tiny
  systems.  With delta_V = 0 the matrix has one V-constant per conductor
  component in its kernel (V is defined up to a constant, Eq. 4); the
  system is consistent, so one V node per component is pinned to zero and
  the mass-weighted mean is removed afterwards (first option of Section 4).
* ``gmres``: restarted, right-preconditioned GMRES(m) on the symmetrically
  equilibrated system D^-1/2 M D^-1/2 y = D^-1/2 b (D = |diag M|), with
  classical Gram-Schmidt with a second pass whenever the first drops the
  norm below 1/sqrt(2) of its value ("twice is enough"), complex Givens
  rotations for the
  Hessenberg least-squares problem, and block-Jacobi preconditioning.  The
  stopping test is on the true equilibrated residual, i.e. the residual in
  the D^-1/2-weighted norm.
* ``solve_gmres``: the plain FP64 method.  The excitation must be
  divergence-free (Section 2, below Eq. 1); then, with delta_V = 0, the
  gauged system's solution has W^T A = 0, so the penalty term contributes
  nothing at the solution.  The Krylov iteration therefore runs on the
  operator without the penalty (singular, but consistent for such sources,
  its kernel being {(G psi, -i omega psi|_c)}) while the block-Jacobi blocks
  keep it (they must be invertible); the Coulomb gauge of Eq. 3 is then
  restored exactly by the discrete projection A <- A - G psi,
  V <- V + i omega psi|_c with (W^T G) psi = W^T A.  This returns the gauged
  system's solution.  For sources that are not divergence-free, or
  delta_V > 0, it iterates on the gauged operator instead.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .assemble import System
from .blocks import dof_coords, rcb_blocks


def equilibration(sysm: System) -> np.ndarray:
    """s = |diag M|^-1/2 per DOF."""
    return 1.0 / np.sqrt(np.abs(sysm.diag()))


def _pins(sysm: System) -> np.ndarray:
    topo = sysm.topo
    if sysm.delta_v != 0.0 or topo.nc == 0:
        return np.zeros(0, dtype=np.int64)
    first = np.full(topo.ncomp, -1, dtype=np.int64)
    for i in range(topo.nc - 1, -1, -1):
        first[topo.comp[i]] = i
    return topo.ne + first


def direct(sysm: System, b: np.ndarray, dense: bool = False) -> np.ndarray:
    """x = M^-1 b (one V pinned per component if delta_V = 0), means not removed.

    dense=True: numpy.linalg.solve on the explicit M (tiny meshes only).
    Otherwise SuperLU on the equivalent symmetric augmented system

        [ K - i w M_s   -B_s    W        ] [A ]   [b_A]
        [ -B_s^T         M22    0        ] [V ] = [b_V]
        [ W^T            0     -D0 / tau ] [p']   [ 0 ]

    whose elimination of p' = tau D0^-1 W^T A gives back M exactly; it keeps
    the factor sparse where the explicit gauge term would not.
    """
    n = sysm.ndof
    ne, nv = sysm.topo.ne, sysm.topo.nv
    pins = _pins(sysm)
    keep = np.setdiff1d(np.arange(n), pins)
    x = np.zeros(n, dtype=complex)
    if dense:
        M = sysm.matrix()
        x[keep] = np.linalg.solve(M[keep][:, keep].toarray(), b[keep])
        return x
    M11, M12, M22 = sysm.blocks_no_gauge()
    Wp = sysm.W.astype(complex)
    Aug = sp.bmat([[M11, M12, Wp],
                   [M12.T, M22, None],
                   [Wp.T, None, sp.diags(-sysm.D0 / sysm.tau).astype(complex)]], format="csc")
    keep_aug = np.concatenate([keep, n + np.arange(nv)])
    rhs = np.concatenate([b[keep], np.zeros(nv)]).astype(complex)
    sol = spla.splu(Aug[keep_aug][:, keep_aug].tocsc()).solve(rhs)
    x[keep] = sol[: keep.size]
    return x


@dataclass
class BlockJacobi:
    """z_I = (M_II)^-1 r_I over the RCB blocks, gauge included in M_II."""
    blocks: list
    inv: dict = field(default_factory=dict)     # size -> (block index array, inverses [k, s, s])

    @classmethod
    def build(cls, sysm: System, xyz: np.ndarray, b: int, scale: np.ndarray | None = None,
              tau_precond: float | None = None):
        topo = sysm.topo
        blocks = rcb_blocks(dof_coords(xyz, topo.edges, topo.cond_nodes), b)
        Mng = sysm.matrix_no_gauge().tocsr()
        ne = topo.ne
        Wc = sysm.W.tocsr()
        dinv = 1.0 / sysm.D0
        by_size: dict = {}
        for k, I in enumerate(blocks):
            Mb = Mng[I][:, I].toarray()
            Ia = I[I < ne]
            if Ia.size:
                Wi = Wc[Ia]
                G = (Wi @ sp.diags(dinv) @ Wi.T).toarray()
                na = Ia.size                              # A DOFs come first (sorted ids)
                Mb[:na, :na] += (sysm.tau if tau_precond is None else tau_precond) * G
            if scale is not None:
                Mb = scale[I][:, None] * Mb * scale[I][None, :]
            by_size.setdefault(I.size, []).append((k, Mb))
        inv = {}
        for s_, lst in by_size.items():
            idx = np.array([k for k, _ in lst])
            mats = np.stack([m for _, m in lst])
            inv[s_] = (idx, np.linalg.inv(mats))
        return cls(blocks, inv)

    def apply(self, r: np.ndarray) -> np.ndarray:
        z = np.zeros_like(r)
        for s_, (idx, Minv) in self.inv.items():
            I = np.stack([self.blocks[k] for k in idx])     # [k, s]
            z[I] = np.einsum("kij,kj->ki", Minv, r[I])
        return z


@dataclass
class GmresResult:
    x: np.ndarray
    iters: int
    restarts: int
    relres: float
    history: list
    converged: bool


def _givens(a: complex, b: complex):
    """(c, s, r) with [c s; -conj(s) c] [a; b] = [r; 0], c real."""
    if b == 0:
        return 1.0, 0.0 + 0.0j, a
    if a == 0:
        return 0.0, np.conj(b) / abs(b), abs(b)
    t = np.hypot(abs(a), abs(b))
    c = abs(a) / t
    s = (a / abs(a)) * np.conj(b) / t
    return c, s, (a / abs(a)) * t


def gmres(matvec, b: np.ndarray, precond, m: int = 30, tol: float = 1e-10, max_iter: int = 5000,
          x0: np.ndarray | None = None) -> GmresResult:
    """Right-preconditioned restarted GMRES(m), classical Gram-Schmidt with
    selective reorthogonalisation (plain, unblocked)."""
    n = b.size
    x = np.zeros(n, dtype=complex) if x0 is None else x0.astype(complex).copy()
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return GmresResult(x, 0, 0, 0.0, [0.0], True)
    r = b - matvec(x)
    beta = np.linalg.norm(r)
    hist = [beta / bnorm]
    it = 0
    restarts = 0
    while beta / bnorm > tol and it < max_iter:
        V = np.zeros((m + 1, n), dtype=complex)
        H = np.zeros((m + 1, m), dtype=complex)
        cs = np.zeros(m)
        sn = np.zeros(m, dtype=complex)
        g = np.zeros(m + 1, dtype=complex)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(m):
            w = matvec(precond(V[j]))
            w0 = np.linalg.norm(w)
            h1 = V[: j + 1].conj() @ w
            w = w - V[: j + 1].T @ h1
            hn = np.linalg.norm(w)
            h2 = np.zeros_like(h1)
            if hn < w0 / np.sqrt(2.0):
                h2 = V[: j + 1].conj() @ w
                w = w - V[: j + 1].T @ h2
                hn = np.linalg.norm(w)
            H[: j + 1, j] = h1 + h2
            H[j + 1, j] = hn
            if hn != 0.0:
                V[j + 1] = w / hn
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            c, s, rr = _givens(H[j, j], H[j + 1, j])
            cs[j], sn[j] = c, s
            H[j, j], H[j + 1, j] = rr, 0.0
            g[j + 1] = -np.conj(s) * g[j]
            g[j] = c * g[j]
            it += 1
            k = j + 1
            hist.append(abs(g[j + 1]) / bnorm)
            if abs(g[j + 1]) / bnorm <= tol or it >= max_iter or hn == 0.0:
                break
        y = np.zeros(k, dtype=complex)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:]) / H[i, i]
        x = x + precond(V[:k].T @ y)
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        restarts += 1
    return GmresResult(x, it, restarts, beta / bnorm, hist, beta / bnorm <= tol)


def divergence_residual(sysm: System, b: np.ndarray) -> float:
    """||G^T b_A|| / ||b||: zero (to rounding) for divergence-free currents."""
    from .topology import gradient_matrix
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(gradient_matrix(sysm.topo).T @ b[: sysm.topo.ne]) / nb) if nb else 0.0


def coulomb_projection(sysm: System, x: np.ndarray) -> np.ndarray:
    """Shift x along the kernel {(G psi, -i omega psi|_c)} so that W^T A = 0."""
    from .topology import gradient_matrix
    topo = sysm.topo
    G = gradient_matrix(topo)
    L = (sysm.W.T @ G).tocsc()                  # = G^T M_1 G, the P1 stiffness (Laplacian)
    rhs = sysm.W.T @ x[: topo.ne]
    keep = np.arange(1, topo.nv)                # constants are in the kernel of L: pin node 0
    psi = np.zeros(topo.nv, dtype=complex)
    psi[keep] = spla.spsolve(L[keep][:, keep], rhs[keep])
    y = x.copy()
    y[: topo.ne] -= G @ psi
    y[topo.ne:] += 1j * sysm.omega * psi[topo.cond_nodes]
    return y


def solve_gmres(sysm: System, xyz: np.ndarray, b: np.ndarray, block: int = 64, m: int = 30,
                tol: float = 1e-10, max_iter: int = 5000, gauge_in_operator: bool | None = None,
                tau_precond: float | None = None):
    """Plain FP64 method: equilibrate, block-Jacobi, GMRES(m); returns (x, result).

    gauge_in_operator=None picks the penalty-free iteration + Coulomb
    projection when delta_V = 0 and b is divergence-free (see module doc).
    The returned result's relres is the true weighted residual of the gauged
    system at the returned x.
    """
    s = equilibration(sysm)
    P = BlockJacobi.build(sysm, xyz, block, scale=s, tau_precond=tau_precond)
    if gauge_in_operator is None:
        gauge_in_operator = not (sysm.delta_v == 0.0 and divergence_residual(sysm, b) <= 1e-10)
    if gauge_in_operator:
        res = gmres(lambda v: s * sysm.matvec(s * v), s * b, P.apply, m=m, tol=tol, max_iter=max_iter)
        return s * res.x, res
    M0 = sysm.matrix_no_gauge()
    res = gmres(lambda v: s * (M0 @ (s * v)), s * b, P.apply, m=m, tol=tol, max_iter=max_iter)
    x = coulomb_projection(sysm, s * res.x)
    sb = s * b
    res.relres = float(np.linalg.norm(s * (b - sysm.matvec(x))) / np.linalg.norm(sb)) if np.any(sb) else 0.0
    res.converged = res.relres <= tol
    return x, res
