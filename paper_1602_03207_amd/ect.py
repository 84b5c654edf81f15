"""Eddy-current testing scan on the GPU path (Section 3, the per-position
solve and the impedance record; Section 2, Eqs. 11 and 12).

One operator per configuration (with and without the defect) serves every
probe position, since the matrix does not depend on where the probe is; only
the right-hand sides change.  Positions are solved in batches with the
batched multi-RHS GMRES, two coils per position.  For each position the
record holds the 2x2 coil impedance matrices of both configurations, the
change dZ as the defect-volume integral of Eq. 12 (eddy_delta_z_volume), the
plain difference Z_defect - Z_free beside it, and the signals Z_FA and Z_F3
of Eq. 11 computed from the volume form.

Records are appended, one JSON line per position, to an optional log file; a
rerun with the same log and configuration skips the positions already there
(checkpoint and resume of a long scan).
"""
from __future__ import annotations

import json
import os
import time
from dataclasses import dataclass, field

import numpy as np

from . import eddy


def _cplx(a):
    a = np.asarray(a, dtype=np.complex128)
    return np.stack([a.real, a.imag], axis=-1).tolist()


def _uncplx(v):
    a = np.asarray(v, dtype=np.float64)
    return a[..., 0] + 1j * a[..., 1]


@dataclass
class ScanResult:
    z: np.ndarray                      # [npos] probe positions
    Z_defect: np.ndarray               # [npos, 2, 2]
    Z_free: np.ndarray                 # [npos, 2, 2]
    dZ: np.ndarray                     # [npos, 2, 2] defect-volume form (Eq. 12)
    dZ_diff: np.ndarray                # [npos, 2, 2] Z_defect - Z_free
    Z_FA: np.ndarray                   # [npos] absolute signal (Eq. 11)
    Z_F3: np.ndarray                   # [npos] differential signal (Eq. 11)
    iters: np.ndarray                  # [npos, 2 configurations (defect, free), 2 coils]
    converged: np.ndarray              # [npos, 2, 2] bool
    solved: int = 0                    # positions solved in this run (the rest came from the log)
    seconds: float = 0.0               # wall time of this run's solves
    timings: dict = field(default_factory=dict)


class EctScan:
    """Two operators (defect, defect-free) on one geometry.

    nu_*, sigma_*: per-region values of the two configurations; a region
    conducts in a configuration where its sigma is > 0 there.  delta_V is 0
    (V fixed by its mean per conductor component), as the batched solver
    requires.
    """

    def __init__(self, xyz, tet, region, nu_defect, sigma_defect, nu_free, sigma_free, omega: float, tau: float,
                 block_size: int = 64, tau_precond: float = 0.0, device="cuda"):
        self.nu_d = np.asarray(nu_defect, dtype=np.float64)
        self.sig_d = np.asarray(sigma_defect, dtype=np.float64)
        self.nu_0 = np.asarray(nu_free, dtype=np.float64)
        self.sig_0 = np.asarray(sigma_free, dtype=np.float64)
        if not (self.nu_d.shape == self.sig_d.shape == self.nu_0.shape == self.sig_0.shape):
            raise ValueError("per-region arrays must have one length")
        if np.array_equal(self.nu_d, self.nu_0) and np.array_equal(self.sig_d, self.sig_0):
            raise ValueError("the two configurations are identical")
        self.omega = float(omega)
        self.nt = int(np.asarray(tet).shape[0])
        self.mesh_d = eddy.Mesh(xyz, tet, region, (self.sig_d > 0).astype(np.int32))
        self.mesh_0 = eddy.Mesh(xyz, tet, region, (self.sig_0 > 0).astype(np.int32))
        self.op_d = eddy.Operator(self.mesh_d, tau=tau, block_size=block_size, device=device, tau_precond=tau_precond)
        self.op_0 = eddy.Operator(self.mesh_0, tau=tau, block_size=block_size, device=device, tau_precond=tau_precond)
        self.op_d.assemble(self.nu_d, self.sig_d, self.omega)
        self.op_0.assemble(self.nu_0, self.sig_0, self.omega)
        self.device = self.op_d.device

    def _header(self, currents, tol, precision):
        return {"kind": "ect_scan", "nt": self.nt, "ndof_defect": self.op_d.ndof, "ndof_free": self.op_0.ndof,
                "omega": self.omega, "nu_defect": self.nu_d.tolist(), "sigma_defect": self.sig_d.tolist(),
                "nu_free": self.nu_0.tolist(), "sigma_free": self.sig_0.tolist(),
                "currents": [float(c) for c in currents], "tol": float(tol), "precision": precision}

    @staticmethod
    def _read_log(path, header):
        done = {}
        if not path or not os.path.exists(path):
            return done
        with open(path) as f:
            lines = [ln for ln in f.read().splitlines() if ln.strip()]
        if not lines:
            return done
        h = json.loads(lines[0])
        if h != header:
            raise ValueError(f"{path} was written for another scan configuration")
        for ln in lines[1:]:
            try:
                r = json.loads(ln)
            except json.JSONDecodeError:        # a record cut off by an interrupted run
                continue
            done[float(r["z"])] = r
        return done

    def run(self, positions, sources, currents=(1.0, 1.0), tol=1e-8, restart=48, max_iter=20000,
            precision="mixed", batch=8, log=None) -> ScanResult:
        """positions: probe positions; sources(z) -> (J1, J2), per-tetrahedron
        coil currents [nt, 3] (host or device, float64) carrying currents[0]
        and currents[1] amperes; batch: right-hand sides per batched solve
        (two per position)."""
        import torch
        z_all = [float(z) for z in positions]
        cur = np.asarray(currents, dtype=np.float64)
        if cur.shape != (2,):
            raise ValueError("two coil currents")
        header = self._header(cur, tol, precision)
        done = self._read_log(log, header)
        todo = [z for z in z_all if z not in done]
        per = max(1, int(batch) // 2)
        t_solve = 0.0
        fh = None
        if log:
            new = not os.path.exists(log) or os.path.getsize(log) == 0
            fh = open(log, "a")
            if new:
                fh.write(json.dumps(header) + "\n")
                fh.flush()
        try:
            for i0 in range(0, len(todo), per):
                zs = todo[i0:i0 + per]
                Js = []
                for z in zs:
                    for J in sources(z):
                        Js.append(torch.as_tensor(J, dtype=torch.float64).to(self.device).contiguous())
                if len(Js) != 2 * len(zs):
                    raise ValueError("sources(z) must return two coil currents")
                Bd = torch.stack([self.op_d.rhs_from_current(J) for J in Js])
                B0 = torch.stack([self.op_0.rhs_from_current(J) for J in Js])
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                Xd, rd = self.op_d.solve_batched(Bd, tol=tol, restart=restart, max_iter=max_iter, precision=precision)
                X0, r0 = self.op_0.solve_batched(B0, tol=tol, restart=restart, max_iter=max_iter, precision=precision)
                torch.cuda.synchronize()
                t_solve += time.perf_counter() - t0
                for j, z in enumerate(zs):
                    sl = slice(2 * j, 2 * j + 2)
                    Zd = self.op_d.impedance(Xd[sl], Bd[sl], cur)
                    Z0 = self.op_0.impedance(X0[sl], B0[sl], cur)
                    dZ = eddy.delta_z_volume(self.op_d, Xd[sl], self.op_0, X0[sl], cur, cur)
                    _, fa, f3 = eddy.ect_signals(dZ[None])
                    rec = {"z": z, "Z_defect": _cplx(Zd), "Z_free": _cplx(Z0), "dZ": _cplx(dZ),
                           "dZ_diff": _cplx(Zd - Z0), "Z_FA": _cplx(fa[0]), "Z_F3": _cplx(f3[0]),
                           "iters": [[rd[2 * j].iters, rd[2 * j + 1].iters], [r0[2 * j].iters, r0[2 * j + 1].iters]],
                           "converged": [[rd[2 * j].converged, rd[2 * j + 1].converged],
                                         [r0[2 * j].converged, r0[2 * j + 1].converged]]}
                    done[z] = rec
                    if fh:
                        fh.write(json.dumps(rec) + "\n")
                        fh.flush()
                        os.fsync(fh.fileno())
        finally:
            if fh:
                fh.close()
        recs = [done[z] for z in z_all]
        res = ScanResult(
            z=np.array(z_all),
            Z_defect=np.array([_uncplx(r["Z_defect"]) for r in recs]).reshape(-1, 2, 2),
            Z_free=np.array([_uncplx(r["Z_free"]) for r in recs]).reshape(-1, 2, 2),
            dZ=np.array([_uncplx(r["dZ"]) for r in recs]).reshape(-1, 2, 2),
            dZ_diff=np.array([_uncplx(r["dZ_diff"]) for r in recs]).reshape(-1, 2, 2),
            Z_FA=np.array([_uncplx(r["Z_FA"]) for r in recs]).reshape(-1),
            Z_F3=np.array([_uncplx(r["Z_F3"]) for r in recs]).reshape(-1),
            iters=np.array([r["iters"] for r in recs], dtype=np.int64).reshape(-1, 2, 2),
            converged=np.array([r["converged"] for r in recs], dtype=bool).reshape(-1, 2, 2),
            solved=len(todo), seconds=t_solve)
        return res
