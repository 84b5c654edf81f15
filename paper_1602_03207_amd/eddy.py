"""Python binding of libeddy.so (argument marshalling only).

Every step of the solver runs in the HIP library; this module only turns
numpy arrays and torch device tensors into the plain pointers of the C ABI
(include/eddy.h), allocates the device workspaces as torch tensors and passes
torch's current HIP stream.  If the library is missing the import fails.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libeddy.so")


class EddyError(RuntimeError):
    pass


class _Params(C.Structure):
    _fields_ = [("tau_gauge", C.c_double), ("delta_v", C.c_double), ("block_size", C.c_int32),
                ("tau_precond", C.c_double)]


class _Opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("restart", C.c_int32), ("max_iter", C.c_int32), ("precision", C.c_int32),
                ("gnn_theta", C.c_void_p), ("graph", C.c_int32)]


class _Tuning(C.Structure):
    _fields_ = [("spmv_grid_full", C.c_int32), ("spmv_grid_c128", C.c_int32), ("spmv_grid_c64", C.c_int32),
                ("spmv_sched_c128", C.c_int32), ("spmv_sched_c64", C.c_int32),
                ("spmv_us_c128", C.c_float), ("spmv_us_c64", C.c_float),
                ("spmv_us_sched_c128", C.c_float * 2), ("spmv_us_sched_c64", C.c_float * 2),
                ("sell_nnz_real", C.c_int64)]


class _Report(C.Structure):
    _fields_ = [("iters", C.c_int32), ("restarts", C.c_int32), ("converged", C.c_int32),
                ("breakdown", C.c_int32), ("relres", C.c_double), ("est_relres", C.c_double),
                ("seconds", C.c_double), ("gauge_in_operator", C.c_int32), ("cg_iters", C.c_int32),
                ("div_residual", C.c_double), ("precision_used", C.c_int32), ("reorth_steps", C.c_int32),
                ("learned_cycles", C.c_int32), ("fell_back", C.c_int32)]


EXPORTS = [
    "eddy_mesh_create", "eddy_mesh_create_ibc", "eddy_ibc_split", "eddy_mesh_destroy", "eddy_mesh_counts", "eddy_mesh_edges",
    "eddy_mesh_conductor_nodes", "eddy_mesh_blocks", "eddy_op_workspace_bytes", "eddy_op_create",
    "eddy_op_destroy", "eddy_op_assemble", "eddy_rhs_from_current", "eddy_solve_workspace_bytes",
    "eddy_solve", "eddy_solve_batched_workspace_bytes", "eddy_solve_batched",
    "eddy_solve_multifreq_workspace_bytes", "eddy_solve_multifreq", "eddy_impedance", "eddy_delta_z_volume",
    "eddy_ect_signals", "eddy_edge_field", "eddy_spmv", "eddy_precond_apply", "eddy_export", "eddy_profile", "eddy_op_tuning",
    "eddy_mesh_subdomains", "eddy_gnn_static_features", "eddy_gnn_scratch_bytes", "eddy_gnn_pair",
    "eddy_gnn_forward", "eddy_gnn_train_step",
    "eddy_status_string", "eddy_last_error",
]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_1602_03207_amd.build.build()")
    lib = C.CDLL(LIB_PATH)
    P, I32, I64, D, VP = C.POINTER, C.c_int32, C.c_int64, C.c_double, C.c_void_p
    sig = {
        "eddy_mesh_create": [I64, P(D), I64, P(I32), P(I32), I32, P(I32), P(VP)],
        "eddy_mesh_create_ibc": [I64, P(D), I64, P(I32), P(I32), I32, P(I32), I64, P(I32), P(I32), P(VP)],
        "eddy_ibc_split": [I64, P(D), I64, P(I32), P(I32), I32, P(I32), P(I64), P(I64), P(I64), P(D), P(I32), P(I32),
                           P(I32), P(I32), P(I32)],
        "eddy_mesh_destroy": [VP],
        "eddy_mesh_counts": [VP, P(I64), P(I64), P(I64), P(I64), P(I32)],
        "eddy_mesh_edges": [VP, P(I32)],
        "eddy_mesh_conductor_nodes": [VP, P(I32)],
        "eddy_mesh_blocks": [VP, I32, P(I64), P(I32), P(I32)],
        "eddy_op_workspace_bytes": [VP, P(_Params), P(C.c_size_t)],
        "eddy_op_create": [VP, P(_Params), VP, C.c_size_t, VP, P(VP)],
        "eddy_op_destroy": [VP],
        "eddy_op_assemble": [VP, P(D), P(D), D, VP],
        "eddy_rhs_from_current": [VP, VP, VP, VP],
        "eddy_solve_workspace_bytes": [VP, P(_Opts), P(C.c_size_t)],
        "eddy_solve": [VP, VP, VP, P(_Opts), VP, C.c_size_t, P(_Report), VP],
        "eddy_solve_batched_workspace_bytes": [VP, I32, P(_Opts), P(C.c_size_t)],
        "eddy_solve_batched": [VP, I32, VP, VP, P(_Opts), VP, C.c_size_t, P(_Report), VP],
        "eddy_solve_multifreq_workspace_bytes": [P(VP), I32, I32, P(_Opts), P(C.c_size_t)],
        "eddy_solve_multifreq": [P(VP), I32, I32, P(I32), VP, VP, P(_Opts), VP, C.c_size_t, P(_Report), VP],
        "eddy_impedance": [VP, I32, VP, I32, VP, P(D), P(D), VP],
        "eddy_delta_z_volume": [VP, I32, VP, VP, I32, VP, P(D), P(D), P(D), VP],
        "eddy_ect_signals": [I32, P(D), P(D), P(D), P(D), P(D)],
        "eddy_edge_field": [VP, VP, VP, VP],
        "eddy_spmv": [VP, VP, VP, VP],
        "eddy_precond_apply": [VP, VP, VP, VP],
        "eddy_export": [VP, P(I32), P(I32), P(D), P(I32), P(I32), P(D), P(D), P(D), VP],
        "eddy_profile": [VP, I32, P(D), P(I64)],
        "eddy_op_tuning": [VP, P(_Tuning)],
        "eddy_mesh_subdomains": [VP, I32, P(I32), P(I32)],
        "eddy_gnn_static_features": [VP, P(C.c_float)],
        "eddy_gnn_scratch_bytes": [I32, P(C.c_size_t)],
        "eddy_gnn_pair": [VP, VP, VP, VP, VP, VP, VP, VP],
        "eddy_gnn_forward": [VP, I32, VP, VP, VP, VP, C.c_size_t, VP],
        "eddy_gnn_train_step": [VP, I32, VP, VP, VP, VP, VP, VP, I32, C.c_float, VP, VP, VP, C.c_size_t, VP],
        "eddy_status_string": [I32],
        "eddy_last_error": [],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = C.c_int32
    lib.eddy_mesh_destroy.restype = None
    lib.eddy_op_destroy.restype = None
    lib.eddy_status_string.restype = C.c_char_p
    lib.eddy_last_error.restype = C.c_char_p
    return lib


_lib = _load()


def _check(status: int, what: str) -> int:
    if status < 0:
        msg = _lib.eddy_last_error().decode()
        raise EddyError(f"{what}: {_lib.eddy_status_string(status).decode()} ({msg})")
    return status


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t):
    return C.c_void_p(t.data_ptr())


GNN_P, GNN_FIN, GNN_FOUT, GNN_PARAMS = 64, 16, 16, 10448


def ect_signals(Z_defect, Z_free=None):
    """(dZ [npos,2,2], Z_FA [npos], Z_F3 [npos]) from per-position 2x2 coil impedance
    matrices with and without the defect (eddy_ect_signals); Z_free=None takes
    Z_defect as the change dZ itself."""
    Zd = np.ascontiguousarray(np.asarray(Z_defect, dtype=np.complex128).reshape(-1, 2, 2))
    Z0 = None
    if Z_free is not None:
        Z0 = np.ascontiguousarray(np.asarray(Z_free, dtype=np.complex128).reshape(-1, 2, 2))
        if Zd.shape != Z0.shape:
            raise ValueError("Z_defect and Z_free shapes differ")
    npos = Zd.shape[0]
    dZ = np.empty_like(Zd)
    fa = np.empty(npos, np.complex128)
    f3 = np.empty(npos, np.complex128)
    D = C.POINTER(C.c_double)
    _check(_lib.eddy_ect_signals(npos, Zd.ctypes.data_as(D), None if Z0 is None else Z0.ctypes.data_as(D),
                                 dZ.ctypes.data_as(D), fa.ctypes.data_as(D), f3.ctypes.data_as(D)),
           "eddy_ect_signals")
    return dZ, fa, f3


def delta_z_volume(op_defect, x_defect, op_free, x_free, currents_k, currents_l):
    """dZ[k, l] as the defect-region volume integral (eddy_delta_z_volume).

    x_defect: [nk, op_defect.ndof], x_free: [nl, op_free.ndof] complex128 device
    solutions of the two configurations on one geometry."""
    xd = x_defect.reshape(-1, op_defect.ndof).contiguous()
    x0 = x_free.reshape(-1, op_free.ndof).contiguous()
    ck = np.ascontiguousarray(currents_k, dtype=np.float64)
    cl = np.ascontiguousarray(currents_l, dtype=np.float64)
    if ck.size != xd.shape[0] or cl.size != x0.shape[0]:
        raise ValueError("one current per solution")
    dZ = np.empty((xd.shape[0], x0.shape[0]), np.complex128)
    _check(_lib.eddy_delta_z_volume(op_defect._h, xd.shape[0], _dev(xd), op_free._h, x0.shape[0], _dev(x0),
                                    _ptr(ck, C.c_double), _ptr(cl, C.c_double),
                                    dZ.ctypes.data_as(C.POINTER(C.c_double)), _stream()), "eddy_delta_z_volume")
    return dZ


def ibc_split(xyz, tet, region, is_ibc):
    """eddy_ibc_split: the mesh without the tetrahedra of the flagged regions
    and its interface triangles with them.  Returns a dict with xyz, tet,
    region, faces, face_region, node_map."""
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    tet = np.ascontiguousarray(tet, dtype=np.int32)
    region = np.ascontiguousarray(region, dtype=np.int32)
    flags = np.ascontiguousarray(np.asarray(is_ibc).astype(np.int32))
    nv, nt = xyz.shape[0], tet.shape[0]
    a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
    args = (nv, _ptr(xyz, C.c_double), nt, _ptr(tet, C.c_int32), _ptr(region, C.c_int32), flags.size,
            _ptr(flags, C.c_int32), C.byref(a), C.byref(b), C.byref(c))
    nul = [None] * 6
    _check(_lib.eddy_ibc_split(*args, *nul), "eddy_ibc_split")
    out = {"xyz": np.empty((a.value, 3)), "tet": np.empty((b.value, 4), np.int32),
           "region": np.empty(b.value, np.int32), "faces": np.empty((c.value, 3), np.int32),
           "face_region": np.empty(c.value, np.int32), "node_map": np.empty(nv, np.int32)}
    _check(_lib.eddy_ibc_split(*args, _ptr(out["xyz"], C.c_double), _ptr(out["tet"], C.c_int32),
                               _ptr(out["region"], C.c_int32), _ptr(out["faces"], C.c_int32),
                               _ptr(out["face_region"], C.c_int32), _ptr(out["node_map"], C.c_int32)),
           "eddy_ibc_split")
    return out


class Mesh:
    """Host mesh handle: tetrahedra, regions, conductor flags per region, and
    optional impedance-boundary triangles (faces [nf, 3], face_region [nf])."""

    def __init__(self, xyz, tet, region, is_conductor, faces=None, face_region=None):
        self.xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        self.tet = np.ascontiguousarray(tet, dtype=np.int32)
        self.region = np.ascontiguousarray(region, dtype=np.int32)
        self.is_conductor = np.ascontiguousarray(np.asarray(is_conductor).astype(np.int32))
        self.faces = np.ascontiguousarray(np.zeros((0, 3)) if faces is None else faces, dtype=np.int32)
        self.face_region = np.ascontiguousarray(np.zeros(0) if face_region is None else face_region, dtype=np.int32)
        self.nf = self.faces.shape[0]
        h = C.c_void_p()
        _check(_lib.eddy_mesh_create_ibc(self.xyz.shape[0], _ptr(self.xyz, C.c_double), self.tet.shape[0],
                                         _ptr(self.tet, C.c_int32), _ptr(self.region, C.c_int32),
                                         self.is_conductor.size, _ptr(self.is_conductor, C.c_int32), self.nf,
                                         _ptr(self.faces, C.c_int32) if self.nf else None,
                                         _ptr(self.face_region, C.c_int32) if self.nf else None, C.byref(h)),
               "eddy_mesh_create_ibc")
        self._h = h
        ne, nc, nnz, nnzw, ncomp = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64(), C.c_int32()
        _check(_lib.eddy_mesh_counts(h, C.byref(ne), C.byref(nc), C.byref(nnz), C.byref(nnzw), C.byref(ncomp)),
               "eddy_mesh_counts")
        self.nv, self.nt = self.xyz.shape[0], self.tet.shape[0]
        self.ne, self.nc, self.nnz, self.nnz_w, self.ncomp = ne.value, nc.value, nnz.value, nnzw.value, ncomp.value
        self.ndof = self.ne + self.nc

    @classmethod
    def from_synth(cls, mesh, conductor_regions):
        flags = np.zeros(int(mesh.region.max()) + 1 if len(mesh.region_names) == 0 else len(mesh.region_names), np.int32)
        flags[list(conductor_regions)] = 1
        return cls(mesh.xyz, mesh.tet, mesh.region, flags)

    def edges(self) -> np.ndarray:
        out = np.empty((self.ne, 2), np.int32)
        _check(_lib.eddy_mesh_edges(self._h, _ptr(out, C.c_int32)), "eddy_mesh_edges")
        return out

    def conductor_nodes(self) -> np.ndarray:
        out = np.empty(self.nc, np.int32)
        if self.nc:
            _check(_lib.eddy_mesh_conductor_nodes(self._h, _ptr(out, C.c_int32)), "eddy_mesh_conductor_nodes")
        return out

    def subdomains(self, block_size: int):
        """(sub_of_dof [ndof], adjacency [64, 64]) of the learned correction (eddy_mesh_subdomains)."""
        sub = np.empty(self.ndof, np.int32)
        adj = np.empty(GNN_P * GNN_P, np.int32)
        _check(_lib.eddy_mesh_subdomains(self._h, block_size, _ptr(sub, C.c_int32), _ptr(adj, C.c_int32)),
               "eddy_mesh_subdomains")
        return sub, adj.reshape(GNN_P, GNN_P)

    def blocks(self, block_size: int):
        nb = C.c_int64()
        _check(_lib.eddy_mesh_blocks(self._h, block_size, C.byref(nb), None, None), "eddy_mesh_blocks")
        ptr = np.empty(nb.value + 1, np.int32)
        dofs = np.empty(self.ndof, np.int32)
        _check(_lib.eddy_mesh_blocks(self._h, block_size, C.byref(nb), _ptr(ptr, C.c_int32), _ptr(dofs, C.c_int32)),
               "eddy_mesh_blocks")
        return ptr, dofs

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.eddy_mesh_destroy(h)
            self._h = None


@dataclass
class SolveReport:
    iters: int
    restarts: int
    converged: bool
    breakdown: bool
    relres: float
    est_relres: float
    seconds: float
    gauge_in_operator: bool = False
    cg_iters: int = 0
    div_residual: float = 0.0
    precision_used: int = 0
    reorth_steps: int = 0
    learned_cycles: int = 0
    fell_back: bool = False


def _aligned(nbytes: int, device):
    import torch
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf, C.c_void_p(buf.data_ptr() + off)


class Operator:
    """Device operator: workspace, assembly, RHS, solve and outputs."""

    def __init__(self, mesh: Mesh, tau: float = 1.0, delta_v: float = 0.0, block_size: int = 64, device="cuda",
                 tau_precond: float = 0.0):
        import torch
        self.mesh = mesh
        self.device = torch.device(device)
        self.params = _Params(tau, delta_v, block_size, tau_precond)
        nbytes = C.c_size_t()
        _check(_lib.eddy_op_workspace_bytes(mesh._h, C.byref(self.params), C.byref(nbytes)), "eddy_op_workspace_bytes")
        self.ws_bytes = nbytes.value
        self._ws, self._wsp = _aligned(self.ws_bytes, self.device)
        h = C.c_void_p()
        _check(_lib.eddy_op_create(mesh._h, C.byref(self.params), self._wsp, self.ws_bytes, _stream(), C.byref(h)),
               "eddy_op_create")
        self._h = h
        self.ndof, self.ne, self.nc, self.nt, self.nv = mesh.ndof, mesh.ne, mesh.nc, mesh.nt, mesh.nv
        self._solve_ws = None
        self.omega = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.eddy_op_destroy(h)
            self._h = None

    def assemble(self, nu, sigma, omega: float):
        nu = np.ascontiguousarray(nu, dtype=np.float64)
        sigma = np.ascontiguousarray(sigma, dtype=np.float64)
        _check(_lib.eddy_op_assemble(self._h, _ptr(nu, C.c_double), _ptr(sigma, C.c_double), float(omega), _stream()),
               "eddy_op_assemble")
        self.omega = float(omega)

    def _c128(self, n=None):
        import torch
        return torch.empty(self.ndof if n is None else n, dtype=torch.complex128, device=self.device)

    def rhs_from_current(self, J, out=None):
        """J: float64 device tensor [nt, 3] -> b: complex128 [ndof]."""
        assert J.dtype.is_floating_point and J.is_contiguous() and J.numel() == 3 * self.nt
        b = self._c128() if out is None else out
        _check(_lib.eddy_rhs_from_current(self._h, _dev(J), _dev(b), _stream()), "eddy_rhs_from_current")
        return b

    def solve(self, b, tol=1e-10, restart=30, max_iter=5000, out=None, precision="fp64", gnn_theta=None,
              graph=False):
        """precision: "fp64", "mixed" (complex64 Krylov process, FP64 outer residual), or
        "mixed16" (as mixed, with the block-Jacobi inverses and the Krylov basis in complex half).
        gnn_theta: float32 device tensor of EDDY_GNN_PARAMS network parameters
        (the learned coarse correction with fallback), or None.  graph: run the
        Arnoldi steps between residual checks as captured HIP graphs."""
        if gnn_theta is not None:
            assert gnn_theta.dtype.is_floating_point and gnn_theta.element_size() == 4 and gnn_theta.is_contiguous()
            assert gnn_theta.numel() == GNN_PARAMS
        opts = _Opts(tol, restart, max_iter, {"fp64": 0, "mixed": 1, "mixed16": 2}[precision],
                     None if gnn_theta is None else gnn_theta.data_ptr(), 1 if graph else 0)
        nbytes = C.c_size_t()
        _check(_lib.eddy_solve_workspace_bytes(self._h, C.byref(opts), C.byref(nbytes)), "eddy_solve_workspace_bytes")
        if self._solve_ws is None or self._solve_ws[2] < nbytes.value:
            buf, p = _aligned(nbytes.value, self.device)
            self._solve_ws = (buf, p, nbytes.value)
        x = self._c128() if out is None else out
        rep = _Report()
        st = _check(_lib.eddy_solve(self._h, _dev(b), _dev(x), C.byref(opts), self._solve_ws[1], self._solve_ws[2],
                                    C.byref(rep), _stream()), "eddy_solve")
        return x, SolveReport(rep.iters, rep.restarts, bool(rep.converged), bool(rep.breakdown), rep.relres,
                              rep.est_relres, rep.seconds, bool(rep.gauge_in_operator), rep.cg_iters,
                              rep.div_residual, rep.precision_used, rep.reorth_steps, rep.learned_cycles,
                              bool(rep.fell_back))

    def solve_batched(self, B, tol=1e-10, restart=30, max_iter=5000, out=None, precision="fp64"):
        """B: complex128 device tensor [nrhs, ndof] -> (X [nrhs, ndof], [SolveReport])."""
        import torch
        B = B.reshape(-1, self.ndof).contiguous()
        nrhs = B.shape[0]
        opts = _Opts(tol, restart, max_iter, {"fp64": 0, "mixed": 1, "mixed16": 2}[precision])
        nbytes = C.c_size_t()
        _check(_lib.eddy_solve_batched_workspace_bytes(self._h, nrhs, C.byref(opts), C.byref(nbytes)),
               "eddy_solve_batched_workspace_bytes")
        key = ("batch", nbytes.value)
        if getattr(self, "_batch_ws", None) is None or self._batch_ws[2] < nbytes.value:
            buf, p = _aligned(nbytes.value, self.device)
            self._batch_ws = (buf, p, nbytes.value)
        X = torch.empty_like(B) if out is None else out
        reps = (_Report * nrhs)()
        _check(_lib.eddy_solve_batched(self._h, nrhs, _dev(B), _dev(X), C.byref(opts), self._batch_ws[1],
                                       self._batch_ws[2], reps, _stream()), "eddy_solve_batched")
        return X, [SolveReport(r.iters, r.restarts, bool(r.converged), bool(r.breakdown), r.relres, r.est_relres,
                               r.seconds, bool(r.gauge_in_operator), r.cg_iters, r.div_residual, r.precision_used,
                               r.reorth_steps) for r in reps]

    def spmv(self, x, out=None):
        y = self._c128() if out is None else out
        _check(_lib.eddy_spmv(self._h, _dev(x), _dev(y), _stream()), "eddy_spmv")
        return y

    def precond_apply(self, r, out=None):
        z = self._c128() if out is None else out
        _check(_lib.eddy_precond_apply(self._h, _dev(r), _dev(z), _stream()), "eddy_precond_apply")
        return z

    def edge_field(self, x, out=None):
        E = self._c128(self.ne) if out is None else out
        _check(_lib.eddy_edge_field(self._h, _dev(x), _dev(E), _stream()), "eddy_edge_field")
        return E

    def impedance(self, xs, bs, currents):
        """xs: [nsol, ndof], bs: [nsrc, ndof] complex128 device; returns Z[nsol, nsrc] (numpy)."""
        xs = xs.reshape(-1, self.ndof).contiguous()
        bs = bs.reshape(-1, self.ndof).contiguous()
        cur = np.ascontiguousarray(currents, dtype=np.float64)
        Z = np.empty((xs.shape[0], bs.shape[0]), dtype=np.complex128)
        _check(_lib.eddy_impedance(self._h, xs.shape[0], _dev(xs), bs.shape[0], _dev(bs), _ptr(cur, C.c_double),
                                   Z.ctypes.data_as(C.POINTER(C.c_double)), _stream()), "eddy_impedance")
        return Z

    PROFILE_CLASSES = ("block_apply", "gauge_wt", "spmv", "cgs2")

    def profile(self, enable: bool = True):
        """Read-and-reset the per-class GMRES kernel timings; enable/disable timing."""
        ms = np.zeros(4)
        cnt = np.zeros(4, np.int64)
        _check(_lib.eddy_profile(self._h, int(enable), _ptr(ms, C.c_double), _ptr(cnt, C.c_int64)), "eddy_profile")
        return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(self.PROFILE_CLASSES)}

    # ---- learned coarse correction (thin wrappers of eddy_gnn_*)
    def gnn_static_features(self):
        out = np.empty(GNN_P * 4, np.float32)
        _check(_lib.eddy_gnn_static_features(self._h, _ptr(out, C.c_float)), "eddy_gnn_static_features")
        return out.reshape(GNN_P, 4)

    def _gnn_scratch(self, nsamp):
        nb = C.c_size_t()
        _check(_lib.eddy_gnn_scratch_bytes(nsamp, C.byref(nb)), "eddy_gnn_scratch_bytes")
        key = ("gnn", nsamp)
        cache = getattr(self, "_gnn_ws", None)
        if cache is None or cache[0] != key:
            buf, p = _aligned(nb.value, self.device)
            self._gnn_ws = (key, buf, p, nb.value)
        return self._gnn_ws[2], self._gnn_ws[3]

    def gnn_pair(self, b, x, xstar=None):
        """Features X [64, 16] and (with xstar) targets c* [64, 2], weights w [64]
        of the pair r = b - M x, e = xstar - x (complex128 device vectors)."""
        import torch
        X = torch.empty((GNN_P, GNN_FIN), dtype=torch.float32, device=self.device)
        cs = torch.empty((GNN_P, 2), dtype=torch.float32, device=self.device)
        w = torch.empty(GNN_P, dtype=torch.float32, device=self.device)
        t = xstar is not None
        _check(_lib.eddy_gnn_pair(self._h, _dev(b), _dev(x), _dev(xstar) if t else None, _dev(X),
                                  _dev(cs) if t else None, _dev(w) if t else None, _stream()), "eddy_gnn_pair")
        return X, cs, w

    def gnn_forward(self, theta, X):
        """Y [nsamp, 64, 16] of the network for X [nsamp, 64, 16] (float32 device)."""
        import torch
        X = X.reshape(-1, GNN_P, GNN_FIN).contiguous()
        Y = torch.empty((X.shape[0], GNN_P, GNN_FOUT), dtype=torch.float32, device=self.device)
        p, nb = self._gnn_scratch(X.shape[0])
        _check(_lib.eddy_gnn_forward(self._h, X.shape[0], _dev(theta), _dev(X), _dev(Y), p, nb, _stream()),
               "eddy_gnn_forward")
        return Y

    def gnn_train_step(self, theta, m, v, X, cstar, w, step, lr, grad_out=None):
        """One Adam step (in place on theta, m, v); returns per-sample losses."""
        import torch
        X = X.reshape(-1, GNN_P, GNN_FIN).contiguous()
        ns = X.shape[0]
        loss = torch.empty(ns, dtype=torch.float32, device=self.device)
        p, nb = self._gnn_scratch(ns)
        _check(_lib.eddy_gnn_train_step(self._h, ns, _dev(theta), _dev(m), _dev(v), _dev(X),
                                        _dev(cstar.contiguous()), _dev(w.contiguous()), int(step), float(lr),
                                        _dev(loss), None if grad_out is None else _dev(grad_out), p, nb,
                                        _stream()), "eddy_gnn_train_step")
        return loss

    def tuning(self) -> dict:
        """Launch shapes the autotuner chose at the first assemble (eddy_op_tuning)."""
        t = _Tuning()
        _check(_lib.eddy_op_tuning(self._h, C.byref(t)), "eddy_op_tuning")
        out = {}
        for f, _ in _Tuning._fields_:
            v = getattr(t, f)
            out[f] = list(v) if isinstance(v, C.Array) else v
        return out

    def export(self):
        """Host copies of the stored arrays (see eddy_export)."""
        m = self.mesh
        out = {
            "rowptr": np.empty(self.ndof + 1, np.int32), "col": np.empty(m.nnz, np.int32),
            "val": np.empty(m.nnz, np.complex128), "wrowptr": np.empty(self.ne + 1, np.int32),
            "wcol": np.empty(m.nnz_w, np.int32), "wval": np.empty(m.nnz_w, np.float64),
            "d0": np.empty(self.nv, np.float64), "s": np.empty(self.ndof, np.float64),
        }
        I, D = C.c_int32, C.c_double
        _check(_lib.eddy_export(self._h, _ptr(out["rowptr"], I), _ptr(out["col"], I),
                                out["val"].ctypes.data_as(C.POINTER(D)), _ptr(out["wrowptr"], I), _ptr(out["wcol"], I),
                                _ptr(out["wval"], D), _ptr(out["d0"], D), _ptr(out["s"], D), _stream()), "eddy_export")
        return out


def solve_multifreq(ops, B, op_of_rhs, tol=1e-10, restart=30, max_iter=5000, out=None, precision="mixed"):
    """eddy_solve_multifreq: B complex128 device [nrhs, ndof]; system r belongs
    to ops[op_of_rhs[r]] (nondecreasing).  Returns (X [nrhs, ndof], [SolveReport])."""
    import torch
    ops = list(ops)
    ndof = ops[0].ndof
    B = B.reshape(-1, ndof).contiguous()
    nrhs = B.shape[0]
    idx = np.ascontiguousarray(op_of_rhs, dtype=np.int32)
    if idx.size != nrhs:
        raise ValueError("op_of_rhs needs one entry per right-hand side")
    handles = (C.c_void_p * len(ops))(*[o._h.value if isinstance(o._h, C.c_void_p) else o._h for o in ops])
    opts = _Opts(tol, restart, max_iter, {"fp64": 0, "mixed": 1, "mixed16": 2}[precision])
    nbytes = C.c_size_t()
    _check(_lib.eddy_solve_multifreq_workspace_bytes(handles, len(ops), nrhs, C.byref(opts), C.byref(nbytes)),
           "eddy_solve_multifreq_workspace_bytes")
    buf, p = _aligned(nbytes.value, ops[0].device)
    X = torch.empty_like(B) if out is None else out
    reps = (_Report * nrhs)()
    _check(_lib.eddy_solve_multifreq(handles, len(ops), nrhs, _ptr(idx, C.c_int32), _dev(B), _dev(X), C.byref(opts),
                                     p, nbytes.value, reps, _stream()), "eddy_solve_multifreq")
    del buf
    return X, [SolveReport(r.iters, r.restarts, bool(r.converged), bool(r.breakdown), r.relres, r.est_relres,
                           r.seconds, bool(r.gauge_in_operator), r.cg_iters, r.div_residual, r.precision_used,
                           r.reorth_steps) for r in reps]
