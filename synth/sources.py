"""Seeded source currents, one constant vector per tetrahedron.

Every current here is built as J_K = grad(alpha_h) x grad(beta_h) on each
tetrahedron K, where alpha_h and beta_h are the piecewise-linear
interpolants of two scalar fields.  Since alpha_h * grad(beta_h) has
continuous tangential traces, its curl J has continuous normal components
across faces and zero divergence inside each tetrahedron: the discrete
current is exactly divergence-free, as the paper requires of the excitation
in the insulator (Section 2, below Eq. 1).  Where alpha vanishes on the
outer boundary, J.n = 0 there as well.

The gradient of a linear interpolant is obtained with a generic 3x3 linear
solve per tetrahedron; no basis function of the method is evaluated here.
"""
from __future__ import annotations

import numpy as np


def grad_cross(xyz: np.ndarray, tet: np.ndarray, alpha: np.ndarray, beta: np.ndarray) -> np.ndarray:
    """J[nt, 3] = grad(alpha_h) x grad(beta_h) per tetrahedron."""
    p = xyz[tet]
    E = p[:, 1:, :] - p[:, :1, :]                       # rows p_i - p_0
    da = alpha[tet[:, 1:]] - alpha[tet[:, :1]]          # [nt, 3]
    db = beta[tet[:, 1:]] - beta[tet[:, :1]]
    ga = np.linalg.solve(E, da[..., None])[..., 0]       # E g = d  (g = gradient)
    gb = np.linalg.solve(E, db[..., None])[..., 0]
    return np.cross(ga, gb)


def cube_current(mesh, seed: int = 0, kmax: int = 1, scale: float = 1.0) -> np.ndarray:
    """Smooth seeded current on the unit cube with J.n = 0 on the boundary.

    alpha = sin(pi x) sin(pi y) sin(pi z) * (1 + 0.5 * s1(x)),
    beta  = s2(x), where s1 and s2 are random trigonometric sums
    sum_k a_k cos(2 pi k.x + phi_k) over k in {0..kmax}^3 with
    a_k ~ N(0, 1) 2^-|k|_1 and phi_k ~ U(0, 2 pi) from default_rng(seed).
    """
    rng = np.random.default_rng(seed)
    x = mesh.xyz
    L = float(mesh.meta.get("length", 1.0)) if hasattr(mesh, "meta") else 1.0
    ks = np.array([(i, j, k) for i in range(kmax + 1) for j in range(kmax + 1) for k in range(kmax + 1)], dtype=float)
    amp = 2.0 ** (-ks.sum(axis=1))

    def trig():
        a = rng.standard_normal(len(ks)) * amp
        ph = rng.uniform(0, 2 * np.pi, len(ks))
        return (a[None, :] * np.cos(2 * np.pi * (x / L) @ ks.T + ph[None, :])).sum(axis=1)

    s1 = trig()
    s2 = trig()
    bubble = np.prod(np.sin(np.pi * x / L), axis=1)
    alpha = bubble * (1.0 + 0.5 * s1)
    alpha[np.abs(bubble) < 1e-14] = 0.0                 # exact zeros on the boundary
    return scale * grad_cross(x, mesh.tet, alpha, s2)


def _ramp(t: np.ndarray, t0: float, t1: float) -> np.ndarray:
    return np.clip(t, t0, t1) - t0


def coil_current(mesh, z_center: float, r0: float, r1: float, half_len: float, current: float = 1.0) -> np.ndarray:
    """Azimuthal coil current of total `current` amperes (one turn) through the
    cross-section [r0, r1] x [z_center - half_len, z_center + half_len].

    alpha = ramp(z) with unit slope over the coil's axial extent, beta =
    J0 * ramp(r) with slope J0 = current / ((r1 - r0) * 2 half_len) over its
    radial extent, so grad(alpha) x grad(beta) = J0 theta-hat inside.
    """
    x = mesh.xyz
    r = np.hypot(x[:, 0], x[:, 1])
    J0 = current / ((r1 - r0) * 2.0 * half_len)
    alpha = _ramp(x[:, 2], z_center - half_len, z_center + half_len)
    beta = J0 * _ramp(r, r0, r1)
    return grad_cross(x, mesh.tet, alpha, beta)


def probe_currents(mesh, z_probe: float, r_coil=(7.6e-3, 9.1e-3), side=1.5e-3, gap=0.5e-3, current=1.0):
    """The two coils of a differential bobbin probe centred at z_probe.

    Coil 1 (generator) sits below z_probe, coil 2 (receiver) above; each has
    a side x side cross-section, the coils are `gap` apart axially.
    Returns (J1[nt,3], J2[nt,3]).
    """
    hl = 0.5 * side
    zc = 0.5 * gap + hl
    J1 = coil_current(mesh, z_probe - zc, r_coil[0], r_coil[1], hl, current)
    J2 = coil_current(mesh, z_probe + zc, r_coil[0], r_coil[1], hl, current)
    return J1, J2


def solenoid_current(mesh, R1: float, R2: float, J0: float = 1.0) -> np.ndarray:
    """J = J0 theta-hat in the annulus R1 < r < R2 over the full height."""
    x = mesh.xyz
    r = np.hypot(x[:, 0], x[:, 1])
    return grad_cross(x, mesh.tet, x[:, 2].copy(), J0 * _ramp(r, R1, R2))
