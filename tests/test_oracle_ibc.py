"""Pins of the impedance-boundary oracle (oracle/ibc.py; Section 2, Eqs. 8-10).

* Triangle integrals against quadrature, with barycentric gradients from the
  triangle's own parametrisation (not the cross-product formula).
* The surface de Rham identities B_G = M_G G and S_G = G^T M_G G per
  triangle (surface gradients of P1 are Whitney traces).
* Thin-sheet limit: surface terms with the real coefficient sigma * d agree
  with a volume layer of thickness d and conductivity sigma as d -> 0
  (first order in d), which pins the assembly of the surface terms against
  the volume terms they mirror.
* The impedance condition itself: a plate removed from the mesh with 1/Z on
  its interface converges under mesh refinement to a volume plate resolved
  at delta / 8, measured on the O(delta) correction beyond a perfect
  conductor.  The opposite normal (the sign of the surface term) and a real
  coefficient (the (1 - i) of Z dropped) stay far off.
* The mesh split: every interface triangle is a face of a kept tetrahedron
  and of a removed one; nodes keep their order.
"""
import numpy as np
import pytest

from synth import box, grad_cross

from oracle.assemble import assemble
from oracle.ibc import FACE_EDGES, face_matrices, split, surface_conductance
from oracle.solve import direct


def _param_grads(p):
    """Surface gradients of l1 = s, l2 = t, l0 = 1 - s - t for x = p0 + s e1 + t e2."""
    J = np.stack([p[1] - p[0], p[2] - p[0]], axis=1)          # 3 x 2
    P = J @ np.linalg.inv(J.T @ J)                             # columns: grad s, grad t
    g1, g2 = P[:, 0], P[:, 1]
    return np.stack([-(g1 + g2), g1, g2])


def test_triangle_integrals_against_quadrature():
    rng = np.random.default_rng(5)
    xyz = rng.normal(size=(3 * 6, 3))
    faces = np.arange(18).reshape(6, 3)
    fm = face_matrices(xyz, faces)
    # edge-midpoint rule: exact for quadratics on a triangle
    bary = np.array([[0.5, 0.5, 0.0], [0.5, 0.0, 0.5], [0.0, 0.5, 0.5]])
    for f in range(6):
        p = xyz[faces[f]]
        area = 0.5 * np.linalg.norm(np.cross(p[1] - p[0], p[2] - p[0]))
        g = _param_grads(p)
        M = np.zeros((3, 3)); B = np.zeros((3, 3))
        for lam in bary:
            w = np.array([lam[a] * g[b] - lam[b] * g[a] for a, b in FACE_EDGES])
            M += (area / 3) * w @ w.T
            B += (area / 3) * w @ g.T
        assert abs(fm["area"][f] - area) <= 1e-14 * area
        assert np.allclose(fm["grad"][f], g, rtol=0, atol=1e-12 * np.abs(g).max())
        assert np.allclose(fm["M"][f], M, rtol=0, atol=1e-12 * np.abs(M).max())
        assert np.allclose(fm["B"][f], B, rtol=0, atol=1e-12 * np.abs(B).max())
        assert np.allclose(fm["S"][f], area * g @ g.T, rtol=0, atol=1e-12 * area * np.abs(g).max() ** 2)


def test_surface_de_rham_identities():
    rng = np.random.default_rng(6)
    xyz = rng.normal(size=(30, 3))
    faces = np.sort(rng.choice(30, size=(10, 3), replace=True), axis=1)
    faces = faces[(faces[:, 0] < faces[:, 1]) & (faces[:, 1] < faces[:, 2])]
    fm = face_matrices(xyz, faces)
    G = np.array([[-1.0, 1.0, 0.0], [-1.0, 0.0, 1.0], [0.0, -1.0, 1.0]])
    for f in range(faces.shape[0]):
        M, B, S = fm["M"][f], fm["B"][f], fm["S"][f]
        assert np.allclose(B, M @ G, atol=1e-12 * np.abs(B).max())
        assert np.allclose(S, G.T @ M @ G, atol=1e-12 * np.abs(S).max())


def _source(m, lo, hi):
    """Divergence-free current grad(alpha) x grad(beta), alpha a bubble on the box [lo, hi]."""
    x = m.xyz
    t = np.clip((x - lo) / (hi - lo), 0.0, 1.0)
    alpha = np.prod(np.sin(np.pi * t), axis=1)
    beta = x[:, 0] + 0.3 * x[:, 1]
    return grad_cross(x, m.tet, alpha, beta)


def test_surface_terms_match_a_thin_volume_layer():
    omega, z0, G = 50.0, 0.5, 0.5          # sheet conductance sigma * d = G
    xs = np.linspace(0, 1, 9)
    errs = []
    for d in (4e-3, 2e-3, 1e-3):
        zs = np.sort(np.concatenate([np.linspace(0, 1, 9), [z0 + d]]))
        m = box(xs, xs, zs)
        cz = m.xyz[m.tet][:, :, 2].mean(axis=1)
        layer = (cz > z0) & (cz < z0 + d)
        J = _source(m, np.array([0.2, 0.2, 0.62]), np.array([0.8, 0.8, 0.88]))
        nu = np.array([1.0, 1.0])
        region = layer.astype(np.int32)
        sv = assemble(m.xyz, m.tet, region, nu, np.array([0.0, G / d]), omega, tau=1.0, conductor_regions=[1])
        # the same mesh with the layer as air and a conducting sheet on z = z0
        fa = np.sort(m.tet[layer][:, [[0, 1, 2], [0, 1, 3], [0, 2, 3], [1, 2, 3]]].reshape(-1, 3), axis=1)
        fa = np.unique(fa[np.all(np.abs(m.xyz[fa][:, :, 2] - z0) < 1e-12, axis=1)], axis=0)
        assert fa.shape[0] == 2 * 8 * 8
        ss = assemble(m.xyz, m.tet, np.zeros_like(region), nu, np.array([0.0, 0.0]), omega, tau=1.0,
                      conductor_regions=[], faces=fa, face_coef=np.full(fa.shape[0], G, dtype=complex))
        sa = assemble(m.xyz, m.tet, np.zeros_like(region), nu, np.array([0.0, 0.0]), omega, tau=1.0,
                      conductor_regions=[])
        b = sv.rhs(J)
        assert np.array_equal(b[:sv.topo.ne], ss.rhs(J)[:ss.topo.ne])
        ne = sv.topo.ne
        zv = b[:ne] @ direct(sv, b)[:ne]
        zs_ = b[:ne] @ direct(ss, ss.rhs(J))[:ne]
        za = b[:ne] @ direct(sa, sa.rhs(J))[:ne]
        errs.append(abs(zv - zs_) / abs(zv - za))
        assert abs(zv - za) > 1e-2 * abs(za)           # the sheet matters
    # first order in d
    assert errs[-1] < 0.05
    assert 1.5 < errs[0] / errs[1] < 2.6 and 1.5 < errs[1] / errs[2] < 2.6


def _plate_case(nx, sig, omega=50.0, zp=0.25):
    """Plate z < zp resolved with h = delta / 8 near its surface (lateral
    spacing 1 / (nx - 1)); returns the coupling b^T A of the volume model and
    of the plate removed with surface coefficients 1/Z (Eq. 8), its opposite
    (the other normal), |1/Z| (a real coefficient) and 1e8 / Z (a perfect
    conductor)."""
    delta = np.sqrt(2.0 / (omega * sig))
    xs = np.linspace(0, 1, nx)
    zin = zp - np.concatenate([np.arange(0, 4 * delta, delta / 8), 4 * delta * 1.4 ** np.arange(1, 8)])
    zin = zin[zin > 0.0]
    zout = zp + np.concatenate([np.arange(1, 9) * delta / 8, delta + 0.3 / (nx - 1) * 1.5 ** np.arange(1, 9)])
    zout = zout[zout < 0.99]
    m = box(xs, xs, np.unique(np.concatenate([[0.0, 1.0], zin, zout])))
    cz = m.xyz[m.tet][:, :, 2].mean(axis=1)
    region = (cz < zp).astype(np.int32)
    nu, sg = np.array([1.0, 1.0]), np.array([0.0, sig])
    J = _source(m, np.array([0.2, 0.2, 0.3]), np.array([0.8, 0.8, 0.6]))
    sv = assemble(m.xyz, m.tet, region, nu, sg, omega, tau=1.0, conductor_regions=[1])
    bv = sv.rhs(J)
    out = {"volume": bv[:sv.topo.ne] @ direct(sv, bv)[:sv.topo.ne]}
    sp_ = split(m.xyz, m.tet, region, [1])
    coef = surface_conductance(sg[sp_["face_region"]], nu[sp_["face_region"]], omega)
    Ja = J[region == 0]
    for name, c in (("ibc", coef), ("flip", -coef), ("real", np.abs(coef) + 0j), ("pec", 1e8 * coef)):
        si = assemble(sp_["xyz"], sp_["tet"], sp_["region"], nu, sg, omega, tau=1.0, conductor_regions=[],
                      faces=sp_["faces"], face_coef=c)
        bi = si.rhs(Ja)
        out[name] = bi[:si.topo.ne] @ direct(si, bi)[:si.topo.ne]
    return out


def test_impedance_condition_matches_a_resolved_plate():
    """Skin depth 0.04 (sigma = 25, nu = 1, omega = 50).  At this depth the
    plate is nearly a perfect conductor; what the impedance condition adds is
    the O(delta) correction beyond it, so errors are measured against that
    correction |Z_vol - Z_pec|.  The error of Eq. 8 falls under lateral
    refinement (the two models share only the air mesh: their discretisation
    errors differ); the opposite normal and a real coefficient stay off."""
    r = {}
    for nx in (5, 9):
        z = _plate_case(nx, 25.0)
        d = abs(z["volume"] - z["pec"])
        assert d > 1e-3 * abs(z["volume"])
        r[nx] = {k: abs(z["volume"] - z[k]) / d for k in ("ibc", "flip", "real")}
        print(nx, {k: round(v, 3) for k, v in r[nx].items()})
    assert r[9]["ibc"] < 0.4 and r[9]["ibc"] < 0.5 * r[5]["ibc"]
    assert r[9]["flip"] > 2.0 and r[9]["real"] > 0.45


def test_split_interface_and_numbering():
    xs = np.linspace(0, 1, 5)
    m = box(xs, xs, xs)
    cen = m.xyz[m.tet].mean(axis=1)
    region = np.where(np.all((cen > 0.25) & (cen < 0.75), axis=1), 2, 0).astype(np.int32)
    sp_ = split(m.xyz, m.tet, region, [2])
    nm = sp_["node_map"]
    kept = nm >= 0
    assert np.all(np.diff(np.flatnonzero(kept)) > 0) and np.array_equal(nm[kept], np.arange(kept.sum()))
    # the removed block's 8 interior cells leave one interior node unused
    assert (~kept).sum() == 1
    # interface = boundary of the removed 2x2x2 block: 6 sides x 4 squares x 2 triangles
    assert sp_["faces"].shape[0] == 48
    kf = np.sort(sp_["tet"][:, [[0, 1, 2], [0, 1, 3], [0, 2, 3], [1, 2, 3]]].reshape(-1, 3), axis=1)
    ks = {tuple(f) for f in kf}
    assert all(tuple(f) in ks for f in sp_["faces"])
    c = sp_["xyz"][sp_["faces"]]
    on_box = np.all((c >= 0.25 - 1e-12) & (c <= 0.75 + 1e-12), axis=(1, 2))
    assert on_box.all() and np.all(sp_["face_region"] == 2)


def test_surface_conductance_is_the_skin_depth_form():
    # delta = sqrt(2 / (omega mu sigma)); 1/Z = delta sigma / (1 - i): |1/Z| = delta sigma / sqrt(2), phase +45 deg
    sig, mu, om = 2e6, 4e-7 * np.pi, 2 * np.pi * 1e5
    c = surface_conductance(sig, 1.0 / mu, om)
    delta = 1.0 / np.sqrt(np.pi * 1e5 * mu * sig)          # the textbook f-form of the skin depth
    assert abs(abs(c) - delta * sig / np.sqrt(2)) <= 1e-12 * abs(c)
    assert abs(np.angle(c) - np.pi / 4) <= 1e-14
