"""Seeded synthetic tetrahedral meshes.

Pure geometry: node coordinates, tetrahedra and a region label per
tetrahedron.  Nothing in this module evaluates a basis function, an element
integral or any other step of the finite-element method; both the CPU oracle
and the GPU path read these arrays as input.

Three families are produced:

* ``cube``      -- the unit cube split into n^3 cubes of 6 tetrahedra each
                   (Kuhn split along the main diagonal), with the conductor
                   sub-box [0.25, 0.75]^3 labelled by tetrahedron centroid.
* ``cylinder``  -- an extruded O-grid slab: a solid conducting cylinder of
                   radius ``a`` inside a solenoid annulus [R1, R2], closed by an
                   insulating annulus up to ``R_out``.
* ``tube``      -- the steam-generator tube family: a conducting tube, a
                   support plate with four lobed flow holes, two coaxial coils
                   inside the tube, in an air cylinder.

Every 2-D cross-section is a ring triangulation conforming to the material
radii; prisms are split into 3 tetrahedra with a rule that depends only on
the global node numbers, so neighbouring prisms always agree on the diagonal
of their shared quadrilateral face.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np


@dataclass
class Mesh:
    xyz: np.ndarray              # float64 [nv, 3], metres (or unit-less)
    tet: np.ndarray              # int32   [nt, 4]
    region: np.ndarray           # int32   [nt]
    region_names: list = field(default_factory=list)
    meta: dict = field(default_factory=dict)

    @property
    def nv(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def nt(self) -> int:
        return int(self.tet.shape[0])


# ---------------------------------------------------------------------------
# Unit cube, Kuhn split
# ---------------------------------------------------------------------------

def cube(n: int, lo: float = 0.25, hi: float = 0.75, length: float = 1.0) -> Mesh:
    """n^3 cubes x 6 tetrahedra.  Region 1 = centroid inside [lo, hi]^3."""
    m = n + 1
    g = np.arange(m)
    k, j, i = np.meshgrid(g, g, g, indexing="ij")
    xyz = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1).astype(np.float64) * (length / n)

    def nid(ii, jj, kk):
        return ii + m * (jj + m * kk)

    ci, cj, ck = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    ci, cj, ck = ci.ravel(), cj.ravel(), ck.ravel()
    perms = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
    tets = []
    for p in perms:
        off = np.zeros((4, 3), dtype=np.int64)
        for s in range(1, 4):
            off[s] = off[s - 1]
            off[s, p[s - 1]] += 1
        cols = [nid(ci + off[s, 0], cj + off[s, 1], ck + off[s, 2]) for s in range(4)]
        tets.append(np.stack(cols, axis=1))
    # order: cube-major, then the 6 permutations
    tet = np.stack(tets, axis=1).reshape(-1, 4).astype(np.int32)
    cen = xyz[tet].mean(axis=1)
    inside = np.all((cen > lo * length) & (cen < hi * length), axis=1)
    region = inside.astype(np.int32)
    return Mesh(xyz, tet, region, ["air", "conductor"], {"family": "cube", "n": n})


def box(x, y, z) -> Mesh:
    """Tensor-product grid with node coordinates x, y, z (increasing), each
    cell split into 6 tetrahedra as in cube(); region 0 everywhere (callers
    set regions from the centroids)."""
    x, y, z = (np.asarray(a, dtype=np.float64) for a in (x, y, z))
    nx, ny, nz = x.size, y.size, z.size
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    xyz = np.stack([x[i.ravel()], y[j.ravel()], z[k.ravel()]], axis=1)

    def nid(ii, jj, kk):
        return ii + nx * (jj + ny * kk)

    ci, cj, ck = np.meshgrid(np.arange(nx - 1), np.arange(ny - 1), np.arange(nz - 1), indexing="ij")
    ci, cj, ck = ci.ravel(), cj.ravel(), ck.ravel()
    perms = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
    tets = []
    for p in perms:
        off = np.zeros((4, 3), dtype=np.int64)
        for s in range(1, 4):
            off[s] = off[s - 1]
            off[s, p[s - 1]] += 1
        tets.append(np.stack([nid(ci + off[s, 0], cj + off[s, 1], ck + off[s, 2]) for s in range(4)], axis=1))
    tet = np.stack(tets, axis=1).reshape(-1, 4).astype(np.int32)
    return Mesh(xyz, tet, np.zeros(tet.shape[0], dtype=np.int32), ["air"], {"family": "box"})


# ---------------------------------------------------------------------------
# 2-D ring triangulations
# ---------------------------------------------------------------------------

def _ring_counts(radii: np.ndarray, h_theta: float, n_min: int, multiple: int, n_max: int) -> np.ndarray:
    cnt = np.maximum(n_min, np.ceil(2 * np.pi * radii / h_theta / multiple).astype(int) * multiple)
    # never let the count drop outward (keeps the zip well shaped)
    return np.minimum(np.maximum.accumulate(cnt), max(n_max, n_min))


def ring_triangulation(radii, h_theta: float, n_min: int = 8, multiple: int = 4, n_max: int = 1 << 30):
    """Triangulate the disk r <= radii[-1] with node rings at the given radii.

    Returns (xy [np2, 2], tri [nt2, 3]).  Node 0 is the centre; ring i holds
    counts[i] nodes starting at angle 0.
    """
    radii = np.asarray(radii, dtype=np.float64)
    assert np.all(np.diff(radii) > 0) and radii[0] > 0
    counts = _ring_counts(radii, h_theta, n_min, multiple, n_max)
    xy = [np.zeros((1, 2))]
    starts = []
    base = 1
    for r, c in zip(radii, counts):
        th = 2 * np.pi * np.arange(c) / c
        xy.append(np.stack([r * np.cos(th), r * np.sin(th)], axis=1))
        starts.append(base)
        base += c
    xy = np.concatenate(xy)
    tris = []
    # centre fan
    c0, s0 = counts[0], starts[0]
    for a in range(c0):
        tris.append((0, s0 + a, s0 + (a + 1) % c0))
    # zip consecutive rings by angle
    for i in range(len(radii) - 1):
        na, nb = counts[i], counts[i + 1]
        sa, sb = starts[i], starts[i + 1]
        ia = ib = 0
        while ia < na or ib < nb:
            ta = (ia + 1) / na
            tb = (ib + 1) / nb
            if ib >= nb or (ia < na and ta < tb):
                tris.append((sa + ia % na, sa + (ia + 1) % na, sb + ib % nb))
                ia += 1
            else:
                tris.append((sa + ia % na, sb + (ib + 1) % nb, sb + ib % nb))
                ib += 1
    return xy, np.asarray(tris, dtype=np.int64)


def extrude(xy: np.ndarray, tri: np.ndarray, z: np.ndarray):
    """Extrude a 2-D triangulation over the z-levels; 3 tetrahedra per prism.

    Layer k has 2-D node p at global id p + k*np2.  In a prism whose base
    triangle has 2-D ids a < b < c, the quadrilateral face over edge (u, v),
    u < v, is cut by the diagonal from u at the bottom to v at the top; the
    three tetrahedra below realise exactly those three diagonals.
    """
    z = np.asarray(z, dtype=np.float64)
    np2 = xy.shape[0]
    nl = z.shape[0]
    xyz = np.empty((np2 * nl, 3))
    xyz[:, 0] = np.tile(xy[:, 0], nl)
    xyz[:, 1] = np.tile(xy[:, 1], nl)
    xyz[:, 2] = np.repeat(z, np2)
    s = np.sort(tri, axis=1)
    a, b, c = s[:, 0], s[:, 1], s[:, 2]
    k = np.arange(nl - 1)[:, None]
    a0, b0, c0 = a + k * np2, b + k * np2, c + k * np2
    a1, b1, c1 = a0 + np2, b0 + np2, c0 + np2
    t1 = np.stack([a0, b0, c0, c1], axis=-1)
    t2 = np.stack([a0, b0, b1, c1], axis=-1)
    t3 = np.stack([a0, a1, b1, c1], axis=-1)
    tet = np.stack([t1, t2, t3], axis=2).reshape(-1, 4)   # layer-major, prism, split
    prism_tri = np.broadcast_to(np.arange(tri.shape[0])[None, :, None], (nl - 1, tri.shape[0], 3)).reshape(-1)
    prism_layer = np.broadcast_to(np.arange(nl - 1)[:, None, None], (nl - 1, tri.shape[0], 3)).reshape(-1)
    return xyz, tet.astype(np.int32), prism_tri, prism_layer


def _graded(x0: float, x1: float, h0: float, h1: float) -> np.ndarray:
    """Points from x0 to x1 (inclusive) with spacing growing from h0 to h1."""
    L = x1 - x0
    if L <= 0:
        return np.array([x0])
    n = max(1, int(np.ceil(2 * L / (h0 + h1))))
    t = np.linspace(0.0, 1.0, n + 1)
    # spacing linear in t: h(t) = h0 + (h1-h0) t  -> position = integral
    pos = h0 * t + 0.5 * (h1 - h0) * t * t
    pos = pos / pos[-1] * L
    return x0 + pos


def _uniform(x0: float, x1: float, h: float) -> np.ndarray:
    n = max(1, int(np.ceil((x1 - x0) / h - 1e-9)))
    return np.linspace(x0, x1, n + 1)


def _join(*parts) -> np.ndarray:
    out = [parts[0]]
    for p in parts[1:]:
        out.append(p[1:] if np.isclose(p[0], out[-1][-1]) else p)
    return np.concatenate(out)


# ---------------------------------------------------------------------------
# Conducting cylinder in a solenoid (slab of height H)
# ---------------------------------------------------------------------------

def cylinder(a=0.5, R1=0.6, R2=0.8, R_out=1.0, H=0.1, h=0.05, nz=None) -> Mesh:
    """Regions: 0 air (a<r<R1 and r>R2), 1 conductor (r<a), 2 coil (R1<r<R2)."""
    radii = _join(_uniform(h, a, h), _uniform(a, R1, h), _uniform(R1, R2, h), _uniform(R2, R_out, h))
    xy, tri = ring_triangulation(radii, h_theta=h, n_min=8, multiple=4)
    nz = nz if nz is not None else max(1, int(round(H / h)))
    z = np.linspace(0.0, H, nz + 1)
    xyz, tet, ptri, _ = extrude(xy, tri, z)
    rc = np.linalg.norm(xy[tri].mean(axis=1), axis=1)[ptri]
    region = np.zeros(tet.shape[0], dtype=np.int32)
    region[rc < a] = 1
    region[(rc > R1) & (rc < R2)] = 2
    return Mesh(xyz, tet, region, ["air", "conductor", "coil"],
                {"family": "cylinder", "a": a, "R1": R1, "R2": R2, "R_out": R_out, "H": H, "h": h})


# ---------------------------------------------------------------------------
# Steam-generator tube family
# ---------------------------------------------------------------------------

TUBE_DEFAULTS = dict(
    r_coil=(7.6e-3, 9.1e-3),        # coil annulus radii (both coils)
    r_tube=(9.84e-3, 11.11e-3),     # tube wall
    plate_gap=0.2e-3,               # radial gap between tube and plate
    R_out=30e-3,                    # air cylinder radius
    z_half=100e-3,                  # domain z in [-z_half, z_half]
    plate_half=10e-3,               # plate z in [-plate_half, plate_half]
    scan_half=20e-3,                # fine z-spacing over [-scan_half, scan_half]
    lobe_depth=2.5e-3,              # radial depth of the four flow lobes
    lobe_halfwidth_deg=18.0,        # angular half-width of each lobe
    h_z=0.4e-3,                     # axial spacing in the scan zone
    h_z_end=5e-3,                   # axial spacing at the ends
    h_wall=0.21e-3,                 # radial spacing in the tube wall
    h_coil=0.5e-3,                  # radial spacing in the coil and gap
    h_theta=1.0e-3,                 # target azimuthal spacing
    n_theta_max=64,                 # azimuthal node count cap (reached at the tube)
    h_core=1.5e-3,                  # radial spacing inside the coil
    h_out=3.0e-3,                   # radial spacing at R_out
    deposits=(),                    # tuples (r0, r1, z0, z1) of deposit annuli
)

TUBE_REGIONS = ["air", "tube", "plate", "deposit"]


def tube(**kw) -> Mesh:
    """Tube + lobed support plate + deposits in an air cylinder.

    Regions: 0 air (incl. coils and lobes), 1 tube wall, 2 support plate,
    3 deposit.  Coils are not a region: their current is given per
    tetrahedron by ``synth.sources.coil_current``.
    """
    p = dict(TUBE_DEFAULTS)
    p.update(kw)
    rc0, rc1 = p["r_coil"]
    rt0, rt1 = p["r_tube"]
    rp0 = rt1 + p["plate_gap"]
    R = p["R_out"]
    rads = [
        _uniform(p["h_core"], rc0, p["h_core"]),
        _uniform(rc0, rc1, p["h_coil"]),
        _uniform(rc1, rt0, p["h_coil"]),
        _uniform(rt0, rt1, p["h_wall"]),
        _uniform(rt1, rp0, p["h_wall"]),
        _graded(rp0, rp0 + p["lobe_depth"], p["h_wall"], 2 * p["h_wall"]),
    ]
    r_last = rp0 + p["lobe_depth"]
    rads.append(_graded(r_last, R, 2 * p["h_wall"], p["h_out"]))
    radii = _join(*rads)
    xy, tri = ring_triangulation(radii, h_theta=p["h_theta"], n_min=16, multiple=4, n_max=p["n_theta_max"])
    zs, zp, zh = p["scan_half"], p["plate_half"], p["z_half"]
    zfine = _uniform(-zs, zs, p["h_z"])
    z = _join(-_graded(zs, zh, p["h_z"], p["h_z_end"])[::-1], zfine, _graded(zs, zh, p["h_z"], p["h_z_end"]))
    # snap the plate faces onto z-levels so the plate is z-conforming
    for zz in (-zp, zp):
        z[np.argmin(np.abs(z - zz))] = zz
    xyz, tet, ptri, player = extrude(xy, tri, z)
    c2 = xy[tri].mean(axis=1)
    r2 = np.linalg.norm(c2, axis=1)
    th2 = np.degrees(np.arctan2(c2[:, 1], c2[:, 0])) % 90.0
    zc = 0.5 * (z[player] + z[player + 1])
    rc = r2[ptri]
    region = np.zeros(tet.shape[0], dtype=np.int32)
    region[(rc > rt0) & (rc < rt1)] = 1
    in_plate = (rc > rp0) & (np.abs(zc) < zp)
    lobe = (rc < rp0 + p["lobe_depth"]) & (np.abs(th2[ptri] - 45.0) < p["lobe_halfwidth_deg"])
    region[in_plate & ~lobe] = 2
    for (d0, d1, z0, z1) in p["deposits"]:
        region[(rc > d0) & (rc < d1) & (zc > z0) & (zc < z1) & (region == 0)] = 3
    meta = {"family": "tube", **{k: v for k, v in p.items() if k != "deposits"},
            "deposits": [list(d) for d in p["deposits"]], "n_rings": int(len(radii)), "n_z": int(len(z))}
    return Mesh(xyz, tet, region, list(TUBE_REGIONS), meta)


def tube_materials(freq_hz: float, sigma_tube=1e6, sigma_plate=2e6, sigma_deposit=1e4, mu_r=1.0):
    """(nu[nreg], sigma[nreg], omega) for the tube regions, SI units."""
    mu0 = 4e-7 * np.pi
    nu = np.full(len(TUBE_REGIONS), 1.0 / (mu0 * mu_r))
    sigma = np.array([0.0, sigma_tube, sigma_plate, sigma_deposit])
    return nu, sigma, 2 * np.pi * freq_hz


def perturbed_tube(seed: int, **kw):
    """A tube of the family above with seeded defects, for training and
    held-out evaluation of the learned correction: 1-3 deposit annuli
    (thickness U(0.1, 0.5) mm on the tube's outer surface, length U(2, 10) mm,
    centred in the scan zone) and, with probability 1/2, an axial crack in the
    wall (width one azimuthal cell, depth U(10%, 80%) of the wall from the
    outside, length U(2, 8) mm) whose tetrahedra become air.  Returns the mesh
    and conductivity factors (tube, plate) drawn from U(0.7, 1.3).
    """
    rng = np.random.default_rng(seed)
    p = dict(TUBE_DEFAULTS)
    p.update(kw)
    rt0, rt1 = p["r_tube"]
    zs = p["scan_half"]
    deps = []
    for _ in range(int(rng.integers(1, 4))):
        th = rng.uniform(0.1e-3, 0.5e-3)
        ln = rng.uniform(2e-3, 10e-3)
        zc = rng.uniform(-zs + ln / 2, zs - ln / 2)
        deps.append((rt1, rt1 + th, zc - ln / 2, zc + ln / 2))
    m = tube(deposits=deps, **kw)
    if rng.random() < 0.5:
        cen = m.xyz[m.tet].mean(axis=1)
        r = np.hypot(cen[:, 0], cen[:, 1])
        ang = np.arctan2(cen[:, 1], cen[:, 0])
        a0 = rng.uniform(-np.pi, np.pi)
        half_w = 0.5 * p["h_theta"] / rt1 + 1e-9
        depth = rng.uniform(0.1, 0.8) * (rt1 - rt0)
        ln = rng.uniform(2e-3, 8e-3)
        zc = rng.uniform(-zs + ln / 2, zs - ln / 2)
        dang = np.angle(np.exp(1j * (ang - a0)))
        crack = (m.region == 1) & (np.abs(dang) < 2 * half_w) & (r > rt1 - depth) & (np.abs(cen[:, 2] - zc) < ln / 2)
        m.region = np.where(crack, 0, m.region).astype(np.int32)
        m.meta["crack"] = {"angle": float(a0), "depth": float(depth), "length": float(ln), "z": float(zc),
                           "tets": int(crack.sum())}
    return m, (float(rng.uniform(0.7, 1.3)), float(rng.uniform(0.7, 1.3)))
