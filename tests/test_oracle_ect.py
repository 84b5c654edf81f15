"""Pins of the eddy-current-testing outputs of the oracle (Section 2, Eqs. 11
and 12).

* Eq. 12 (the impedance change as a volume integral over the defect) against
  the plain definition dZ = Z_defect - Z_free, each Z from its own direct
  solve: the two agree only if the assembled sigma-coupling blocks (B, S),
  the element mass and curl, and the sign convention E = i omega A + grad V
  are mutually consistent, so a dropped term, a sign or a transposed
  operand in any of them fails this test.  The tetrahedra's local vertex
  order is shuffled so that both edge orientations occur.  Cases: a conducting and magnetic
  defect touching the conductor (one conductor component) and a detached one
  (its own component, its own V constant).
* dZ is symmetric (reciprocity), which the volume form does not impose.
* Eq. 11 on a hand-worked example.
"""
import numpy as np
import pytest

from synth import cube, cube_current
from oracle.assemble import assemble
from oracle.post import delta_z_volume, ect_signals, impedance
from oracle.solve import direct


def defect_cube(box):
    """cube(8) with a defect box (region 2) and the local vertex order of every
    tetrahedron shuffled (seeded), so that edge orientations take both signs."""
    m = cube(8)
    rng = np.random.default_rng(7)
    m.tet = np.take_along_axis(m.tet, np.argsort(rng.random(m.tet.shape), axis=1), axis=1).astype(np.int32)
    cen = m.xyz[m.tet].mean(axis=1)
    lo, hi = np.array(box[0]), np.array(box[1])
    inbox = np.all((cen > lo) & (cen < hi), axis=1) & (m.region == 0)
    region = m.region.copy()
    region[inbox] = 2
    return m, region


@pytest.mark.parametrize("box", [((0.75, 0.375, 0.375), (0.875, 0.625, 0.625)),
                                 ((0.875, 0.25, 0.5), (1.0, 0.5, 0.75))], ids=["attached", "detached"])
def test_volume_delta_z_equals_impedance_difference(box):
    m, region = defect_cube(box)
    assert (region == 2).sum() >= 12
    omega = 40.0
    nu0, sig0 = np.array([1.0, 1.0, 1.0]), np.array([0.0, 1.0, 0.0])
    nud, sigd = np.array([1.0, 1.0, 0.5]), np.array([0.0, 1.0, 0.3])
    s0 = assemble(m.xyz, m.tet, region, nu0, sig0, omega, tau=1.0, conductor_regions=[1])
    sd = assemble(m.xyz, m.tet, region, nud, sigd, omega, tau=1.0, conductor_regions=[1, 2])
    assert sd.topo.nc > s0.topo.nc
    J = [cube_current(m, 3), cube_current(m, 4)]
    cur = [1.0, 2.0]
    b0 = [s0.rhs(j) for j in J]
    bd = [sd.rhs(j) for j in J]
    x0 = [direct(s0, b) for b in b0]
    xd = [direct(sd, b) for b in bd]
    Z0 = impedance(s0, b0, x0, cur)
    Zd = impedance(sd, bd, xd, cur)
    dZ = delta_z_volume(m.xyz, m.tet, region, sd, nud, sigd, xd, s0, nu0, sig0, x0, cur, cur)
    diff = Zd - Z0
    assert np.max(np.abs(diff)) > 1e-4 * np.max(np.abs(Z0))          # the defect is visible
    assert np.max(np.abs(dZ - diff)) <= 1e-9 * np.max(np.abs(diff))
    assert abs(dZ[0, 1] - dZ[1, 0]) <= 1e-9 * abs(dZ[0, 1])
    # the magnetic and the ohmic parts are both present
    dZ_ohm = delta_z_volume(m.xyz, m.tet, region, sd, nu0, sigd, xd, s0, nu0, sig0, x0, cur, cur)
    assert np.max(np.abs(dZ_ohm - dZ)) > 1e-3 * np.max(np.abs(dZ))


def test_ect_signals_hand_example():
    dZ = np.array([[[1 + 2j, 3 - 1j], [3 - 1j, -2 + 0.5j]]])
    Zd = dZ + 5.0
    Z0 = np.full_like(dZ, 5.0)
    d, fa, f3 = ect_signals(Zd, Z0)
    # (i/2)(4 + i) = -0.5 + 2i ;  (i/2)(3 + 1.5i) = -0.75 + 1.5i
    assert np.allclose(d, dZ, rtol=0, atol=1e-15)
    assert abs(fa[0] - (-0.5 + 2j)) <= 1e-15 and abs(f3[0] - (-0.75 + 1.5j)) <= 1e-15
