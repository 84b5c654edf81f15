"""Pins for the oracle's topology and global assembly.

Truth sources: the discrete de Rham sequence (exact integer identity C G = 0
and the commuting identities K G = 0, W = M_1 G, B_sigma = M_sigma G_c),
complex symmetry of M (real basis functions, Section 2), the dimension of the
un-gauged kernel {(G psi, -i omega psi|_c)} (= number of nodes), the edge
count of the Kuhn cube (Euler: E = V + F - C - 1 for the cell complex), and
divergence-free right-hand sides for divergence-free currents.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from synth import cube, cube_current, tube
from oracle.assemble import assemble
from oracle.topology import build, gradient_matrix, curl_matrix


def cube_system(n, omega=50.0, tau=1.0, delta_v=0.0, sigma_out=0.0):
    m = cube(n)
    return m, assemble(m.xyz, m.tet, m.region, nu=[1.0, 1.0], sigma=[sigma_out, 1.0], omega=omega,
                       tau=tau, delta_v=delta_v, conductor_regions=[1] if sigma_out == 0 else [0, 1])


def test_counts_c1():
    m, s = cube_system(8)
    t = s.topo
    assert (m.nv, m.nt, t.ne, int(t.cond_tet.sum()), t.nc, t.ndof) == (729, 3072, 4184, 384, 125, 4309)
    assert t.ncomp == 1


@pytest.mark.parametrize("n", [2, 3, 5])
def test_euler_characteristic(n):
    m = cube(n)
    t = build(m.tet, m.nv, m.region, [1])
    nf = curl_matrix(m.tet, t).shape[0]
    # Euler characteristic of a ball: V - E + F - T = 1
    assert m.nv - t.ne + nf - m.nt == 1


def test_de_rham_exact_integer():
    m = cube(4)
    t = build(m.tet, m.nv, m.region, [1])
    CG = curl_matrix(m.tet, t) @ gradient_matrix(t)
    assert CG.count_nonzero() == 0 or np.max(np.abs(CG.data)) == 0.0


def test_de_rham_tube():
    m = tube(h_z=4e-3, h_z_end=20e-3, h_theta=3e-3, n_theta_max=24, h_wall=0.6e-3, h_coil=1.5e-3,
             h_core=3e-3, h_out=8e-3)
    t = build(m.tet, m.nv, m.region, [1, 2, 3])
    CG = curl_matrix(m.tet, t) @ gradient_matrix(t)
    assert np.max(np.abs(CG.data), initial=0.0) == 0.0


def test_stiffness_kills_gradients_and_W_is_mass_times_gradient():
    m, s = cube_system(4)
    G = gradient_matrix(s.topo)
    assert np.max(np.abs((s.K @ G).data), initial=0.0) <= 1e-12 * np.max(np.abs(s.K.data))
    s1 = assemble(m.xyz, m.tet, m.region, nu=[1.0, 1.0], sigma=[1.0, 1.0], omega=50.0,
                  conductor_regions=[1])
    d = (s.W - s1.Msig @ G)
    assert np.max(np.abs(d.data), initial=0.0) <= 1e-14 * np.max(np.abs(s.W.data))
    Gc = G[:, s.topo.cond_nodes]
    d2 = s.Bsig - s.Msig @ Gc
    assert np.max(np.abs(d2.data), initial=0.0) <= 1e-14 * np.max(np.abs(s.Bsig.data))


def test_matrix_complex_symmetric_not_hermitian():
    _, s = cube_system(4)
    M = s.matrix()
    assert abs(M - M.T).max() <= 1e-14 * abs(M).max()
    assert abs(M - M.conj().T).max() > 1e-3 * abs(M).max()


def test_ungauged_kernel_dimension_is_node_count():
    m, s = cube_system(4)
    M0 = s.matrix_no_gauge().toarray()
    sv = np.linalg.svd(M0, compute_uv=False)
    k = int(np.sum(sv < 1e-10 * sv[0]))
    assert k == m.nv == 125
    # and the gauge removes every direction but the V constant per component
    sv2 = np.linalg.svd(s.matrix().toarray(), compute_uv=False)
    assert int(np.sum(sv2 < 1e-10 * sv2[0])) == s.topo.ncomp


def test_kernel_vectors_explicit():
    """(G psi, -i omega psi|_c) is annihilated by the un-gauged matrix."""
    m, s = cube_system(4)
    rng = np.random.default_rng(3)
    psi = rng.normal(size=m.nv)
    x = np.concatenate([gradient_matrix(s.topo) @ psi, -1j * s.omega * psi[s.topo.cond_nodes]])
    y = s.matrix_no_gauge() @ x
    assert np.linalg.norm(y) <= 1e-12 * np.linalg.norm(s.matrix_no_gauge().toarray()) * np.linalg.norm(x)


def test_rhs_divergence_free_and_quadrature():
    m, s = cube_system(8)
    J = cube_current(m, seed=0)
    b = s.rhs(J)
    G = gradient_matrix(s.topo)
    assert np.linalg.norm(G.T @ b[: s.topo.ne]) <= 1e-13 * np.linalg.norm(b)
    assert np.all(b[s.topo.ne:] == 0)
    # b_e = int J . w_e for constant J: equals M_1 applied to the edge
    # interpolant of J (constant fields lie in the Nedelec space, Section 3's
    # "mass matrix times interpolant" rule) -- check for a uniform J
    J0 = np.array([0.3, -1.2, 0.7])
    b0 = s.rhs(np.tile(J0, (m.nt, 1)))
    s1 = assemble(m.xyz, m.tet, m.region, nu=[1.0, 1.0], sigma=[1.0, 1.0], omega=1.0, conductor_regions=[1])
    interp = (m.xyz[s.topo.edges[:, 1]] - m.xyz[s.topo.edges[:, 0]]) @ J0
    assert np.allclose(b0[: s.topo.ne].real, s1.Msig @ interp, rtol=1e-12, atol=1e-15)


def test_lumped_mass_is_volume():
    m, s = cube_system(4)
    assert abs(s.D0.sum() - 1.0) < 1e-14
    assert abs(s.lumped_c.sum() - 0.125) < 1e-14
