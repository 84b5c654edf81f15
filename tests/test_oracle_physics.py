"""Physics pins for the oracle.

* Bessel cylinder: an infinite conducting cylinder (radius a) inside a
  solenoid current sheet J0 theta-hat on R1 < r < R2.  The time-harmonic
  model of Eq. 1 gives H_z = H0 J_0(k r) / J_0(k a) in the conductor with
  k = (1 + i) / delta, delta = sqrt(2 / (omega mu sigma)) (Section 2, the skin
  depth below Eq. 8), H0 = J0 (R2 - R1) in the gap, J0 (R2 - r) in the coil,
  0 outside; E_theta = k H0 J_1(k r) / (sigma J_0(k a)) in the conductor.  A
  slab with the natural boundary conditions of Eq. 4 reproduces the infinite
  problem exactly, so the discrete field must converge at O(h).
* Manufactured solution: A = grad(q^3) x c with q = x(1-x)y(1-y)z(1-z),
  sigma = 1 everywhere, V = 0.  Then div A = 0, A = 0 and curl A = 0 on the
  boundary, and the source is J = -Laplace(A) - i omega A (first line of Eq. 4).
* Exact discrete identities derived from the block structure of M:
  Joule loss int sigma |E_h|^2 = omega Im(b^T A) and
  Re(b^T A) = A^H (K + tau P) A - delta_V V^H N V;
  reciprocity b_2^T x_1 = b_1^T x_2 (M = M^T); passivity Re Z_kk >= 0.
* Gauge (delta_V = 0, divergence-free b): W^T A = 0 and (A, V) independent
  of tau.
"""
import numpy as np
import pytest
import scipy.special as ss
import sympy as sy

from synth import cube, cube_current, cylinder, solenoid_current
from oracle.assemble import assemble
from oracle.elements import element_matrices
from oracle.post import remove_v_mean, curl_per_tet, joule_loss, edge_field, impedance
from oracle.solve import direct, solve_gmres
from oracle.topology import LOCAL_EDGES


# ---------------------------------------------------------------- Bessel

def bessel_case(h, a=0.5, R1=0.6, R2=0.8, Ro=1.0, delta=0.25):
    omega = 2.0 / delta ** 2
    m = cylinder(a, R1, R2, Ro, H=2 * h, h=h)
    s = assemble(m.xyz, m.tet, m.region, nu=[1.0, 1.0, 1.0], sigma=[0.0, 1.0, 0.0], omega=omega, tau=1.0)
    b = s.rhs(solenoid_current(m, R1, R2, 1.0))
    x, res = solve_gmres(s, m.xyz, b, block=64, tol=1e-11, max_iter=6000)
    assert res.converged
    x = remove_v_mean(s, x)
    B = curl_per_tet(s, m.xyz, m.tet, x[: s.topo.ne])
    c = m.xyz[m.tet].mean(axis=1)
    r = np.hypot(c[:, 0], c[:, 1])
    k = (1 + 1j) / delta
    H0 = R2 - R1
    Hz = np.where(r < a, H0 * ss.jv(0, k * r) / ss.jv(0, k * a),
                  np.where(r < R1, H0, np.where(r < R2, R2 - r, 0.0)))
    vol = s.vol
    err = np.sqrt(np.sum(vol * np.abs(B[:, 2] - Hz) ** 2) / np.sum(vol * np.abs(Hz) ** 2))
    err_conj = np.sqrt(np.sum(vol * np.abs(B[:, 2] - np.conj(Hz)) ** 2) / np.sum(vol * np.abs(Hz) ** 2))
    # E_theta in the conductor
    el = element_matrices(m.xyz, m.tet)
    lam_c = 0.25
    wc = lam_c * (el["grad"][:, LOCAL_EDGES[:, 1]] - el["grad"][:, LOCAL_EDGES[:, 0]])   # w_l at centroid
    A = x[: s.topo.ne]
    Eh = 1j * omega * np.einsum("tl,tlx->tx", s.topo.sign * A[s.topo.tet2edge], wc)
    cond = s.topo.cond_tet
    V = x[s.topo.ne:]
    Vt = V[s.topo.vmap[m.tet[cond]]]
    Eh[cond] += np.einsum("ti,tix->tx", Vt, el["grad"][cond])
    th = np.stack([-c[:, 1], c[:, 0], np.zeros_like(r)], 1) / r[:, None]
    Et = np.einsum("tx,tx->t", Eh, th)[cond]
    Eex = (k * H0 * ss.jv(1, k * r) / ss.jv(0, k * a))[cond]
    errE = np.sqrt(np.sum(vol[cond] * np.abs(Et - Eex) ** 2) / np.sum(vol[cond] * np.abs(Eex) ** 2))
    return err, err_conj, errE, np.abs(B[:, :2]).max() / np.abs(Hz).max()


def test_bessel_cylinder_converges():
    e1, c1, E1, t1 = bessel_case(0.1)
    e2, c2, E2, t2 = bessel_case(0.05)
    assert e1 < 0.07 and e2 < 0.035, (e1, e2)
    assert np.log2(e1 / e2) > 0.8
    assert E1 < 0.12 and E2 < 0.06 and np.log2(E1 / E2) > 0.8, (E1, E2)
    # the conjugate (e^{+i omega t}) field is far off: catches a sign flip of i omega
    assert c1 > 0.5 and c2 > 0.5
    # transverse B is pure discretisation error: O(h) as well
    assert t2 < 0.02 and t1 / t2 > 1.7


# ---------------------------------------------------------------- MMS

def mms_fields(omega):
    x, y, z = sy.symbols("x y z", real=True)
    q = x * (1 - x) * y * (1 - y) * z * (1 - z)
    phi = q ** 3
    c = sy.Matrix([1, -2, 3]) * 1000
    grad = sy.Matrix([sy.diff(phi, v) for v in (x, y, z)])
    A = grad.cross(c)

    def curl(F):
        return sy.Matrix([sy.diff(F[2], y) - sy.diff(F[1], z),
                          sy.diff(F[0], z) - sy.diff(F[2], x),
                          sy.diff(F[1], x) - sy.diff(F[0], y)])

    cA = curl(A)
    J = curl(cA) - sy.I * omega * A
    f = lambda F: sy.lambdify((x, y, z), list(F), "numpy")
    return f(A), f(cA), f(J)


def mms_case(n, omega=10.0):
    fA, fcA, fJ = mms_fields(omega)
    m = cube(n)
    region = np.zeros(m.nt, dtype=np.int32)
    s = assemble(m.xyz, m.tet, region, nu=[1.0], sigma=[1.0], omega=omega, tau=1.0)
    c = m.xyz[m.tet].mean(axis=1)

    def ev(f, pts):
        return np.stack([np.broadcast_to(np.asarray(v, dtype=complex), pts.shape[:1]) for v in f(*pts.T)], 1)

    # per-tet source: average of J over the 4-point (degree-2) rule
    a_, b_ = 0.5854101966249685, 0.1381966011250105
    P = m.xyz[m.tet]
    Jk = np.zeros((m.nt, 3), dtype=complex)
    for i in range(4):
        wts = np.full(4, b_)
        wts[i] = a_
        Jk += 0.25 * ev(fJ, np.einsum("j,tjx->tx", wts, P))
    b = s.rhs(Jk.real) + 1j * s.rhs(Jk.imag)
    x, res = solve_gmres(s, m.xyz, b, block=64, tol=1e-12, max_iter=8000)
    assert res.converged
    x = remove_v_mean(s, x)
    B = curl_per_tet(s, m.xyz, m.tet, x[: s.topo.ne])
    Bex = ev(fcA, c)
    el = element_matrices(m.xyz, m.tet)
    wc = 0.25 * (el["grad"][:, LOCAL_EDGES[:, 1]] - el["grad"][:, LOCAL_EDGES[:, 0]])
    Ah = np.einsum("tl,tlx->tx", s.topo.sign * x[: s.topo.ne][s.topo.tet2edge], wc)
    Aex = ev(fA, c)
    vol = s.vol[:, None]
    eB = np.sqrt(np.sum(vol * np.abs(B - Bex) ** 2) / np.sum(vol * np.abs(Bex) ** 2))
    eA = np.sqrt(np.sum(vol * np.abs(Ah - Aex) ** 2) / np.sum(vol * np.abs(Aex) ** 2))
    return eB, eA, np.abs(x[s.topo.ne:]).max() / np.abs(x[: s.topo.ne]).max()


def test_manufactured_solution_h_convergence():
    e4 = mms_case(4)
    e8 = mms_case(8)
    e16 = mms_case(16)
    for k in (0, 1):
        r1 = np.log2(e4[k] / e8[k])
        r2 = np.log2(e8[k] / e16[k])
        assert r2 > 0.85, (k, e4, e8, e16)
        assert e16[k] < e8[k] < e4[k]
    assert e16[0] < 0.2 and e16[1] < 0.2
    # V -> 0 under refinement (the exact V is zero)
    assert e16[2] < 1e-3 and e8[2] / e16[2] > 4 and e4[2] / e8[2] > 4


# ---------------------------------------------------------------- identities

@pytest.mark.parametrize("delta_v", [0.0, 1e-3])
def test_energy_identities(delta_v):
    m = cube(8)
    s = assemble(m.xyz, m.tet, m.region, nu=[1.0, 1.0], sigma=[0.0, 1.0], omega=50.0, tau=1.0, delta_v=delta_v)
    b = s.rhs(cube_current(m, 0))
    x = direct(s, b)
    x = remove_v_mean(s, x) if delta_v == 0 else x
    ne = s.topo.ne
    A, V = x[:ne], x[ne:]
    btA = b[:ne] @ A
    assert abs(joule_loss(s, x) - s.omega * btA.imag) <= 1e-10 * abs(btA)
    P = s.W @ ((s.W.T @ A) / s.D0)
    quad = np.real(np.conj(A) @ (s.K @ A) + s.tau * np.conj(A) @ P) - delta_v * np.real(np.conj(V) @ (s.Nsig @ V))
    assert abs(btA.real - quad) <= 1e-10 * abs(btA)


def test_reciprocity_and_passivity():
    m = cube(8)
    s = assemble(m.xyz, m.tet, m.region, nu=[1.0, 1.0], sigma=[0.0, 1.0], omega=50.0, tau=1.0)
    b1 = s.rhs(cube_current(m, 0))
    b2 = s.rhs(cube_current(m, 1))
    x1 = direct(s, b1)
    x2 = direct(s, b2)
    Z = impedance(s, [b1, b2], [x1, x2], [1.0, 1.0])
    assert abs(Z[0, 1] - Z[1, 0]) <= 1e-10 * abs(Z[0, 1])
    assert Z[0, 0].real > 0 and Z[1, 1].real > 0
    # Im Z_kk = -omega L_kk < 0 (inductive, e^{-i omega t} convention)
    assert Z[0, 0].imag < 0 and Z[1, 1].imag < 0


def test_gauge_tau_independence():
    m = cube(4)
    sols = []
    for tau in (0.1, 1.0, 10.0):
        s = assemble(m.xyz, m.tet, m.region, nu=[1.0, 1.0], sigma=[0.0, 1.0], omega=50.0, tau=tau)
        b = s.rhs(cube_current(m, 2))
        x = remove_v_mean(s, direct(s, b))
        ne = s.topo.ne
        assert np.linalg.norm(s.W.T @ x[:ne]) <= 1e-10 * np.linalg.norm(s.W.T @ np.abs(x[:ne]))
        sols.append(x)
    for x in sols[1:]:
        assert np.linalg.norm(x[:ne] - sols[0][:ne]) <= 1e-9 * np.linalg.norm(sols[0][:ne])
        assert np.linalg.norm(x[ne:] - sols[0][ne:]) <= 1e-8 * np.linalg.norm(sols[0][ne:])
