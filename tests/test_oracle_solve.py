"""Pins for the oracle's solvers: dense brute force on tiny meshes, SuperLU on
the augmented form, and the plain GMRES with block-Jacobi."""
import numpy as np
import pytest

from synth import cube, cube_current
from oracle.assemble import assemble
from oracle.blocks import rcb_blocks, dof_coords
from oracle.post import remove_v_mean
from oracle.solve import direct, solve_gmres, gmres, BlockJacobi, equilibration


def sys_for(n, delta_v=0.0, seed=0):
    m = cube(n)
    s = assemble(m.xyz, m.tet, m.region, nu=[1.0, 1.0], sigma=[0.0, 1.0], omega=50.0, tau=1.0, delta_v=delta_v)
    return m, s, s.rhs(cube_current(m, seed))


@pytest.mark.parametrize("n", [2, 4])
def test_direct_matches_dense(n):
    m, s, b = sys_for(n)
    xd = direct(s, b, dense=True)
    xs = direct(s, b)
    assert np.linalg.norm(xs - xd) <= 1e-10 * np.linalg.norm(xd)
    M = s.matrix()
    assert np.linalg.norm(M @ xd - b) <= 1e-12 * np.linalg.norm(b)


def test_dense_with_delta_v_penalty_is_nonsingular():
    m, s, b = sys_for(4, delta_v=1e-3)
    x = np.linalg.solve(s.matrix().toarray(), b)
    assert np.linalg.norm(direct(s, b) - x) <= 1e-10 * np.linalg.norm(x)


@pytest.mark.parametrize("n,block", [(4, 32), (8, 64)])
def test_gmres_matches_direct(n, block):
    m, s, b = sys_for(n)
    xd = remove_v_mean(s, direct(s, b))
    xg, res = solve_gmres(s, m.xyz, b, block=block, tol=1e-13, max_iter=4000)
    xg = remove_v_mean(s, xg)
    assert res.converged
    assert np.linalg.norm(xg - xd) <= 1e-9 * np.linalg.norm(xd)
    # the reported residual is the true equilibrated residual
    sc = equilibration(s)
    r = sc * (b - s.matvec(xg))
    assert abs(np.linalg.norm(r) / np.linalg.norm(sc * b) - res.relres) <= 1e-3 * res.relres + 1e-16


def test_gmres_unpreconditioned_small_dense():
    """GMRES on a random dense complex system against numpy.linalg.solve."""
    rng = np.random.default_rng(5)
    n = 60
    A = np.eye(n) * 4 + rng.normal(size=(n, n)) * 0.3 + 1j * rng.normal(size=(n, n)) * 0.3
    b = rng.normal(size=n) + 1j * rng.normal(size=n)
    res = gmres(lambda v: A @ v, b, lambda v: v, m=10, tol=1e-13, max_iter=2000)
    assert res.converged and res.restarts > 1
    assert np.linalg.norm(res.x - np.linalg.solve(A, b)) <= 1e-11 * np.linalg.norm(b)
    # full GMRES terminates in at most n steps
    res2 = gmres(lambda v: A @ v, b, lambda v: v, m=n, tol=1e-12, max_iter=n)
    assert res2.iters <= n and res2.converged


def test_block_jacobi_exact_on_block_diagonal():
    """With a single block covering everything, the preconditioner is M^-1."""
    m, s, b = sys_for(2, delta_v=1e-2)
    P = BlockJacobi.build(s, m.xyz, b=10 ** 6)
    z = P.apply(b)
    assert np.linalg.norm(s.matrix() @ z - b) <= 1e-10 * np.linalg.norm(b)


def test_rcb_partition_invariants():
    m, s, _ = sys_for(8)
    c = dof_coords(m.xyz, s.topo.edges, s.topo.cond_nodes)
    for bsz in (16, 64, 100):
        blocks = rcb_blocks(c, bsz)
        allids = np.concatenate(blocks)
        assert np.array_equal(np.sort(allids), np.arange(s.ndof))
        sizes = np.array([x.size for x in blocks])
        assert sizes.max() <= bsz
        # near-equal sizes: at most a factor 2 apart, ceil(n/b) rounded to a power-of-two tree
        assert sizes.min() >= bsz // 4
        for blk in blocks:
            assert np.all(np.diff(blk) > 0)


def test_penalty_free_iteration_returns_the_gauged_solution():
    """GMRES on the operator without the gauge term, then the Coulomb
    projection, gives the gauged system's solution (delta_V = 0,
    divergence-free b); iterating on the gauged operator agrees."""
    from oracle.solve import coulomb_projection, divergence_residual
    m, s, b = sys_for(4)
    assert divergence_residual(s, b) < 1e-13
    xd = remove_v_mean(s, direct(s, b))
    x0, r0 = solve_gmres(s, m.xyz, b, block=32, tol=1e-13, gauge_in_operator=False)
    x1, r1 = solve_gmres(s, m.xyz, b, block=32, tol=1e-13, gauge_in_operator=True)
    for x in (x0, x1):
        assert np.linalg.norm(remove_v_mean(s, x) - xd) <= 1e-9 * np.linalg.norm(xd)
    assert np.linalg.norm(s.W.T @ x0[: s.topo.ne]) <= 1e-12 * np.linalg.norm(s.W.T @ np.abs(x0[: s.topo.ne]))
    # the projection is idempotent and only moves along the kernel
    y = coulomb_projection(s, x0)
    assert np.linalg.norm(y - x0) <= 1e-10 * np.linalg.norm(x0)
