"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every symbol the header declares, builds the same topology and block
partition as the oracle, and rejects bad input with the documented codes."""
import os
import re

import numpy as np
import pytest

from synth import cube, tube

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def lib():
    from paper_1602_03207_amd import eddy
    return eddy


def test_exports_every_declared_symbol():
    eddy = lib()
    hdr = open(os.path.join(ROOT, "include", "eddy.h")).read()
    declared = set(re.findall(r"^\s*(?:const char\*|void|eddy_status)\s+(eddy_\w+)\s*\(", hdr, re.M))
    assert len(declared) >= 20
    for name in declared:
        assert hasattr(eddy._lib, name), name
    assert declared == set(eddy.EXPORTS)


def test_mesh_matches_oracle_topology_c1():
    from oracle.topology import build
    from oracle.blocks import rcb_blocks, dof_coords
    eddy = lib()
    m = cube(8)
    M = eddy.Mesh(m.xyz, m.tet, m.region, [0, 1])
    t = build(m.tet, m.nv, m.region, [1])
    assert (M.ne, M.nc, M.ncomp) == (t.ne, t.nc, t.ncomp) == (4184, 125, 1)
    assert M.nnz == 70717 and M.nnz_w == 27952
    assert np.array_equal(M.edges(), t.edges)
    assert np.array_equal(M.conductor_nodes(), t.cond_nodes)
    for b in (16, 64):
        ptr, dofs = M.blocks(b)
        ob = rcb_blocks(dof_coords(m.xyz, t.edges, t.cond_nodes), b)
        assert len(ptr) - 1 == len(ob)
        for k, blk in enumerate(ob):
            assert np.array_equal(dofs[ptr[k]:ptr[k + 1]], blk)


def test_mesh_matches_oracle_small_tube():
    from oracle.topology import build
    from oracle.blocks import rcb_blocks, dof_coords
    eddy = lib()
    m = tube(h_z=2e-3, h_z_end=20e-3, h_theta=2.5e-3, n_theta_max=32, h_wall=0.5e-3, h_coil=1.0e-3,
             h_core=2e-3, h_out=6e-3)
    M = eddy.Mesh(m.xyz, m.tet, m.region, [0, 1, 1, 1])
    t = build(m.tet, m.nv, m.region, [1, 2, 3])
    assert np.array_equal(M.edges(), t.edges)
    assert np.array_equal(M.conductor_nodes(), t.cond_nodes)
    assert M.ncomp == t.ncomp == 2
    ptr, dofs = M.blocks(64)
    ob = rcb_blocks(dof_coords(m.xyz, t.edges, t.cond_nodes), 64)
    assert len(ob) == len(ptr) - 1
    assert all(np.array_equal(dofs[ptr[k]:ptr[k + 1]], ob[k]) for k in range(len(ob)))


def test_bad_inputs_rejected():
    eddy = lib()
    m = cube(2)
    bad = m.tet.copy()
    bad[0, 0] = m.nv + 5
    with pytest.raises(eddy.EddyError, match="invalid argument"):
        eddy.Mesh(m.xyz, bad, m.region, [0, 1])
    flat = m.tet.copy()
    flat[0] = [0, 1, 2, 2]          # degenerate: repeated node
    with pytest.raises(eddy.EddyError, match="invalid mesh"):
        eddy.Mesh(m.xyz, flat, m.region, [0, 1])
    reg = m.region.copy()
    reg[3] = 7
    with pytest.raises(eddy.EddyError, match="invalid argument"):
        eddy.Mesh(m.xyz, m.tet, reg, [0, 1])
    M = eddy.Mesh(m.xyz, m.tet, m.region, [0, 1])
    with pytest.raises(eddy.EddyError):
        M.blocks(0)
    with pytest.raises(eddy.EddyError):
        M.blocks(65)


def test_either_tet_orientation_accepted():
    eddy = lib()
    m = cube(3)
    tet = m.tet.copy()
    tet[::2] = tet[::2][:, [1, 0, 2, 3]]
    M1 = eddy.Mesh(m.xyz, m.tet, m.region, [0, 1])
    M2 = eddy.Mesh(m.xyz, tet, m.region, [0, 1])
    assert np.array_equal(M1.edges(), M2.edges()) and M1.nnz == M2.nnz


def test_ect_signals_host_call_matches_oracle():
    """eddy_ect_signals runs on the host: Eq. 11 against the oracle on seeded
    values, with and without the defect-free matrices."""
    from oracle.post import ect_signals as oracle_signals
    eddy = lib()
    rng = np.random.default_rng(5)
    Zd = rng.normal(size=(7, 2, 2)) + 1j * rng.normal(size=(7, 2, 2))
    Z0 = rng.normal(size=(7, 2, 2)) + 1j * rng.normal(size=(7, 2, 2))
    dZ, fa, f3 = eddy.ect_signals(Zd, Z0)
    odZ, ofa, of3 = oracle_signals(Zd, Z0)
    assert np.allclose(dZ, odZ, rtol=0, atol=1e-15)
    assert np.allclose(fa, ofa, rtol=0, atol=1e-15) and np.allclose(f3, of3, rtol=0, atol=1e-15)
    dZ2, fa2, f32 = eddy.ect_signals(dZ)
    assert np.array_equal(dZ2, dZ) and np.allclose(fa2, ofa, rtol=0, atol=1e-15)
    assert eddy.ect_signals(np.zeros((0, 2, 2)))[1].shape == (0,)


@pytest.mark.parametrize("case", ["c1", "tube"])
def test_subdomains_and_adjacency_match_oracle(case):
    """Learned-correction subdomains (host) against the oracle's construction
    from its own block partition and matrix pattern."""
    import oracle.gnn as G
    from oracle.assemble import assemble
    from oracle.blocks import rcb_blocks, dof_coords
    eddy = lib()
    if case == "c1":
        m, cond, nu, sig = cube(8), [1], [1.0, 1.0], [0.0, 1.0]
    else:
        m = tube(h_z=4e-3, h_z_end=20e-3, h_theta=3e-3, n_theta_max=24, h_wall=0.6e-3, h_coil=1.5e-3,
                 h_core=3e-3, h_out=8e-3)
        cond, nu, sig = [1, 2, 3], [1.0] * 4, [0.0, 1.0, 2.0, 0.5]
    flags = [1 if r in cond else 0 for r in range(len(nu))]
    M = eddy.Mesh(m.xyz, m.tet, m.region, flags)
    sub, adj = M.subdomains(64)
    s = assemble(m.xyz, m.tet, m.region, nu, sig, 1.0, conductor_regions=cond)
    blocks = rcb_blocks(dof_coords(m.xyz, s.topo.edges, s.topo.cond_nodes), 64)
    osub = G.subdomains(blocks)
    assert np.array_equal(sub, osub)
    assert np.array_equal(adj, G.adjacency(s.topo, np.asarray(m.tet), osub))
    assert adj.sum() > 0 and np.array_equal(adj, adj.T)
