"""Plain FP64 CPU oracle for the Coulomb-gauged time-harmonic A-V eddy-current
system (Riahi, "A Fast Eddy-current Non Destructive Testing Finite Element
Solver in Steam Generator", Sections 2-3).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: only the test-suite, the smoke check and the benchmark's
CPU-baseline leg use it.  It shares no code with the GPU path; the only
common inputs are the seeded meshes and currents of the ``synth`` package.

Every step is written for a reader holding the paper: closed-form element
integrals of lowest-order Nedelec (Whitney) and P1 functions, assembly with
``scipy.sparse``, a direct SuperLU solve (the paper's solver family, Section
4) and a plainly written restarted GMRES with the block-Jacobi preconditioner
used on the GPU.  Readings where the paper is silent or garbled:

* gauge: the div-div term of Eqs. 5-7 vanishes identically on Whitney
  elements, so it is realised as the weak-divergence penalty
  tau * W D0^-1 W^T with W_{e,n} = int w_e . grad(lambda_n) and D0 the
  lumped P1 mass;
* sign of grad V: E = i omega A + grad V everywhere (Eq. 2);
* the sigma term of L11 is kept (present in the mixed form, Eq. 7);
* real basis functions make the system complex-symmetric (not Hermitian);
* V is fixed per conductor component by removing its mass-weighted mean
  (first option of Section 4), with an optional delta * sigma * V penalty;
* convergence is measured in the D^-1/2-weighted norm, D = |diag M|.

Parity status per function is listed in ``PINS`` below.
"""

PINS = {
    "topology.build": "pinned: de Rham C.G = 0 exactly; edge counts of the Kuhn cube",
    "elements.element_matrices": "pinned: brute-force quadrature of Whitney/P1 functions",
    "assemble.assemble": "pinned: K.G = 0, W = M1.G, B_sigma = M_sigma.G, symmetry, null-space dimension",
    "assemble.rhs": "pinned: quadrature; G^T b = 0 for divergence-free currents",
    "blocks.rcb_blocks": "pinned: partition invariants (cover, sizes, spatial split)",
    "solve.direct": "pinned: dense numpy.linalg.solve on tiny meshes; residual",
    "solve.gmres": "pinned: agreement with the direct solve; residual history",
    "ibc.*": "pinned: triangle quadrature, surface de Rham identities, thin-sheet limit of a volume layer, "
             "convergence to a resolved volume plate (Leontovich limit) against wrong-normal / real-coefficient mutations",
    "post.*": "pinned: Bessel cylinder closed form, energy identity, reciprocity, passivity, h-convergence",
}
