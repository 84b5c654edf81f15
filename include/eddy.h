/*
 * eddy.h -- C ABI of the MI355X eddy-current A-V solver.
 *
 * Solves the time-harmonic, Coulomb-gauged A-V eddy-current system of
 * Riahi, "A Fast Eddy-current Non Destructive Testing Finite Element Solver
 * in Steam Generator": the model of Section 2 (Eq. 1), potentials
 * E = i omega A + grad V, mu H = curl A (Eq. 2), the mixed sesquilinear form
 * L of Eq. 7 with its blocks L11, L12, L21, L22, and the global block system
 * of Section 3 with right-hand side (J_h ; 0).  A is discretised with
 * lowest-order Nedelec (Whitney) edge elements, V with P1 on the nodes of
 * the conducting sub-mesh:
 *
 *   M11 = K_nu + tau W D0^-1 W^T - i omega M_sigma      (A rows, A columns)
 *   M12 = -B_sigma,  M21 = -B_sigma^T                     (A-V coupling)
 *   M22 = (i / omega) S_sigma + delta_V N_sigma           (V rows, V columns)
 *
 * The div-div gauge term of Eqs. 5-7 vanishes on Whitney elements and is
 * realised as the weak-divergence penalty tau W D0^-1 W^T, W = int w_e.grad l_n,
 * D0 the lumped P1 mass.  The matrix is complex-symmetric.
 *
 * Conventions (every call):
 *   - SI units; time factor e^{-i omega t} (Eq. 1).
 *   - DOF order [A on edges ; V on conductor nodes].  Edges are the sorted
 *     node pairs (lo, hi) in lexicographic order, oriented lo -> hi;
 *     conductor nodes are in increasing global node id.
 *   - Complex values are interleaved (re, im) doubles (eddy_c128).
 *   - "dev" pointers are device (HBM) pointers owned by the caller; "host"
 *     pointers are host memory owned by the caller.  Host inputs are copied
 *     during the call.  The library never allocates device memory: every
 *     device buffer comes from a caller-owned workspace whose size it
 *     reports.  Handles own host metadata only.
 *   - `stream` is a hipStream_t (0 = the null stream).  Calls that return
 *     host data synchronise that stream; the others only enqueue work.
 *   - Every call returns an eddy_status; negative = error (message in
 *     eddy_last_error(), thread-local), positive = warning.  No call throws.
 */
#ifndef EDDY_H
#define EDDY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  EDDY_OK = 0,
  EDDY_ERR_ARG = -1,             /* invalid argument or size                 */
  EDDY_ERR_MESH = -2,            /* degenerate tetrahedron / bad indices     */
  EDDY_ERR_WORKSPACE = -3,       /* workspace missing or too small           */
  EDDY_ERR_DEVICE = -4,          /* HIP runtime error                        */
  EDDY_ERR_SINGULAR_BLOCK = -5,  /* zero pivot in a preconditioner block     */
  EDDY_WARN_NOT_CONVERGED = 1    /* solve hit max_iter; x holds the iterate  */
} eddy_status;

typedef struct { double re, im; } eddy_c128;
typedef void* eddy_stream;                 /* hipStream_t */
typedef struct eddy_mesh eddy_mesh;        /* opaque, host */
typedef struct eddy_op eddy_op;            /* opaque, host metadata + workspace view */

typedef struct {
  double tau_gauge;    /* gauge penalty 1/mu~ (Eq. 3); > 0                        */
  double delta_v;      /* optional V penalty delta*sigma*V (Section 4); >= 0      */
  int32_t block_size;  /* block-Jacobi block size b, 1..64                         */
  double tau_precond;  /* penalty inside the block-Jacobi blocks (a preconditioner */
                       /* parameter: they must be invertible); 0 = tau_gauge      */
} eddy_params;

typedef struct {
  double tol;          /* stop when ||D^-1/2 (b - M x)|| <= tol ||D^-1/2 b||      */
  int32_t restart;     /* GMRES restart length m, 1..64                            */
  int32_t max_iter;    /* total Arnoldi steps                                      */
  int32_t precision;   /* 0: FP64 throughout.  1: mixed -- each cycle's Krylov     */
                       /* process (SpMV, block-Jacobi apply, CGS2, basis) runs in  */
                       /* complex64; cycle residual, Hessenberg least squares,     */
                       /* solution update and final residual stay FP64.  2: as 1, */
                       /* with the block-Jacobi inverses and the Krylov basis     */
                       /* stored in complex half precision (IEEE binary16 parts;  */
                       /* the unit basis vectors scaled by 2^14), float32         */
                       /* arithmetic; with gnn_theta the basis stays complex64    */
  const float* gnn_theta;  /* NULL: plain block-Jacobi.  Otherwise the device      */
                           /* parameters (EDDY_GNN_PARAMS floats) of the learned    */
                           /* coarse correction, applied inside flexible GMRES     */
                           /* with fallback (see eddy_gnn_* below)                 */
  int32_t graph;       /* 1: run the Arnoldi steps between two reads of the        */
                       /* residual estimates (8 steps) as captured HIP graphs,     */
                       /* kept per operator for the last solve workspace,         */
                       /* precision, restart length and operator mode (a new one   */
                       /* recaptures).  eddy_solve only; not used in learned or    */
                       /* profiled cycles.  Results are identical to graph = 0.    */
} eddy_solve_opts;

typedef struct {
  int32_t iters;       /* Arnoldi steps taken                                      */
  int32_t restarts;    /* completed cycles                                         */
  int32_t converged;   /* 1 if the true weighted residual met tol                  */
  int32_t breakdown;   /* 1 if a zero residual estimate ended the solve: the cycle
                          that produced it did not reduce the true residual (a
                          zero estimate with progress only restarts)             */
  double relres;       /* true weighted relative residual of the returned x        */
  double est_relres;   /* Arnoldi estimate at exit                                 */
  double seconds;      /* wall time of the call                                    */
  int32_t gauge_in_operator;  /* 1: iterated on the gauged operator; 0: on the    */
                              /* penalty-free operator + Coulomb projection        */
  int32_t cg_iters;    /* CG steps of the projection's nodal Poisson solve         */
  double div_residual; /* ||G^T b_A|| / ||b||: discrete divergence of the source   */
  int32_t precision_used;  /* 1 if the complex64 inner loop ran (mixed mode needs */
                           /* the penalty-free operator; else FP64 is used)        */
  int32_t reorth_steps;    /* Arnoldi steps whose basis vector got the second      */
                           /* Gram-Schmidt pass: every step in eddy_solve (delayed */
                           /* scheme); in eddy_solve_batched, the steps where the  */
                           /* norm dropped below 1/sqrt(2) of ||w||                */
  int32_t learned_cycles;  /* cycles run with the learned correction               */
  int32_t fell_back;       /* 1 if the plain residual judged the learned cycles    */
                           /* worse and the solve returned to plain block-Jacobi   */
} eddy_solve_report;

/* Launch shapes the operator picked by timing candidates on its own matrix
 * at its first eddy_op_assemble (see eddy_op_tuning). */
typedef struct {
  int32_t spmv_grid_full;   /* workgroups of an uncapped SpMV launch (one per 4 slices) */
  int32_t spmv_grid_c128;   /* chosen cap for the complex128 SpMV (0 = uncapped)       */
  int32_t spmv_grid_c64;    /* chosen cap for the complex64 SpMV (0 = uncapped)        */
  int32_t spmv_sched_c128;  /* chosen schedule: 0 all XCDs sweep the rows together,    */
  int32_t spmv_sched_c64;   /*   1 each XCD takes a contiguous range of rows           */
  float spmv_us_c128;       /* measured time per SpMV at the chosen shape, microseconds */
  float spmv_us_c64;
  float spmv_us_sched_c128[2];  /* best time of each schedule                          */
  float spmv_us_sched_c64[2];
  int64_t sell_nnz_real;    /* nonzeros in the sliced-ELL slices whose values are all  */
                            /* real (stored real: 8-byte and 4-byte values in the     */
                            /* complex128 and complex64 copies)                       */
} eddy_tuning;

/* ---- mesh (host) -------------------------------------------------------
 * eddy_mesh_create: nv nodes xyz[nv*3] (host, metres), nt tetrahedra
 * tet[nt*4] (host, 0-based node ids, either orientation), region[nt]
 * (host, 0..nreg-1), is_conductor[nreg] (host, nonzero = conducting region,
 * i.e. sigma > 0 there; V lives on the nodes of those tetrahedra).  Builds
 * edges, the CSR pattern of M and of W, scatter maps, conductor components.
 * Errors: EDDY_ERR_ARG (sizes, indices), EDDY_ERR_MESH (|det| below
 * 1e-12 * (longest edge)^3). */
eddy_status eddy_mesh_create(int64_t nv, const double* xyz, int64_t nt, const int32_t* tet,
                             const int32_t* region, int32_t nreg, const int32_t* is_conductor,
                             eddy_mesh** out);
/* eddy_mesh_create_ibc: as eddy_mesh_create, plus nf impedance-boundary
 * triangles face[nf*3] (host, node ids, any order) with face_region[nf]
 * (host): the impedance boundary condition of Section 2, Eqs. 8-10, on the
 * boundary Gamma_p of a plate that is not meshed.  With Z = (1 - i) /
 * (delta sigma) and delta = sqrt(2 / (omega mu sigma)) of the face's
 * region (sigma, nu = 1/mu as given at eddy_op_assemble), the plate enters
 * as a surface conductor of coefficient 1/Z: M11 gains -i omega (1/Z) int
 * w_e . w_f, M12 = M21^T gains -(1/Z) int w_e . grad l_n and M22 gains
 * (i/omega)(1/Z) int grad l_m . grad l_n over the triangles (tangential
 * traces, surface gradients).  V lives on the triangles' nodes, which join
 * conductor components like conducting tetrahedra (lumped weights |T|/3).
 * Every face region must be flagged conducting; every triangle edge must
 * be an edge of the tetrahedra.  Errors as eddy_mesh_create, plus
 * EDDY_ERR_ARG for face indices or regions and EDDY_ERR_MESH for repeated
 * nodes or an edge not in the mesh.  eddy_ibc_split builds such a mesh. */
eddy_status eddy_mesh_create_ibc(int64_t nv, const double* xyz, int64_t nt, const int32_t* tet,
                                 const int32_t* region, int32_t nreg, const int32_t* is_conductor,
                                 int64_t nf, const int32_t* face, const int32_t* face_region,
                                 eddy_mesh** out);
/* eddy_ibc_split (host only): remove the tetrahedra of the regions with
 * is_ibc[r] != 0 and return the rest with its nodes renumbered in
 * increasing old id (node_map[nv]: new id or -1), and the interface
 * triangles (faces of a removed tetrahedron that are also faces of a kept
 * one; node triples increasing, in lexicographic order) with the region of
 * the removed tetrahedron.  Call once with every output array NULL to get
 * nv_out, nt_out, nf_out, then with arrays of those sizes (xyz_out
 * [nv_out*3], tet_out [nt_out*4], region_out [nt_out], face_out [nf_out*3],
 * face_region_out [nf_out], node_map [nv]); all caller-owned.  Errors:
 * EDDY_ERR_ARG (sizes, indices, some but not all outputs NULL). */
eddy_status eddy_ibc_split(int64_t nv, const double* xyz, int64_t nt, const int32_t* tet,
                           const int32_t* region, int32_t nreg, const int32_t* is_ibc, int64_t* nv_out,
                           int64_t* nt_out, int64_t* nf_out, double* xyz_out, int32_t* tet_out,
                           int32_t* region_out, int32_t* face_out, int32_t* face_region_out,
                           int32_t* node_map);
void eddy_mesh_destroy(eddy_mesh* mesh);
/* Counts: edges, conductor nodes, nnz of the stored M (structural pattern of
 * all element couplings, gauge excluded), nnz of W, conductor components. */
eddy_status eddy_mesh_counts(const eddy_mesh* mesh, int64_t* ne, int64_t* nc, int64_t* nnz,
                             int64_t* nnz_w, int32_t* ncomp);
/* edge_nodes[ne*2] (host): (lo, hi) per edge.  cond_nodes[nc] (host). */
eddy_status eddy_mesh_edges(const eddy_mesh* mesh, int32_t* edge_nodes);
eddy_status eddy_mesh_conductor_nodes(const eddy_mesh* mesh, int32_t* cond_nodes);
/* Block-Jacobi partition for block size b (recursive coordinate bisection of
 * the DOF positions: edge midpoints and conductor nodes).  Call with
 * block_ptr = block_dofs = NULL to get *nblocks; then block_ptr[nblocks+1]
 * and block_dofs[ndof] (host) receive the blocks in order. */
eddy_status eddy_mesh_blocks(const eddy_mesh* mesh, int32_t block_size, int64_t* nblocks,
                             int32_t* block_ptr, int32_t* block_dofs);

/* ---- operator ----------------------------------------------------------
 * eddy_op_workspace_bytes: device bytes the operator needs for `params`.
 * eddy_op_create: uploads mesh data and maps into dev_ws (device, >= bytes,
 * 256-byte aligned, owned by the caller and kept alive until
 * eddy_op_destroy).  The mesh may be destroyed afterwards. */
eddy_status eddy_op_workspace_bytes(const eddy_mesh* mesh, const eddy_params* params, size_t* bytes);
eddy_status eddy_op_create(const eddy_mesh* mesh, const eddy_params* params, void* dev_ws,
                           size_t ws_bytes, eddy_stream stream, eddy_op** out);
void eddy_op_destroy(eddy_op* op);
/* Assemble M for nu[nreg] = 1/mu (host), sigma[nreg] (host, S/m; zero
 * exactly on the non-conducting regions) and omega (rad/s): element kernel,
 * deterministic scatter into CSR (no atomics), W and D0, symmetric
 * equilibration D^-1/2 M D^-1/2 with D = |diag M|, then the dense inverses of
 * the preconditioner's diagonal blocks (gauge included).  Reusable: call
 * again for new materials or frequency.  Errors: EDDY_ERR_ARG,
 * EDDY_ERR_SINGULAR_BLOCK (reported after synchronising). */
eddy_status eddy_op_assemble(eddy_op* op, const double* nu, const double* sigma, double omega,
                             eddy_stream stream);
/* b[ndof] (dev) = [int J . w_e ; 0] for a current constant per tetrahedron,
 * J_dev[nt*3] (dev, A/m^2): the source term of Eq. 5 (Section 3, right-hand side). */
eddy_status eddy_rhs_from_current(const eddy_op* op, const double* J_dev, eddy_c128* b_dev,
                                  eddy_stream stream);

/* ---- solve -------------------------------------------------------------
 * Right-preconditioned restarted GMRES(m) with classical Gram-Schmidt and
 * selective reorthogonalisation (a second pass whenever the first loses more
 * than 1 - 1/sqrt(2) of the norm), block-Jacobi preconditioning, on the equilibrated
 * system; x0 = 0.  When delta_V = 0 and the source is divergence-free
 * (||G^T b_A|| <= 1e-10 ||b||, as Section 2 requires of the excitation), the
 * gauged solution has W^T A = 0, so GMRES iterates on the operator without
 * the penalty term (its kernel {(G psi, -i omega psi|_c)} is harmless for
 * such sources) with the gauged blocks as preconditioner, and the Coulomb
 * gauge of Eq. 3 is then restored by the projection A -= G psi,
 * V += i omega psi|_c, (W^T G) psi = W^T A (nodal Jacobi-CG).  Otherwise it
 * iterates on the gauged operator.  Either way `relres` is the gauged
 * system's true weighted residual at the returned x.  b_dev[ndof] and x_dev[ndof] are device buffers (may not
 * alias).  On return x holds [A ; V] with the mass-weighted mean of V removed
 * per conductor component (Section 4).  ws: device workspace of at least
 * eddy_solve_workspace_bytes.  rep (host) may be NULL. */
eddy_status eddy_solve_workspace_bytes(const eddy_op* op, const eddy_solve_opts* opts, size_t* bytes);
eddy_status eddy_solve(eddy_op* op, const eddy_c128* b_dev, eddy_c128* x_dev, const eddy_solve_opts* opts,
                       void* ws, size_t ws_bytes, eddy_solve_report* rep, eddy_stream stream);

/* Batched solve: nrhs systems with the same operator, e.g. the probe
 * positions of a scan (Section 3: one triangulation holds every probe
 * position, only the right-hand side changes; Section 4: positions are
 * independent).  Each system runs its own GMRES (same algorithm, options and
 * result as eddy_solve); the SpMV and block-Jacobi launches serve every
 * active system at once, reading the matrix and block inverses once per
 * pass of up to 8 systems.  b_dev[nrhs][ndof], x_dev[nrhs][ndof] (device,
 * no aliasing); rep[nrhs] (host) may be NULL.  Requires delta_V = 0 and
 * divergence-free sources (EDDY_ERR_ARG otherwise).  ws: device workspace of
 * at least eddy_solve_batched_workspace_bytes. */
eddy_status eddy_solve_batched_workspace_bytes(const eddy_op* op, int32_t nrhs, const eddy_solve_opts* opts,
                                               size_t* bytes);
eddy_status eddy_solve_batched(eddy_op* op, int32_t nrhs, const eddy_c128* b_dev, eddy_c128* x_dev,
                               const eddy_solve_opts* opts, void* ws, size_t ws_bytes, eddy_solve_report* rep,
                               eddy_stream stream);
/* eddy_solve_multifreq: the batched solve for systems of different
 * frequencies (Section 4: probe positions times frequencies of one scan).
 * ops[nops]: operators of one mesh, block size and material set assembled
 * at different omega; system r (right-hand side r of b_dev [nrhs][ndof],
 * solution r of x_dev) belongs to ops[op_of_rhs[r]] (host, nondecreasing).
 * On the penalty-free operator every entry is P + c(omega) Q with P, Q real
 * (c = -i omega on A-A entries, i / omega on V-V entries, 0 on the
 * couplings), so the inner SpMV reads one frequency-factored copy of the
 * matrix (built from ops[0] in the workspace) for all systems, each scaled
 * by its own operator's equilibration; block inverses, the FP64 true
 * residual and the post-processing are each system's own operator's.
 * Requirements as eddy_solve_batched, plus: precision >= 1 and no
 * impedance-boundary faces when more than one operator is used (1/Z scales
 * with sqrt(omega)).  Workspace: eddy_solve_multifreq_workspace_bytes.
 * Errors: EDDY_ERR_ARG (mismatched operators, unordered op_of_rhs, the
 * requirements), EDDY_ERR_WORKSPACE, as eddy_solve_batched otherwise. */
eddy_status eddy_solve_multifreq_workspace_bytes(eddy_op* const* ops, int32_t nops, int32_t nrhs,
                                                 const eddy_solve_opts* opts, size_t* bytes);
eddy_status eddy_solve_multifreq(eddy_op* const* ops, int32_t nops, int32_t nrhs, const int32_t* op_of_rhs,
                                 const eddy_c128* b_dev, eddy_c128* x_dev, const eddy_solve_opts* opts,
                                 void* ws, size_t ws_bytes, eddy_solve_report* rep, eddy_stream stream);

/* ---- outputs -----------------------------------------------------------
 * Coil impedance Z[k*nsrc + l] (host) = -(i omega / (I_k I_l)) b_l^T A_k for
 * solutions x_dev[k*ndof ...] (k < nsol) and right-hand sides b_dev[l*ndof
 * ...] (l < nsrc); currents[nsrc] (host, A).  Unconjugated product: the
 * coils lie in the insulator, where E = i omega A (Eq. 2). */
eddy_status eddy_impedance(const eddy_op* op, int32_t nsol, const eddy_c128* x_dev, int32_t nsrc,
                           const eddy_c128* b_dev, const double* currents, eddy_c128* Z_host,
                           eddy_stream stream);
/* E_dev[ne] = i omega A_e + (V_hi - V_lo on edges of conducting tetrahedra):
 * the edge degrees of freedom of E = i omega A + grad V (Eq. 2). */
eddy_status eddy_edge_field(const eddy_op* op, const eddy_c128* x_dev, eddy_c128* E_dev, eddy_stream stream);

/* Impedance change caused by a defect, as a volume integral over the defect
 * region (Section 2, Eq. 12, with the vacuum taken as sigma = 0): for two
 * operators assembled on the same geometry (xyz, tet, region; checked through
 * a hash taken at eddy_mesh_create, else EDDY_ERR_MESH) and the same omega,
 * `op_defect` with the defect's (nu, sigma) and `op_free` without it,
 *   dZ[k*nl + l] = (1 / (I_k I_l)) * sum over tetrahedra where (nu, sigma)
 *     differ of [ i omega dnu int curl A_k . curl A0_l - dsig int E_k . E0_l ],
 * dnu, dsig = defect minus free values, E = i omega A + grad V (Eq. 2),
 * x_defect[nk][ndof(op_defect)] the defect solutions, x_free[nl][ndof(op_free)]
 * the defect-free ones (device, complex128), currents_k[nk], currents_l[nl]
 * (host, A), dZ[nk][nl] host.  V of x_free is taken as 0 at nodes that are not
 * conductor nodes of op_free.  For Galerkin solutions of the two systems this
 * equals Z_defect - Z_free of eddy_impedance exactly (up to solver tolerance),
 * without the cancellation of subtracting two nearly equal impedances.
 * Synchronises `stream`. */
eddy_status eddy_delta_z_volume(const eddy_op* op_defect, int32_t nk, const eddy_c128* x_defect,
                                const eddy_op* op_free, int32_t nl, const eddy_c128* x_free,
                                const double* currents_k, const double* currents_l, eddy_c128* dZ_host,
                                eddy_stream stream);

/* Eddy-current testing signals (Section 2, Eq. 11) for npos probe positions:
 * dZ = Z_defect - Z_free (the impedance change the defect causes), then
 * Z_FA = (i/2)(dZ11 + dZ12) (absolute mode) and Z_F3 = (i/2)(dZ11 - dZ22)
 * (differential mode).  Z_defect, Z_free, dZ: [npos][2][2] row-major
 * (Z[p*4 + k*2 + l] = Z_kl, coil k measuring the field of coil l); Z_FA and
 * Z_F3: [npos].  All host arrays; dZ may be NULL.  Z_free = NULL: Z_defect
 * already holds dZ (e.g. from eddy_delta_z_volume). */
eddy_status eddy_ect_signals(int32_t npos, const eddy_c128* Z_defect, const eddy_c128* Z_free, eddy_c128* dZ,
                             eddy_c128* Z_FA, eddy_c128* Z_F3);

/* ---- learned coarse correction --------------------------------------------
 * A graph network on EDDY_GNN_SUBDOMAINS subdomains (the block-Jacobi blocks
 * in bisection order, grouped into that many runs of equal block count; two
 * subdomains are adjacent if a tetrahedron holds DOFs of both, i.e. the
 * structural pattern of M couples them) predicts one complex
 * coefficient c_p per subdomain; the preconditioned vector z = B r (B the
 * block-Jacobi apply, equilibrated system) becomes z + sum_p c_p Z_p, Z_p = z
 * on subdomain p.  Features per subdomain (EDDY_GNN_FEATURES floats, 8
 * used): ||r_p|| / ||r|| sqrt(P), ||z_p|| / ||z|| sqrt(P), Re and Im of
 * <z_p, r_p> / (||z_p|| ||r_p||), conductor-DOF fraction, log10(omega) / 6,
 * log10(1 + sigma_p / 1e4) / 3 (sigma_p: subdomain mean over its DOFs of the
 * largest conductivity of a tetrahedron containing the DOF), 1.  Network
 * (float32 parameters, EDDY_GNN_PARAMS, order W0 [16x64], b0, W1 [64x64], b1,
 * W2 [64x64], b2, W3 [64x16], b3 [16], row-major): T0 = X W0,
 * H1 = relu(A T0 + b0), H_{l+1} = relu(A (H_l W_l) + b_l) + H_l (l = 1, 2),
 * Y = A (H3 W3) + b3, c_p = Y_p0 + i Y_p1, A = D^-1/2 (adj + I) D^-1/2.
 * Every GEMM operand is rounded to bfloat16 (MFMA, float32 accumulation).
 * Training pair (r, e) with M e = r: c*_p = <Z_p, e - z> / ||Z_p||^2 minimises
 * ||e - z'|| and loss = sum_p w_p |c_p - c*_p|^2, w_p = ||Z_p||^2 / ||e||^2,
 * is the error energy the correction leaves above that minimum. */
#define EDDY_GNN_SUBDOMAINS 64
#define EDDY_GNN_FEATURES 16
#define EDDY_GNN_OUTPUTS 16
#define EDDY_GNN_PARAMS 10448

/* Host: subdomain of every DOF (sub_of_dof[ndof]) and the 0/1 adjacency
 * [P*P] for blocks of block_size DOFs.  Either pointer may be NULL. */
eddy_status eddy_mesh_subdomains(const eddy_mesh* mesh, int32_t block_size, int32_t* sub_of_dof,
                                 int32_t* adjacency);
/* Host copy of the feature columns 4..7 [P*4] set at the last assembly. */
eddy_status eddy_gnn_static_features(const eddy_op* op, float* static4);
/* Device scratch (256-byte aligned) of eddy_gnn_forward / eddy_gnn_train_step for nsamp samples. */
eddy_status eddy_gnn_scratch_bytes(int32_t nsamp, size_t* bytes);
/* Features X [P*16] and, if xstar != NULL, targets cstar [P*2] (re, im) and
 * weights w [P] (all float32, device) of the pair r = b - M x, e = x* - x of
 * the physical system (b, x, xstar: device complex128 [ndof]); the network
 * sees them in the equilibrated variables, where B acts.  Uses the
 * operator's temporaries (not concurrently with another call on it). */
eddy_status eddy_gnn_pair(const eddy_op* op, const eddy_c128* b, const eddy_c128* x, const eddy_c128* xstar,
                          float* X, float* cstar, float* w, eddy_stream stream);
/* Y [nsamp][P*16] = network(theta; X [nsamp][P*16]) (device float32). */
eddy_status eddy_gnn_forward(const eddy_op* op, int32_t nsamp, const float* theta, const float* X, float* Y,
                             void* scratch, size_t scratch_bytes, eddy_stream stream);
/* One training step on a batch (device arrays): per-sample loss [nsamp],
 * the batch-mean gradient grad_mean [EDDY_GNN_PARAMS] (may be NULL), then
 * Adam (beta 0.9, 0.999, eps 1e-8, step >= 1 counting from 1) on theta, m, v
 * unless lr == 0. */
eddy_status eddy_gnn_train_step(const eddy_op* op, int32_t nsamp, float* theta, float* m, float* v, const float* X,
                                const float* cstar, const float* w, int32_t step, float lr, float* loss,
                                float* grad_mean, void* scratch, size_t scratch_bytes, eddy_stream stream);

/* ---- building blocks (parity tests and benchmarks) ---------------------
 * y = M x with the gauge applied in factored form (unscaled system). */
eddy_status eddy_spmv(const eddy_op* op, const eddy_c128* x_dev, eddy_c128* y_dev, eddy_stream stream);
/* z = blockdiag(M)^-1 r over the block-Jacobi blocks (unscaled system). */
eddy_status eddy_precond_apply(const eddy_op* op, const eddy_c128* r_dev, eddy_c128* z_dev, eddy_stream stream);
/* Host copies of the stored (equilibrated) arrays: rowptr[ndof+1], col[nnz],
 * val[nnz] = s_i M_ij s_j (gauge excluded), wval[nnz_w] = s_e W_en in the
 * CSR order of W (rows = edges, columns = nodes, ascending), wrowptr[ne+1],
 * wcol[nnz_w], d0[nv], s[ndof].  Any pointer may be NULL to skip it. */
eddy_status eddy_export(const eddy_op* op, int32_t* rowptr, int32_t* col, eddy_c128* val,
                        int32_t* wrowptr, int32_t* wcol, double* wval, double* d0, double* s,
                        eddy_stream stream);

/* Per-kernel-class timing of the GMRES loop, measured with HIP events on the
 * solve's stream and read at the loop's periodic synchronisation.  The
 * events bracket one Arnoldi step in eight (a different step of each group
 * of eight), so the counts are about an eighth of the iterations.
 * Classes: 0 block-Jacobi apply, 1 gauge product W~^T x, 2 SpMV
 * (+ W~ t), 3 CGS2 orthogonalisation + normalisation.  Returns (host) the
 * accumulated milliseconds ms[4] and launch counts counts[4] since the
 * previous call (either may be NULL), resets them, and turns timing on
 * (enable != 0) or off.  Creating the events is the only allocation. */
eddy_status eddy_profile(eddy_op* op, int32_t enable, double* ms, int64_t* counts);
/* The SpMV grid caps chosen at the first eddy_op_assemble (an autotuner: each
 * candidate cap is timed with HIP events on the operator's own sliced-ELL
 * matrix; the cap changes no result, only which workgroup runs a slice). */
eddy_status eddy_op_tuning(const eddy_op* op, eddy_tuning* out);

const char* eddy_status_string(eddy_status status);
const char* eddy_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* EDDY_H */
