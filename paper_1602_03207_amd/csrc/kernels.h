// Launch wrappers for the HIP kernels (kernels.hip).  All complex vectors are
// double2 (re, im); all launches are asynchronous on `st`.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace eddy {

constexpr int kRedBlocks = 2048;      // blocks of the two-stage reductions

// ---- assembly (Section 2, Eqs. 5-7; Section 3 global blocks)
void launch_element(int64_t nt, int64_t nct, const double* xyz, const int* tet, const int* region,
                    const uint8_t* signbits, const int* cidx, const double* nu_reg, const double* sig_reg,
                    double omega, double delta_v, double2* ebuf, double* wbuf, double* vol4, hipStream_t st);
void launch_gather_c(int64_t n, const int* ptr, const int* list, const double2* buf, double2* out, hipStream_t st);
void launch_gather_r(int64_t n, const int* ptr, const int* list, const double* buf, double* out, hipStream_t st);
void launch_gather_r2c(int64_t n, int64_t ntot, const int* ptr, const int* list, const double* buf, double2* out,
                       hipStream_t st);
void launch_permute_r(int64_t n, const int* perm, const double* in, double* out, hipStream_t st);
void launch_d0tau(int64_t nv, const double* d0, double tau, double* d0tau, hipStream_t st);
void launch_equilibrate(int64_t n, int64_t ne, const int* diagpos, const double2* val, const int* wrowptr,
                        const int* wcol, const double* wval, const double* d0tau, double* s, int* status,
                        hipStream_t st);
void launch_scale_rows(int64_t n, const int* rowptr, const int* col, double2* val, const double* s, hipStream_t st);
void launch_scale_w(int64_t ne, const int* wrowptr, double* wval, const double* s, hipStream_t st);
// block inverses: gauge blocks into gscr (nb * 64 * 64 doubles), then LDS Gauss-Jordan
void launch_block_invert(int64_t nb, const int* blk_ptr, const int* blk_dofs, const int* blk_of, const int* loc_of,
                         const int* rowptr, const int* col, const double2* val, int64_t ne, const int* wrowptr,
                         const int* wcol, const double* wval, const double* d0tau, double* gscr, double2* minv,
                         int* status, hipStream_t st);
void launch_rhs_elem(int64_t nt, const double* xyz, const int* tet, const uint8_t* signbits, const double* J,
                     double* rbuf, hipStream_t st);

// ---- solve
void launch_wt(int64_t nv, const int* wtrowptr, const int* wtcol, const double* wtval, const double* d0tau,
               const double2* x, double2* t, hipStream_t st);
// y = M~ x + W~ t  (A rows, if wrowptr); if b != nullptr: y = b - (...).
// M~ in the sliced ELL layout (ns slices); T = double2 (complex128) or float2
// (complex64) storage and arithmetic.  grid > 0 caps the number of
// workgroups; schedule 0 sweeps the slices with all XCDs together, 1 gives
// each XCD a contiguous range of groups of 4 slices, xcd_groups[9] (device)
// the range boundaries.  Neither changes the result.
template <class T>
void launch_spmv(int64_t ns, const int* sptr, const int* srow, const int* scol, const T* sval, int64_t ne,
                 const int* wrowptr, const int* wcol, const double* wval, const double2* t, const T* x,
                 const double2* b, T* y, hipStream_t st, int grid = 0, int schedule = 0,
                 const int* xcd_groups = nullptr, const int* scplx = nullptr);
// workgroups of an uncapped SpMV launch over ns slices
int spmv_full_grid(int64_t ns);
void launch_sell_gather(int64_t tot, int64_t ns, const int* sptr, const int* src, const double2* val, double2* sval,
                        float2* sval32, int* scplx, hipStream_t st);
// MT: storage of the inverses, T or (with T = float2) packed complex half
// (uint32_t); RT: storage of r (T, or hbasis with T = float2)
template <class T, class MT, class RT>
void launch_block_apply(int64_t nb, const int* blk_ptr, const int* blk_dofs, const MT* minv, const RT* r, T* z,
                        hipStream_t st);
// complex128 -> packed complex half (round to nearest even)
void launch_to_c16(int64_t n, const double2* in, uint32_t* out, hipStream_t st);
// Krylov primitives: storage T, all reductions and Hessenberg entries in FP64
// partial dots V^H w (+ ||w||^2 in slot q if want_norm); flag (device, may be
// null) = 0 skips the launch
template <class T>
void launch_mdot(int64_t n, const T* V, int64_t ldv, int q, const T* w, double2* partial, hipStream_t st,
                 int want_norm = 0, const int* flag = nullptr);
// number of per-block partials launch_mdot writes per vector for length n
int mdot_parts(int64_t n);
void launch_reduce_cols(int q, int nparts, const double2* partial, double2* out, hipStream_t st,
                        const int* flag = nullptr);
template <class T>
void launch_norm2(int64_t n, const T* w, double* partial, double* out_norm, hipStream_t st);
template <class Ti, class To>
void launch_scale_by_inv(int64_t n, const Ti* w, const double* norm, To* v, hipStream_t st);
template <class Ti, class To>
void launch_scale_host(int64_t n, const Ti* w, double a, To* v, hipStream_t st);
template <class VT, class T>
void launch_combine(int64_t n, const VT* V, int64_t ldv, int q, const double2* y, T* u, hipStream_t st);
template <class T>
void launch_axpy(int64_t n, const T* z, double2* x, hipStream_t st);
void launch_to_c64(int64_t n, const double2* in, float2* out, hipStream_t st);
// ---- batched systems (vectors of system r at offset r * stride; grid.z = r;
// `active` (device int[nrhs], may be null) masks systems out)
template <class T, class MT, class RT>
void launch_block_apply_b(int64_t nb, const int* blk_ptr, const int* blk_dofs, const MT* minv, int nrhs,
                          int64_t rstride, const RT* r, int64_t zstride, T* z, const int* active, hipStream_t st);
// the same for complex-half inverses and inputs on the matrix cores (f16
// MFMA, float32 sums); every inverse column past the block size must be zero
// (interleave: z per chunk of 8 systems as [row][8], the input of launch_spmv_b_il)
void launch_block_apply_mfma(int64_t nb, const int* blk_ptr, const int* blk_dofs, const uint32_t* minv, int nrhs,
                             int64_t rstride, const hbasis* r, int64_t zstride, float2* z, const int* active,
                             int interleave, hipStream_t st);
// complex64 batched SpMV with an interleaved input (xil[((c0/8) ld + row) 8 + q])
void launch_spmv_b_il(int64_t n, const int* rowptr, const int* col, const float2* val, int nrhs, int64_t ld,
                      const float2* xil, float2* y, const int* active, hipStream_t st);
template <class T>
void launch_spmv_b(int64_t n, const int* rowptr, const int* col, const T* val, int nrhs, int64_t ld, const T* x,
                   const T* b, T* y, const int* active, hipStream_t st);
void launch_reduce_cols_b(int q, int nparts, const double2* partial, int64_t pstride, double2* out, int64_t ostride,
                          const int* flag, const int* active, int nrhs, hipStream_t st);
template <class T>
void launch_norm2_b(int64_t n, const T* w, int64_t wstride, double* partial, double* out_norm, const int* active,
                    int nrhs, hipStream_t st);
template <class Ti, class To>
void launch_scale_by_inv_b(int64_t n, const Ti* w, int64_t wstride, const double* norm, To* v, int64_t vstride,
                           const int* active, int nrhs, hipStream_t st);
void launch_givens_b(int j, int m, const double2* h1, const double2* h2, int64_t hstride, int64_t h2stride,
                     const double* nrm, double2* H, double* cs, double2* sn, double2* g, const double* beta,
                     const double* bnorm, double* est, const int* active, int nrhs, hipStream_t st);
void launch_backsolve_b(const int* ks, int m, const double2* H, const double2* g, double2* y, int64_t ystride,
                        const int* active, int nrhs, hipStream_t st);
template <class VT, class T>
void launch_combine_b(int64_t n, const VT* V, int64_t ldv, int64_t vstride, const int* qs, const double2* y,
                      int64_t ystride, T* u, int64_t ustride, const int* active, int nrhs, hipStream_t st);
template <class T>
void launch_axpy_b(int64_t n, const T* z, int64_t zstride, double2* x, int64_t xstride, const int* active, int nrhs,
                   hipStream_t st);
void launch_diag_scale_b(int64_t n, const double2* in, int64_t istride, const double* s, int divide, double2* out,
                         int64_t ostride, int nrhs, hipStream_t st);
template <class T>
void launch_to_storage_b(int64_t n, const double2* in, int64_t istride, T* out, int64_t ostride, int nrhs,
                         hipStream_t st);
// Arnoldi by CGS2 with delayed reorthogonalisation (DCGS2): fused dots
// [V^H v, V^H w, v^H v, v^H w] (2q + 2 partial columns of mdot2_parts(n)),
// the step's small linear algebra + lagged Givens rotation, and the fused
// update (finished basis vector into v, next direction into w, ||w||).
int mdot2_parts(int64_t n);
// VT: storage of the basis V and the pending vector v (T, or hbasis with T = float2)
template <class VT, class T>
void launch_mdot2(int64_t n, const VT* V, int64_t ldv, int q, const VT* v, const T* w, double2* partial,
                  hipStream_t st);
// Sall [m x m] / rhoall [m] (may be null) record each step's finishing
// transform (s, rho) for flexible cycles; launch_flex_coeffs then maps the
// least-squares coefficients on the finished preconditioned columns to the
// stored ones.
void launch_dcgs_coef(int j, int m, const double2* dots, double2* Hraw, const double* tnorm, double2* coef,
                      double2* H, double* cs, double2* sn, double2* g, double beta, double bnorm, double* est,
                      double2* Sall, double* rhoall, hipStream_t st);
void launch_flex_coeffs(int k, int m, const double2* Sall, const double* rhoall, double2* y, hipStream_t st);
// the same with beta and ||b|| read from device memory (a captured step
// stays valid across cycles), and the two-value store that sets them
void launch_dcgs_coef_dev(int j, int m, const double2* dots, double2* Hraw, const double* tnorm, double2* coef,
                          double2* H, double* cs, double2* sn, double2* g, const double* beta, const double* bnorm,
                          double* est, double2* Sall, double* rhoall, hipStream_t st);
void launch_set2(double a, double b, double* out, hipStream_t st);
// batched forms (system z: V at z * vstride, w at z * wstride, partial at
// z * pstride, dots and coef at z * dstride, Hessenberg data at the strides
// of launch_givens_b; beta, bnorm, tnorm per system; active masks systems)
template <class VT, class T>
void launch_mdot2_b(int64_t n, const VT* V, int64_t ldv, int64_t vstride, int q, const VT* v, const T* w,
                    int64_t wstride, double2* partial, int64_t pstride, const int* active, int nrhs, hipStream_t st);
void launch_dcgs_coef_b(int j, int m, const double2* dots, int64_t dstride, double2* Hraw, const double* tnorm,
                        double2* coef, double2* H, double* cs, double2* sn, double2* g, const double* beta,
                        const double* bnorm, double* est, const int* active, int nrhs, hipStream_t st);
template <class VT, class T>
void launch_dcgs_update_b(int64_t n, const VT* V, int64_t ldv, int64_t vstride, int q, const double2* coef,
                          int64_t cstride, VT* v, T* w, int64_t wstride, double* rpart, double* out_norm,
                          const int* active, int nrhs, hipStream_t st);
// out_norm may be null: the norm is then left in rpart's kRedBlocks partial
// sums for launch_scale_by_partials
template <class VT, class T>
void launch_dcgs_update(int64_t n, const VT* V, int64_t ldv, int q, const double2* coef, VT* v, T* w, double* rpart,
                        double* out_norm, hipStream_t st);
// v = w / ||w|| from the partial sums of ||w||^2; ||w|| into out_norm
template <class Ti, class To>
void launch_scale_by_partials(int64_t n, const Ti* w, const double* rpart, double* out_norm, To* v, hipStream_t st);
// Hessenberg least squares on the device
void launch_givens(int j, int m, const double2* h1, const double2* h2, const double* nrm, double2* H, double* cs,
                   double2* sn, double2* g, double beta, double bnorm, double* est, hipStream_t st);
void launch_backsolve(int k, int m, const double2* H, const double2* g, double2* y, hipStream_t st);
// several frequencies in one batch (see k_spmv_mf): per system the
// equilibration of its operator and Im c on the A rows (-omega) and V rows
// (1/omega)
struct mf_sys {
  const double* s;
  float w_a, w_v;
};
void launch_factor_pq(int64_t n, int64_t ne, const int* rowptr, const int* col, const double2* val, const double* s,
                      double omega, float2* pq, hipStream_t st);
// y_r = s_r (P + c_r Q)(s_r x_r); u is scratch of the shape of x
void launch_spmv_mf(int64_t n, int64_t ne, const int* rowptr, const int* col, const float2* pq, int nrhs, int64_t ld,
                    const float2* x, float2* u, float2* y, const mf_sys* sys, const int* active, hipStream_t st);
// impedance-boundary triangles: surface-conductor values into fbuf (21 nf
// slots, see k_face) and |T|/3 into area3
void launch_face(int64_t nf, const double* xyz, const int* face, const int* face_region, const double* nu_reg,
                 const double* sig_reg, double omega, double2* fbuf, double* area3, hipStream_t st);
void launch_diag_scale(int64_t n, const double2* in, const double* s, int divide, double2* out, hipStream_t st);
void launch_zero(int64_t n, double2* x, hipStream_t st);
void launch_vmean(int64_t nc, int ncomp, const int* comp, const double* lumped, double2* V, double2* scratch,
                  hipStream_t st);
void launch_udot(int64_t n, const double2* a, const double2* b, double2* partial, double2* out, hipStream_t st);
// Coulomb projection helpers (Poisson solve on W^T G by Jacobi-CG, then the shift)
void launch_edge_divergence(int64_t nv, const int* wtrowptr, const int* wtcol, const int* edges, const double2* b,
                            double2* d, hipStream_t st);
void launch_lap_diag(int64_t nv, const int* wtrowptr, const int* wtcol, const double* wtval, const int* edges,
                     const double* s, double* diag, hipStream_t st);
// L = W^T G assembled per node row; fused CG pieces: q = L p with p^H q (into
// pq), and the update psi, r, z = r / diag with r^H z (into rz_new);
// partial: kRedBlocks double2
void launch_lap_assemble(int64_t nv, const int* wtrowptr, const int* wtcol, const double* wtval, const int* edges,
                         const double* s, const int* lrowptr, const int* lcol, double* lval, hipStream_t st);
// projection CG: partial sums in kRedBlocks slots, summed by the consumer
void launch_lap_spmv_dot(int64_t nv, const int* lrowptr, const int* lcol, const double* lval, const double2* p,
                         double2* q, double2* partial, hipStream_t st);
void launch_cg_update(int64_t n, const double2* rz, const double2* pq_part, const double2* p, const double2* q,
                      const double* diag, double2* psi, double2* r, double2* z, double2* partial, hipStream_t st);
void launch_jacobi(int64_t n, const double2* r, const double* diag, double2* z, hipStream_t st);
void launch_cg_dir(int64_t n, const double2* rz_part, const double2* rz_old, double2* rz_new, const double2* z,
                   double2* p, hipStream_t st);
void launch_project(int64_t ne, int64_t nc, const int* edges, const int* cond_nodes, const double2* psi, double omega,
                    double2* x, hipStream_t st);
// Defect-region volume form of the impedance change for one defect-configuration
// solution xd against nl <= kMaxDzCols free-configuration solutions (x0 + l*ld0);
// out[l] = sum over tetrahedra of i w dnu |K| curl A_d . curl A_0 - dsig int E_d . E_0.
void launch_dz_volume(int64_t nt, const double* xyz, const int* tet, const int* region, const uint8_t* signbits,
                      const int* tet2edge, const double* nu_d, const double* sig_d, const double* nu_0,
                      const double* sig_0, double omega, int64_t ne, const double2* xd, const int* vmap_d, int nl,
                      const double2* x0, int64_t ld0, const int* vmap_0, double2* partial, double2* out,
                      hipStream_t st);
void launch_edge_field(int64_t ne, const int* edge_v, const double2* x, double omega, double2* E, hipStream_t st);

}  // namespace eddy
