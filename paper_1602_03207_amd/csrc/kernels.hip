// HIP kernels of the A-V eddy-current solver, written for gfx950 (CDNA4,
// 64-wide wavefronts).  Every reduction runs in a fixed order, so results are
// bitwise reproducible run to run; assembly uses no atomics.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "kernels.h"

namespace eddy {
namespace {

#include "devmath.h"


// ---------------------------------------------------------------------------
// Element kernel: one thread per tetrahedron.  grad(l_1..3) are the columns
// of E^-1 (E has rows p_i - p_0), obtained from cross products of the rows;
// grad(l_0) = -sum.  For local edges l = (a, b), m = (c, d):
//   K_lm = |K| curl w_l . curl w_m,      curl w_l = 2 grad l_a x grad l_b
//   M_lm = |K|/20 [(1+d_ac) G_bd - (1+d_ad) G_bc - (1+d_bc) G_ad + (1+d_bd) G_ac]
//   W_lk = |K|/4 (grad l_b - grad l_a) . grad l_k
//   S_ij = |K| G_ij,  N_ij = |K| (1 + d_ij) / 20,   G_ij = grad l_i . grad l_j
// Stored (global orientation signs s applied):
//   AA = s_l s_m (nu K_lm - i omega sigma M_lm)        (M11 without gauge)
//   AV = -sigma W_lk                                    (M12 = -B_sigma)
//   VV = delta_V sigma N_ij + i sigma S_ij / omega      (M22)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_element(int64_t nt, int64_t nct, const double* __restrict__ xyz,
                                                      const int* __restrict__ tet, const int* __restrict__ region,
                                                      const uint8_t* __restrict__ signbits,
                                                      const int* __restrict__ cidx, const double* __restrict__ nu_reg,
                                                      const double* __restrict__ sig_reg, double omega, double delta_v,
                                                      double2* __restrict__ ebuf, double* __restrict__ wbuf,
                                                      double* __restrict__ vol4) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nt) return;
  const int4 nd = reinterpret_cast<const int4*>(tet)[t];
  const int n[4] = {nd.x, nd.y, nd.z, nd.w};
  double p[4][3];
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int j = 0; j < 3; ++j) p[k][j] = xyz[3 * (int64_t)n[k] + j];
  double e1[3], e2[3], e3[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    e1[j] = p[1][j] - p[0][j];
    e2[j] = p[2][j] - p[0][j];
    e3[j] = p[3][j] - p[0][j];
  }
  double c23[3] = {e2[1] * e3[2] - e2[2] * e3[1], e2[2] * e3[0] - e2[0] * e3[2], e2[0] * e3[1] - e2[1] * e3[0]};
  double c31[3] = {e3[1] * e1[2] - e3[2] * e1[1], e3[2] * e1[0] - e3[0] * e1[2], e3[0] * e1[1] - e3[1] * e1[0]};
  double c12[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
  const double det = e1[0] * c23[0] + e1[1] * c23[1] + e1[2] * c23[2];
  const double id = 1.0 / det;
  const double vol = fabs(det) * (1.0 / 6.0);
  double g[4][3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    g[1][j] = c23[j] * id;
    g[2][j] = c31[j] * id;
    g[3][j] = c12[j] * id;
    g[0][j] = -(g[1][j] + g[2][j] + g[3][j]);
  }
  double G[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int k = 0; k < 4; ++k) G[i][k] = g[i][0] * g[k][0] + g[i][1] * g[k][1] + g[i][2] * g[k][2];
  constexpr int ea[6] = {0, 0, 0, 1, 1, 2};
  constexpr int eb[6] = {1, 2, 3, 2, 3, 3};
  const uint8_t sb = signbits[t];
  double sg[6], cu[6][3];
#pragma unroll
  for (int l = 0; l < 6; ++l) {
    sg[l] = ((sb >> l) & 1) ? -1.0 : 1.0;
    const double* a = g[ea[l]];
    const double* b = g[eb[l]];
    cu[l][0] = 2.0 * (a[1] * b[2] - a[2] * b[1]);
    cu[l][1] = 2.0 * (a[2] * b[0] - a[0] * b[2]);
    cu[l][2] = 2.0 * (a[0] * b[1] - a[1] * b[0]);
  }
  const int reg = region[t];
  const double nu = nu_reg[reg], sig = sig_reg[reg];
  const double v20 = vol * (1.0 / 20.0);
  int slot = 0;
#pragma unroll
  for (int l = 0; l < 6; ++l) {
#pragma unroll
    for (int m = l; m < 6; ++m) {
      const int a = ea[l], b = eb[l], c = ea[m], d = eb[m];
      const double K = vol * (cu[l][0] * cu[m][0] + cu[l][1] * cu[m][1] + cu[l][2] * cu[m][2]);
      const double M = v20 * ((a == c ? 2.0 : 1.0) * G[b][d] - (a == d ? 2.0 : 1.0) * G[b][c] -
                              (b == c ? 2.0 : 1.0) * G[a][d] + (b == d ? 2.0 : 1.0) * G[a][c]);
      const double ss = sg[l] * sg[m];
      ebuf[(int64_t)slot * nt + t] = make_double2(ss * nu * K, -ss * omega * sig * M);
      ++slot;
    }
  }
  double Wl[6][4];
  const double v4 = vol * 0.25;
#pragma unroll
  for (int l = 0; l < 6; ++l)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      Wl[l][k] = sg[l] * v4 * (G[eb[l]][k] - G[ea[l]][k]);
      wbuf[(int64_t)(l * 4 + k) * nt + t] = Wl[l][k];
    }
  vol4[t] = v4;
  const int c = cidx[t];
  if (c >= 0) {
    const int64_t av0 = 21 * nt, vv0 = 21 * nt + 24 * nct;
#pragma unroll
    for (int l = 0; l < 6; ++l)
#pragma unroll
      for (int k = 0; k < 4; ++k) ebuf[av0 + (int64_t)(l * 4 + k) * nct + c] = make_double2(-sig * Wl[l][k], 0.0);
    int q = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = i; j < 4; ++j) {
        const double N = v20 * (i == j ? 2.0 : 1.0);
        ebuf[vv0 + (int64_t)q * nct + c] = make_double2(delta_v * sig * N, sig * vol * G[i][j] / omega);
        ++q;
      }
  }
}

// ---------------------------------------------------------------------------
// Impedance-boundary triangles (Section 2, Eqs. 8-10).  The plate removed
// from the mesh enters as a surface conductor on its boundary Gamma_p with
// the coefficient c = 1/Z = delta sigma / (1 - i), delta = sqrt(2 nu /
// (omega sigma)) its skin depth, i.e. the volume terms with sigma dV
// replaced by c dS:
//   AA = -i omega c M_lm,   AV = -c B_lk,   VV = (i / omega) c S_ij,
//   M_lm = |T|/12 [(1+d_ac) G_bd - (1+d_ad) G_bc - (1+d_bc) G_ad + (1+d_bd) G_ac],
//   B_lk = |T|/3 (G_bk - G_ak),  S_ij = |T| G_ij,  G_ij = grad l_i . grad l_j,
// with the surface gradients grad l_i = n x (p_(i+2) - p_(i+1)) / (2|T|) and
// local edges (0,1), (0,2), (1,2) running from the lower to the higher node
// id (the nodes of a face are stored increasing).  Slots: AA at q * nf + f
// (q the upper-triangle pair), AV at 6 nf + (l * 3 + k) * nf + f, VV at
// 15 nf + q * nf + f; area3[f] = |T|/3 (lumped V weight).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_face(int64_t nf, const double* __restrict__ xyz,
                                                   const int* __restrict__ face,
                                                   const int* __restrict__ face_region,
                                                   const double* __restrict__ nu_reg,
                                                   const double* __restrict__ sig_reg, double omega,
                                                   double2* __restrict__ fbuf, double* __restrict__ area3) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  double p[3][3];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int j = 0; j < 3; ++j) p[k][j] = xyz[3 * (int64_t)face[3 * f + k] + j];
  double e1[3], e2[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    e1[j] = p[1][j] - p[0][j];
    e2[j] = p[2][j] - p[0][j];
  }
  const double cn[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
  const double two_a = sqrt(cn[0] * cn[0] + cn[1] * cn[1] + cn[2] * cn[2]);
  const double area = 0.5 * two_a;
  const double nh[3] = {cn[0] / two_a, cn[1] / two_a, cn[2] / two_a};
  double g[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double* a = p[(i + 1) % 3];
    const double* b = p[(i + 2) % 3];
    const double d[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    g[i][0] = (nh[1] * d[2] - nh[2] * d[1]) / two_a;
    g[i][1] = (nh[2] * d[0] - nh[0] * d[2]) / two_a;
    g[i][2] = (nh[0] * d[1] - nh[1] * d[0]) / two_a;
  }
  double G[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) G[i][k] = g[i][0] * g[k][0] + g[i][1] * g[k][1] + g[i][2] * g[k][2];
  const int reg = face_region[f];
  const double sig = sig_reg[reg], nu = nu_reg[reg];
  const double delta = sqrt(2.0 * nu / (omega * sig));
  const double cr = 0.5 * delta * sig, ci = 0.5 * delta * sig;     // delta sigma / (1 - i)
  constexpr int ea[3] = {0, 0, 1};
  constexpr int eb[3] = {1, 2, 2};
  const double a12 = area * (1.0 / 12.0);
  int q = 0;
#pragma unroll
  for (int l = 0; l < 3; ++l)
#pragma unroll
    for (int m = l; m < 3; ++m) {
      const int a = ea[l], b = eb[l], c = ea[m], d = eb[m];
      const double M = a12 * ((a == c ? 2.0 : 1.0) * G[b][d] - (a == d ? 2.0 : 1.0) * G[b][c] -
                              (b == c ? 2.0 : 1.0) * G[a][d] + (b == d ? 2.0 : 1.0) * G[a][c]);
      fbuf[(int64_t)q * nf + f] = make_double2(omega * ci * M, -omega * cr * M);
      ++q;
    }
  const double a3 = area * (1.0 / 3.0);
#pragma unroll
  for (int l = 0; l < 3; ++l)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double B = a3 * (G[eb[l]][k] - G[ea[l]][k]);
      fbuf[(int64_t)(6 + l * 3 + k) * nf + f] = make_double2(-cr * B, -ci * B);
    }
  q = 0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = i; j < 3; ++j) {
      const double S = area * G[i][j];
      fbuf[(int64_t)(15 + q) * nf + f] = make_double2(-ci * S / omega, cr * S / omega);
      ++q;
    }
  area3[f] = a3;
}

// out[i] = sum of buf[list[p]] for p in [ptr[i], ptr[i+1]), in list order.
__global__ __launch_bounds__(kThreads) void k_gather_c(int64_t n, const int* __restrict__ ptr,
                                                       const int* __restrict__ list, const double2* __restrict__ buf,
                                                       double2* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double2 s = make_double2(0.0, 0.0);
  for (int p = ptr[i]; p < ptr[i + 1]; ++p) s = cadd(s, buf[list[p]]);
  out[i] = s;
}

__global__ __launch_bounds__(kThreads) void k_gather_r(int64_t n, const int* __restrict__ ptr,
                                                       const int* __restrict__ list, const double* __restrict__ buf,
                                                       double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int p = ptr[i]; p < ptr[i + 1]; ++p) s += buf[list[p]];
  out[i] = s;
}

// rows < n gather real sums into complex outputs; rows n..ntot-1 are zeroed
__global__ __launch_bounds__(kThreads) void k_gather_r2c(int64_t n, int64_t ntot, const int* __restrict__ ptr,
                                                         const int* __restrict__ list, const double* __restrict__ buf,
                                                         double2* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ntot) return;
  double s = 0.0;
  if (i < n)
    for (int p = ptr[i]; p < ptr[i + 1]; ++p) s += buf[list[p]];
  out[i] = make_double2(s, 0.0);
}

__global__ __launch_bounds__(kThreads) void k_permute_r(int64_t n, const int* __restrict__ perm,
                                                        const double* __restrict__ in, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = in[perm[i]];
}

__global__ __launch_bounds__(kThreads) void k_d0tau(int64_t nv, const double* __restrict__ d0, double tau,
                                                    double* __restrict__ d0tau) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nv) d0tau[i] = tau / d0[i];
}

// s_i = |M_ii|^-1/2 with the gauge diagonal tau sum_n W_in^2 / D0_n on A rows.
__global__ __launch_bounds__(kThreads) void k_equilibrate(int64_t n, int64_t ne, const int* __restrict__ diagpos,
                                                          const double2* __restrict__ val,
                                                          const int* __restrict__ wrowptr,
                                                          const int* __restrict__ wcol,
                                                          const double* __restrict__ wval,
                                                          const double* __restrict__ d0tau, double* __restrict__ s,
                                                          int* __restrict__ status) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double2 d = val[diagpos[i]];
  if (i < ne) {
    double gsum = 0.0;
    for (int p = wrowptr[i]; p < wrowptr[i + 1]; ++p) gsum += wval[p] * wval[p] * d0tau[wcol[p]];
    d.x += gsum;
  }
  const double a = sqrt(d.x * d.x + d.y * d.y);
  if (!(a > 0.0)) {
    atomicOr(status, 2);
    s[i] = 1.0;
  } else {
    s[i] = 1.0 / sqrt(a);
  }
}

__global__ __launch_bounds__(kThreads) void k_scale_rows(int64_t n, const int* __restrict__ rowptr,
                                                         const int* __restrict__ col, double2* __restrict__ val,
                                                         const double* __restrict__ s) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double si = s[i];
  for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) {
    const double f = si * s[col[p]];
    double2 v = val[p];
    val[p] = make_double2(v.x * f, v.y * f);
  }
}

__global__ __launch_bounds__(kThreads) void k_scale_w(int64_t ne, const int* __restrict__ wrowptr,
                                                      double* __restrict__ wval, const double* __restrict__ s) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  const double se = s[e];
  for (int p = wrowptr[e]; p < wrowptr[e + 1]; ++p) wval[p] *= se;
}

// Gauge part of one diagonal block: G(i, j) = sum over shared nodes n of
// W~_in W~_jn tau / D0_n for the A rows of the block, W~ rows staged in LDS;
// written column-major to gscr[k * 64 * 64 + j * 64 + i] (rows i < sz).
__global__ __launch_bounds__(kMaxBlock) void k_block_gauge(const int* __restrict__ blk_ptr,
                                                           const int* __restrict__ blk_dofs, int64_t ne,
                                                           const int* __restrict__ wrowptr,
                                                           const int* __restrict__ wcol,
                                                           const double* __restrict__ wval,
                                                           const double* __restrict__ d0tau,
                                                           double* __restrict__ gscr) {
  __shared__ int wn[kMaxBlock][kMaxWRow];
  __shared__ double wv[kMaxBlock][kMaxWRow];
  __shared__ double wd[kMaxBlock][kMaxWRow];
  __shared__ int wc[kMaxBlock];
  const int k = blockIdx.x;
  const int i = threadIdx.x;
  const int b0 = blk_ptr[k];
  const int sz = blk_ptr[k + 1] - b0;
  int cnt = 0;
  if (i < sz) {
    const int r = blk_dofs[b0 + i];
    if (r < ne) {
      cnt = wrowptr[r + 1] - wrowptr[r];      // <= kMaxWRow, checked on the host
      for (int q = 0; q < cnt; ++q) {
        const int nq = wcol[wrowptr[r] + q];
        wn[i][q] = nq;
        wv[i][q] = wval[wrowptr[r] + q];
        wd[i][q] = wval[wrowptr[r] + q] * d0tau[nq];
      }
    }
  }
  wc[i] = cnt;
  __syncthreads();
  if (i >= sz) return;
  double* out = gscr + (int64_t)k * kMaxBlock * kMaxBlock;
  for (int j = 0; j < sz; ++j) {
    const int cj = wc[j];
    // the node lists of W's rows are sorted and unique: a merge visits the
    // shared nodes in ascending order (the order of a double loop over q)
    double acc = 0.0;
    int q = 0, u = 0;
    while (q < cnt && u < cj) {
      const int nq = wn[i][q], nu = wn[j][u];
      if (nq == nu) acc += wd[i][q++] * wv[j][u++];
      else if (nq < nu) ++q;
      else ++u;
    }
    out[j * kMaxBlock + i] = acc;
  }
}

// ---------------------------------------------------------------------------
// Dense inverse of one equilibrated diagonal block per 64-thread workgroup:
// gather the block (CSR part + the gauge part from k_block_gauge) into LDS
// column-major, Gauss-Jordan with partial pivoting (thread i owns row i;
// thread j owns column j for row swaps), undo the column permutation, store
// column-major.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kMaxBlock) void k_block_invert(
    const int* __restrict__ blk_ptr, const int* __restrict__ blk_dofs, const int* __restrict__ blk_of,
    const int* __restrict__ loc_of, const int* __restrict__ rowptr, const int* __restrict__ col,
    const double2* __restrict__ val, const double* __restrict__ gscr, double2* __restrict__ minv,
    int* __restrict__ status) {
  __shared__ double2 A[kMaxBlock * kMaxBlock];   // A(i, j) at j * 64 + i
  __shared__ int perm[kMaxBlock];
  const int k = blockIdx.x;
  const int i = threadIdx.x;
  const int b0 = blk_ptr[k];
  const int sz = blk_ptr[k + 1] - b0;
  const double* gk = gscr + (int64_t)k * kMaxBlock * kMaxBlock;
  for (int j = 0; j < kMaxBlock; ++j)
    A[j * kMaxBlock + i] = make_double2((i < sz && j < sz) ? gk[j * kMaxBlock + i] : 0.0, 0.0);
  __syncthreads();
  if (i < sz) {
    const int r = blk_dofs[b0 + i];
    for (int p = rowptr[r]; p < rowptr[r + 1]; ++p) {
      const int c = col[p];
      if (blk_of[c] == k) {
        const double2 v = val[p];
        A[loc_of[c] * kMaxBlock + i].x += v.x;
        A[loc_of[c] * kMaxBlock + i].y += v.y;
      }
    }
  }
  __syncthreads();
  for (int kk = 0; kk < sz; ++kk) {
    // pivot: largest |A(i, kk)| over i >= kk, lowest row on ties
    double2 a = A[kk * kMaxBlock + i];
    double mag = (i >= kk && i < sz) ? a.x * a.x + a.y * a.y : -1.0;
    int arg = i;
    for (int o = 32; o > 0; o >>= 1) {
      const double om = __shfl_xor(mag, o, 64);
      const int oa = __shfl_xor(arg, o, 64);
      if (om > mag || (om == mag && oa < arg)) {
        mag = om;
        arg = oa;
      }
    }
    const int piv = __shfl(arg, 0, 64);
    const double pmag = __shfl(mag, 0, 64);
    if (i == 0) perm[kk] = piv;
    if (!(pmag > 0.0)) {
      if (i == 0) atomicOr(status, 1);
      return;   // uniform across the workgroup
    }
    if (piv != kk) {   // swap rows kk and piv; thread i owns column i
      const double2 t0 = A[i * kMaxBlock + kk];
      A[i * kMaxBlock + kk] = A[i * kMaxBlock + piv];
      A[i * kMaxBlock + piv] = t0;
    }
    __syncthreads();
    const double2 pv = A[kk * kMaxBlock + kk];
    const double den = pv.x * pv.x + pv.y * pv.y;
    const double2 inv = make_double2(pv.x / den, -pv.y / den);
    __syncthreads();
    // scale row kk (thread i owns column i); A(kk, kk) becomes 1 / pivot
    if (i < sz) A[i * kMaxBlock + kk] = (i == kk) ? inv : cmul(A[i * kMaxBlock + kk], inv);
    __syncthreads();
    if (i < sz && i != kk) {
      const double2 f = A[kk * kMaxBlock + i];
      A[kk * kMaxBlock + i] = make_double2(0.0, 0.0);
      // eight columns per round, all loads before the stores: the compiler
      // cannot tell that row kk (read) and row i (written) never alias, and
      // one dependent LDS round trip per column left the update latency-bound
      int j = 0;
      for (; j + 8 <= sz; j += 8) {
        double2 rk[8], av[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          rk[u] = A[(j + u) * kMaxBlock + kk];
          av[u] = A[(j + u) * kMaxBlock + i];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) A[(j + u) * kMaxBlock + i] = csub(av[u], cmul(f, rk[u]));
      }
      for (; j < sz; ++j) {
        const double2 rk = A[j * kMaxBlock + kk];
        A[j * kMaxBlock + i] = csub(A[j * kMaxBlock + i], cmul(f, rk));
      }
    }
    __syncthreads();
  }
  // undo the row interchanges on the columns, last first (thread i owns row i)
  for (int kk = sz - 1; kk >= 0; --kk) {
    const int p = perm[kk];
    if (p != kk && i < sz) {
      const double2 t0 = A[kk * kMaxBlock + i];
      A[kk * kMaxBlock + i] = A[p * kMaxBlock + i];
      A[p * kMaxBlock + i] = t0;
    }
  }
  __syncthreads();
  // all 64 columns: those past sz are zero (the MFMA apply reads them)
  double2* out = minv + (int64_t)k * kMaxBlock * kMaxBlock;
  for (int j = 0; j < kMaxBlock; ++j) out[j * kMaxBlock + i] = A[j * kMaxBlock + i];
}

// rbuf[l*nt + t] = s_l J_t . |K|/4 (grad l_b - grad l_a)   (int J . w_l)
__global__ __launch_bounds__(kThreads) void k_rhs_elem(int64_t nt, const double* __restrict__ xyz,
                                                       const int* __restrict__ tet,
                                                       const uint8_t* __restrict__ signbits,
                                                       const double* __restrict__ J, double* __restrict__ rbuf) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nt) return;
  const int4 nd = reinterpret_cast<const int4*>(tet)[t];
  const int n[4] = {nd.x, nd.y, nd.z, nd.w};
  double p[4][3];
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int j = 0; j < 3; ++j) p[k][j] = xyz[3 * (int64_t)n[k] + j];
  double e1[3], e2[3], e3[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    e1[j] = p[1][j] - p[0][j];
    e2[j] = p[2][j] - p[0][j];
    e3[j] = p[3][j] - p[0][j];
  }
  const double c23[3] = {e2[1] * e3[2] - e2[2] * e3[1], e2[2] * e3[0] - e2[0] * e3[2], e2[0] * e3[1] - e2[1] * e3[0]};
  const double c31[3] = {e3[1] * e1[2] - e3[2] * e1[1], e3[2] * e1[0] - e3[0] * e1[2], e3[0] * e1[1] - e3[1] * e1[0]};
  const double c12[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
  const double det = e1[0] * c23[0] + e1[1] * c23[1] + e1[2] * c23[2];
  const double v4 = fabs(det) * (1.0 / 24.0);
  const double id = 1.0 / det;
  const double Jx = J[3 * t], Jy = J[3 * t + 1], Jz = J[3 * t + 2];
  // J . grad l_k
  double jg[4];
  jg[1] = (Jx * c23[0] + Jy * c23[1] + Jz * c23[2]) * id;
  jg[2] = (Jx * c31[0] + Jy * c31[1] + Jz * c31[2]) * id;
  jg[3] = (Jx * c12[0] + Jy * c12[1] + Jz * c12[2]) * id;
  jg[0] = -(jg[1] + jg[2] + jg[3]);
  constexpr int ea[6] = {0, 0, 0, 1, 1, 2};
  constexpr int eb[6] = {1, 2, 3, 2, 3, 3};
  const uint8_t sb = signbits[t];
#pragma unroll
  for (int l = 0; l < 6; ++l) {
    const double sgn = ((sb >> l) & 1) ? -1.0 : 1.0;
    rbuf[(int64_t)l * nt + t] = sgn * v4 * (jg[eb[l]] - jg[ea[l]]);
  }
}

// ---------------------------------------------------------------------------
// Solve kernels
// ---------------------------------------------------------------------------
constexpr int kLanes = 8;   // lanes per CSR row

// t_n = (tau / D0_n) sum_e W~_en x_e   (W~^T rows = nodes)
__global__ __launch_bounds__(kThreads) void k_wt(int64_t nv, const int* __restrict__ wtrowptr,
                                                 const int* __restrict__ wtcol, const double* __restrict__ wtval,
                                                 const double* __restrict__ d0tau, const double2* __restrict__ x,
                                                 double2* __restrict__ t) {
  const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kLanes;
  const int lane = threadIdx.x % kLanes;
  double2 acc = make_double2(0.0, 0.0);
  if (row < nv)
    for (int p = wtrowptr[row] + lane; p < wtrowptr[row + 1]; p += kLanes) acc = rfma(wtval[p], x[wtcol[p]], acc);
  for (int o = kLanes / 2; o > 0; o >>= 1) {
    acc.x += __shfl_xor(acc.x, o, kLanes);
    acc.y += __shfl_xor(acc.y, o, kLanes);
  }
  if (row < nv && lane == 0) {
    const double f = d0tau ? d0tau[row] : 1.0;
    t[row] = make_double2(acc.x * f, acc.y * f);
  }
}

// d_n = (G^T b)_n = sum over edges e incident to n of (+b_e if n = hi(e), -b_e if n = lo(e));
// the incident edges are found in node n's row of W~^T (edges sharing a tet with n).
__global__ __launch_bounds__(kThreads) void k_edge_divergence(int64_t nv, const int* __restrict__ wtrowptr,
                                                              const int* __restrict__ wtcol,
                                                              const int* __restrict__ edges,
                                                              const double2* __restrict__ b, double2* __restrict__ d) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nv) return;
  double2 acc = make_double2(0.0, 0.0);
  for (int q = wtrowptr[n]; q < wtrowptr[n + 1]; ++q) {
    const int e = wtcol[q];
    const int lo = edges[2 * e], hi = edges[2 * e + 1];
    if (hi == n) acc = cadd(acc, b[e]);
    else if (lo == n) acc = csub(acc, b[e]);
  }
  d[n] = acc;
}

// diag(W^T G)_n = sum_{e incident to n} W_en G_en, with W_en = W~_en / s_e
__global__ __launch_bounds__(kThreads) void k_lap_diag(int64_t nv, const int* __restrict__ wtrowptr,
                                                       const int* __restrict__ wtcol,
                                                       const double* __restrict__ wtval,
                                                       const int* __restrict__ edges, const double* __restrict__ s,
                                                       double* __restrict__ diag) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nv) return;
  double acc = 0.0;
  for (int q = wtrowptr[n]; q < wtrowptr[n + 1]; ++q) {
    const int e = wtcol[q];
    const int lo = edges[2 * e], hi = edges[2 * e + 1];
    if (hi == n) acc += wtval[q] / s[e];
    else if (lo == n) acc -= wtval[q] / s[e];
  }
  diag[n] = acc;
}

// L = W^T G row by row (one thread per node, fixed order): the entry for
// edge e in row n of W~^T (value s_e W_en) adds W_en at the edge's head and
// subtracts it at its tail.
__global__ __launch_bounds__(kThreads) void k_lap_assemble(int64_t nv, const int* __restrict__ wtrowptr,
                                                           const int* __restrict__ wtcol,
                                                           const double* __restrict__ wtval,
                                                           const int* __restrict__ edges,
                                                           const double* __restrict__ s,
                                                           const int* __restrict__ lrowptr,
                                                           const int* __restrict__ lcol, double* __restrict__ lval) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nv) return;
  const int l0 = lrowptr[n], l1 = lrowptr[n + 1];
  for (int p = l0; p < l1; ++p) lval[p] = 0.0;
  for (int q = wtrowptr[n]; q < wtrowptr[n + 1]; ++q) {
    const int e = wtcol[q];
    const double f = wtval[q] / s[e];
    const int lo = edges[2 * e], hi = edges[2 * e + 1];
    for (int p = l0; p < l1; ++p) {
      if (lcol[p] == hi) lval[p] += f;
      if (lcol[p] == lo) lval[p] -= f;
    }
  }
}

// Projection CG, fused: q = L p with per-block partial sums of p^H q
// (grid-stride over rows, kLanes lanes per row).
__global__ __launch_bounds__(kThreads) void k_lap_spmv_dot(int64_t nv, const int* __restrict__ lrowptr,
                                                           const int* __restrict__ lcol,
                                                           const double* __restrict__ lval,
                                                           const double2* __restrict__ p, double2* __restrict__ q,
                                                           double2* __restrict__ partial) {
  __shared__ double sh[4];
  const int lane = threadIdx.x % kLanes;
  double2 acc = make_double2(0.0, 0.0);
  const int64_t rows_per = (int64_t)gridDim.x * (blockDim.x / kLanes);
  for (int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kLanes; row < nv; row += rows_per) {
    double2 y = make_double2(0.0, 0.0);
    for (int k = lrowptr[row] + lane; k < lrowptr[row + 1]; k += kLanes) y = rfma(lval[k], p[lcol[k]], y);
    for (int o = kLanes / 2; o > 0; o >>= 1) {
      y.x += __shfl_xor(y.x, o, kLanes);
      y.y += __shfl_xor(y.y, o, kLanes);
    }
    if (lane == 0) {
      q[row] = y;
      acc = cfma_conj(p[row], y, acc);
    }
  }
  const double re = block_sum(acc.x, sh), im = block_sum(acc.y, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = make_double2(re, im);
}

// Projection CG, fused: alpha = rz / pq; psi += alpha p; r -= alpha q;
// z = r / diag; per-block partial sums of r^H z.  pq is summed here from the
// kRedBlocks partials of k_lap_spmv_dot, in the fixed order of k_reduce_cols.
__global__ __launch_bounds__(kThreads) void k_cg_update(int64_t n, const double2* __restrict__ rz,
                                                        const double2* __restrict__ pq_part,
                                                        const double2* __restrict__ p,
                                                        const double2* __restrict__ q, const double* __restrict__ diag,
                                                        double2* __restrict__ psi, double2* __restrict__ r,
                                                        double2* __restrict__ z, double2* __restrict__ partial) {
  __shared__ double sh[4];
  __shared__ double den_s;
  double d = 0.0;
  for (int b = threadIdx.x; b < kRedBlocks; b += blockDim.x) d += pq_part[b].x;
  d = block_sum(d, sh);
  if (threadIdx.x == 0) den_s = d;
  __syncthreads();
  const double den = den_s;
  const double a = den != 0.0 ? rz[0].x / den : 0.0;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    psi[i] = rfma(a, p[i], psi[i]);
    const double2 ri = rfma(-a, q[i], r[i]);
    r[i] = ri;
    const double f = diag[i] != 0.0 ? 1.0 / diag[i] : 0.0;
    const double2 zi = make_double2(ri.x * f, ri.y * f);
    z[i] = zi;
    acc = fma(ri.x, zi.x, fma(ri.y, zi.y, acc));
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = make_double2(acc, 0.0);
}

// z = r / diag
__global__ __launch_bounds__(kThreads) void k_jacobi(int64_t n, const double2* __restrict__ r,
                                                     const double* __restrict__ diag, double2* __restrict__ z) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double f = diag[i] != 0.0 ? 1.0 / diag[i] : 0.0;
  z[i] = make_double2(r[i].x * f, r[i].y * f);
}

// p = z + (rz_new / rz_old) p, with rz_new summed here from the kRedBlocks
// partials of k_cg_update (the fixed order of k_reduce_cols); workgroup 0
// stores it for the next iteration's k_cg_update.
__global__ __launch_bounds__(kThreads) void k_cg_dir(int64_t n, const double2* __restrict__ rz_part,
                                                     const double2* __restrict__ rz_old,
                                                     double2* __restrict__ rz_new,
                                                     const double2* __restrict__ z, double2* __restrict__ p) {
  __shared__ double sh[4];
  __shared__ double num_s;
  double a = 0.0;
  for (int b = threadIdx.x; b < kRedBlocks; b += blockDim.x) a += rz_part[b].x;
  a = block_sum(a, sh);
  if (threadIdx.x == 0) {
    num_s = a;
    if (blockIdx.x == 0) rz_new[0] = make_double2(a, 0.0);
  }
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double den = rz_old[0].x;
  const double bta = den != 0.0 ? num_s / den : 0.0;
  p[i] = rfma(bta, p[i], z[i]);
}

// Coulomb projection: A_e -= psi_hi - psi_lo;  V_c += i omega psi(node c)
__global__ __launch_bounds__(kThreads) void k_project(int64_t ne, int64_t nc, const int* __restrict__ edges,
                                                      const int* __restrict__ cond_nodes,
                                                      const double2* __restrict__ psi, double omega,
                                                      double2* __restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ne) {
    x[i] = csub(x[i], csub(psi[edges[2 * i + 1]], psi[edges[2 * i]]));
  } else if (i < ne + nc) {
    const double2 q = psi[cond_nodes[i - ne]];
    x[i] = cadd(x[i], make_double2(-omega * q.y, omega * q.x));
  }
}

// y = M~ x (+ W~ t on A rows if wrowptr), 8 lanes per row; y = b - (...) if b.
// Arithmetic in the storage precision T.
// y = M x (or b - M x) on the sliced ELL copy: one wavefront per slice, one
// lane per row; each step of the loop reads 64 consecutive values and column
// indices (streamed past the L2), the slice width is uniform over the
// wavefront.  Workgroups loop over groups of 4 slices.  Schedule 0: group g,
// g + grid, ... (all XCDs sweep the rows together).  Schedule 1: workgroups
// are dispatched round-robin over the kXcds XCDs (workgroup i on XCD i mod
// kXcds), and each XCD takes a contiguous range of groups holding an equal
// share of the stored entries (xcd_groups[kXcds + 1]), so the rows sharing
// gathered x entries stay under one L2.  Each row's sum has the same
// order in every schedule and grid size.
constexpr int kXcds = 8;
template <class T>
__global__ __launch_bounds__(kThreads) void k_spmv_sell(int64_t ns, const int* __restrict__ sptr,
                                                        const int* __restrict__ srow, const int* __restrict__ scol,
                                                        const T* __restrict__ sval, const T* __restrict__ x,
                                                        const double2* __restrict__ b, T* __restrict__ y,
                                                        int schedule, const int* __restrict__ xcd_groups,
                                                        const int* __restrict__ scplx) {
  static_assert(kSellC == 64, "one wavefront per slice");
  constexpr int kGroup = kThreads / 64;
  const int l = threadIdx.x & 63;
  const int64_t ngroups = (ns + kGroup - 1) / kGroup;
  int64_t g0, g1, gstep;
  if (schedule == 0) {
    g0 = blockIdx.x;
    g1 = ngroups;
    gstep = gridDim.x;
  } else {
    const int64_t xcd = blockIdx.x % kXcds, q = blockIdx.x / kXcds;
    const int64_t nwg = gridDim.x / kXcds + (xcd < (int64_t)(gridDim.x % kXcds) ? 1 : 0);
    g0 = xcd_groups[xcd] + q;      // ranges of equal stored entries
    g1 = xcd_groups[xcd + 1];
    gstep = nwg;
  }
  for (int64_t g = g0; g < g1; g += gstep) {
    const int64_t s = g * kGroup + (threadIdx.x >> 6);
    if (s >= ns) break;
    const int row = srow[s * kSellC + l];
    const int p0 = sptr[s];
    const int w = (sptr[s + 1] - p0) / kSellC;
    const int* __restrict__ c = scol + p0 + l;
    const T* __restrict__ v = sval + p0 + l;
    T acc = zero2<T>();
    // column loads, then gathers, unrolled as deep as occupancy allows
    // (measured: complex64 8 deep, 7 waves per SIMD; complex128 4 deep)
    if constexpr (sizeof(T) == 8) {
      if (scplx && !scplx[s]) {
        // real slice: the same products with a zero imaginary part, values
        // of half the size
        const float* __restrict__ vr = reinterpret_cast<const float*>(sval) + 2 * (int64_t)p0 + l;
#pragma unroll 8
        for (int j = 0; j < w; ++j) {
          const float a = ld_stream(vr + j * kSellC);
          const T xv = x[ld_stream(c + j * kSellC)];
          acc.x = fmaf(a, xv.x, acc.x);
          acc.y = fmaf(a, xv.y, acc.y);
        }
      } else {
#pragma unroll 8
        for (int j = 0; j < w; ++j) acc = cfmaT(ld_stream(v + j * kSellC), x[ld_stream(c + j * kSellC)], acc);
      }
    } else {
      if (scplx && !scplx[s]) {
        const double* __restrict__ vr = reinterpret_cast<const double*>(sval) + 2 * (int64_t)p0 + l;
#pragma unroll 4
        for (int j = 0; j < w; ++j) {
          const double a = ld_stream(vr + j * kSellC);
          const T xv = x[ld_stream(c + j * kSellC)];
          acc.x = fma(a, xv.x, acc.x);
          acc.y = fma(a, xv.y, acc.y);
        }
      } else {
#pragma unroll 4
        for (int j = 0; j < w; ++j) acc = cfmaT(ld_stream(v + j * kSellC), x[ld_stream(c + j * kSellC)], acc);
      }
    }
    if (row >= 0) y[row] = b ? st2<T>(csub(b[row], ld2(acc))) : acc;
  }
}

// y_A += sign * W t over the A rows (factored gauge term; kLanes lanes per row).
template <class T>
__global__ __launch_bounds__(kThreads) void k_gauge_add(int64_t ne, const int* __restrict__ wrowptr,
                                                        const int* __restrict__ wcol, const double* __restrict__ wval,
                                                        const double2* __restrict__ t, double sign,
                                                        T* __restrict__ y) {
  const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kLanes;
  const int lane = threadIdx.x % kLanes;
  double2 ga = make_double2(0.0, 0.0);
  if (row < ne)
    for (int p = wrowptr[row] + lane; p < wrowptr[row + 1]; p += kLanes) ga = rfma(wval[p], t[wcol[p]], ga);
  for (int o = kLanes / 2; o > 0; o >>= 1) {
    ga.x += __shfl_xor(ga.x, o, kLanes);
    ga.y += __shfl_xor(ga.y, o, kLanes);
  }
  if (row < ne && lane == 0) {
    const double2 yo = ld2(y[row]);
    y[row] = st2<T>(make_double2(fma(sign, ga.x, yo.x), fma(sign, ga.y, yo.y)));
  }
}

// Values of the sliced ELL copy from the CSR values (padding = 0).
// Values of the sliced ELL copies from the CSR values (padding = 0), one
// wavefront per slice.  A slice whose values all have a zero imaginary part
// is stored real in both copies: entry j of lane l as the double (complex128
// copy) or float (complex64 copy) at 2 sptr[s] + 64 j + l, the first half of
// the slice's range, and scplx[s] = 0; otherwise complex at sptr[s] + 64 j + l
// and scplx[s] = 1.
__global__ __launch_bounds__(kThreads) void k_sell_values(int64_t ns, const int* __restrict__ sptr,
                                                          const int* __restrict__ src, const double2* __restrict__ val,
                                                          double2* __restrict__ sval, float2* __restrict__ sval32,
                                                          int* __restrict__ scplx) {
  const int64_t s = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int l = threadIdx.x & 63;
  if (s >= ns) return;              // uniform over the wavefront
  const int p0 = sptr[s], w = (sptr[s + 1] - p0) / kSellC;
  bool im = false;
  for (int j = 0; j < w; ++j) {
    const int p = src[p0 + j * kSellC + l];
    if (p >= 0 && val[p].y != 0.0) im = true;
  }
  const bool cplx = __ballot(im) != 0;
  if (l == 0) scplx[s] = cplx ? 1 : 0;
  double* __restrict__ re = reinterpret_cast<double*>(sval) + 2 * (int64_t)p0 + l;
  float* __restrict__ re32 = reinterpret_cast<float*>(sval32) + 2 * (int64_t)p0 + l;
  for (int j = 0; j < w; ++j) {
    const int q = p0 + j * kSellC + l;
    const int p = src[q];
    const double2 v = p >= 0 ? val[p] : make_double2(0.0, 0.0);
    if (cplx) {
      sval[q] = v;
      sval32[q] = make_float2((float)v.x, (float)v.y);
    } else {
      re[j * kSellC] = v.x;
      re32[j * kSellC] = (float)v.x;
    }
  }
}

// z_I = Minv_I r_I, one 64-lane wavefront per block, 4 blocks per workgroup;
// MT the storage of the inverses (T, or packed complex half with T = float2).
template <class T, class MT, class RT>
__global__ __launch_bounds__(kThreads) void k_block_apply(int64_t nb, const int* __restrict__ blk_ptr,
                                                          const int* __restrict__ blk_dofs,
                                                          const MT* __restrict__ minv, const RT* __restrict__ r,
                                                          T* __restrict__ z) {
  __shared__ T rl[4][kMaxBlock];
  const int w = threadIdx.x >> 6, i = threadIdx.x & 63;
  const int64_t k = (int64_t)blockIdx.x * 4 + w;
  int b0 = 0, sz = 0, dof = -1;
  if (k < nb) {
    b0 = blk_ptr[k];
    sz = blk_ptr[k + 1] - b0;
    if (i < sz) dof = blk_dofs[b0 + i];
  }
  rl[w][i] = dof >= 0 ? st2<T>(ld2(r[dof])) : zero2<T>();
  __syncthreads();
  if (dof < 0) return;
  const MT* Mk = minv + k * kMaxBlock * kMaxBlock;
  T acc = zero2<T>();
  for (int j = 0; j < sz; ++j) acc = cfmaT(as_vec(ld_stream(Mk + j * kMaxBlock + i)), rl[w][j], acc);
  z[dof] = acc;
}

// partial[(c*8+k) * kRedBlocks + blockIdx.x] = sum_i conj(V_{c*8+k}[i]) w[i]  (FP64 accumulation).
// With want_norm, the y = 0 slice also writes sum_i |w_i|^2 to slot q.  A
// non-null flag equal to 0 skips the launch (conditional second CGS pass).
// Each workgroup owns 512 consecutive rows (two per thread) and the 8
// vectors c0..c0+7 of slice blockIdx.y; per-block sums go to
// partial[(c0+k) * gridDim.x + blockIdx.x].  With want_norm, slice 0 also
// writes sum |w|^2 to slot q.  A non-null flag equal to 0 skips the launch.
template <class T>
__global__ __launch_bounds__(kThreads) void k_mdot(int64_t n, const T* __restrict__ V, int64_t ldv, int q,
                                                   const T* __restrict__ w, double2* __restrict__ partial,
                                                   int want_norm, const int* __restrict__ flag, int64_t vstride,
                                                   int64_t wstride, int64_t pstride, const int* __restrict__ active) {
  // right-hand side z of a batch (grid.z); strides are 0 for a single system
  const int z = blockIdx.z;
  if ((active && !active[z]) || (flag && flag[z] == 0)) return;
  V += z * vstride;
  w += z * wstride;
  partial += z * pstride;
  __shared__ double2 red[4][9];
  const int c0 = blockIdx.y * 8;
  const int cnt = min(8, q - c0);
  const bool nrm = want_norm && blockIdx.y == 0;
  const int64_t i0 = (int64_t)blockIdx.x * (2 * kThreads) + threadIdx.x;
  const int64_t i1 = i0 + kThreads;
  const bool a0 = i0 < n, a1 = i1 < n;
  const double2 w0 = a0 ? ld2(w[i0]) : make_double2(0.0, 0.0);
  const double2 w1 = a1 ? ld2(w[i1]) : make_double2(0.0, 0.0);
  double2 acc[9];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    acc[k] = make_double2(0.0, 0.0);
    if (k < cnt) {
      const T* Vk = V + (int64_t)(c0 + k) * ldv;
      if (a0) acc[k] = cfma_conj(ld2(Vk[i0]), w0, acc[k]);
      if (a1) acc[k] = cfma_conj(ld2(Vk[i1]), w1, acc[k]);
    }
  }
  acc[8] = make_double2(w0.x * w0.x + w0.y * w0.y + w1.x * w1.x + w1.y * w1.y, 0.0);
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
  const int nk = nrm ? 9 : 8;
#pragma unroll
  for (int k = 0; k < 9; ++k)
    if (k < nk && (k < cnt || k == 8)) {
      const double re = wave_sum(acc[k].x), im = wave_sum(acc[k].y);
      if (ln == 0) red[wv][k] = make_double2(re, im);
    }
  __syncthreads();
  const int t = threadIdx.x;
  const int slot = t < cnt ? t : (nrm && t == 8 ? 8 : -1);
  if (slot >= 0) {
    const double2 r = make_double2((red[0][slot].x + red[1][slot].x) + (red[2][slot].x + red[3][slot].x),
                                   (red[0][slot].y + red[1][slot].y) + (red[2][slot].y + red[3][slot].y));
    const int col = slot == 8 ? q : c0 + slot;
    partial[(int64_t)col * gridDim.x + blockIdx.x] = r;
  }
}

// ---- Arnoldi by classical Gram-Schmidt with delayed reorthogonalisation
// (DCGS2: the second projection of basis vector j is fused with the first
// projection of the next direction; Swirydowicz, Langou, Ananthan, Yang and
// Thomas, Low synchronization Gram-Schmidt and GMRES algorithms, Numer.
// Linear Algebra Appl. 2021).  Per Arnoldi step the basis is read twice
// (one fused dot pass, one fused update pass) instead of four times.
//
// Fused dots of the pending vector v and the new direction w against the q
// finished basis vectors, one read of V: partial columns k < q: V_k^H v,
// q + k: V_k^H w, 2q: v^H v, 2q + 1: v^H w (FP64 sums beyond a thread's
// own rows).  Workgroup (x, y) takes the vectors 8y..8y+7 and the tiles x,
// x + gridDim.x, ...;
// a thread takes R = rows_of<VT>::R consecutive rows of a tile with 16-byte
// loads (vec: every vector 16-byte aligned, ldv a multiple of R; otherwise,
// and for a ragged last group, entry by entry).  A slice with fewer than 8
// vectors repeats its first one in the spare slots, so the loads of a row
// group carry no branches and are all issued before the first product; the
// spare sums are dropped.  The wavefront reductions happen once per
// workgroup; slice y = 0 also forms v^H v and v^H w.
constexpr int kDot2MaxBlocks = 1024;
template <class VT, class T>
__global__ __launch_bounds__(kThreads) void k_mdot2(int64_t n, const VT* __restrict__ V, int64_t ldv, int q,
                                                    const VT* __restrict__ v, const T* __restrict__ w,
                                                    double2* __restrict__ partial, int64_t vstride, int64_t wstride,
                                                    int64_t pstride, const int* __restrict__ active, int vec) {
  constexpr int R = rows_of<VT>::R;
  static_assert(rows_of<T>::R == R, "basis and direction row groups differ");
  // system z of a batch (grid.z); strides are 0 for a single system
  const int zs = blockIdx.z;
  if (active && !active[zs]) return;
  V += zs * vstride;
  v += zs * vstride;
  w += zs * wstride;
  partial += zs * pstride;
  using A = typename dot_acc<T>::type;
  __shared__ double2 red[4][18];
  const int nparts = gridDim.x, bx = blockIdx.x;
  const int c0 = blockIdx.y * 8;
  const int cnt = max(0, min(8, q - c0));
  const bool norms = blockIdx.y == 0;
  const double us = basis_unscale<VT>();
  const VT* Vc[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) Vc[k] = V + (int64_t)(c0 + (k < cnt ? k : 0)) * ldv;
  A as[8], ar[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    to_acc(make_double2(0.0, 0.0), as[k]);
    to_acc(make_double2(0.0, 0.0), ar[k]);
  }
  double aa = 0.0;
  double2 bb = make_double2(0.0, 0.0);
  for (int64_t i0 = ((int64_t)bx * kThreads + threadIdx.x) * R; i0 < n; i0 += (int64_t)nparts * kThreads * R) {
    A vr[R], wr[R];
    if (vec && i0 + R <= n) {
      ld_rows(v + i0, vr);
      ld_rows(w + i0, wr);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        vr[r].x *= us;
        vr[r].y *= us;
      }
      if (cnt > 0) {
        A x[8][R];
#pragma unroll
        for (int k = 0; k < 8; ++k) ld_rows(Vc[k] + i0, x[k]);
#pragma unroll
        for (int k = 0; k < 8; ++k)
#pragma unroll
          for (int r = 0; r < R; ++r) {
            as[k] = cfma_conj(x[k][r], vr[r], as[k]);
            ar[k] = cfma_conj(x[k][r], wr[r], ar[k]);
          }
      }
    } else {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int64_t i = i0 + r;
        to_acc(i < n ? ld2(v[i]) : make_double2(0.0, 0.0), vr[r]);
        to_acc(i < n ? ld2(w[i]) : make_double2(0.0, 0.0), wr[r]);
      }
#pragma unroll
      for (int k = 0; k < 8; ++k)
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int64_t i = i0 + r;
          if (k < cnt && i < n) {
            const A x = raw_as(Vc[k][i], A{});
            as[k] = cfma_conj(x, vr[r], as[k]);
            ar[k] = cfma_conj(x, wr[r], ar[k]);
          }
        }
    }
    if (norms) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const double2 a = make_double2(vr[r].x, vr[r].y), b = make_double2(wr[r].x, wr[r].y);
        aa = fma(a.x, a.x, fma(a.y, a.y, aa));
        bb = cfma_conj(a, b, bb);
      }
    }
  }
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < 8; ++k)
    if (k < cnt) {
      const double sr = wave_sum((double)as[k].x), si = wave_sum((double)as[k].y);
      const double rr = wave_sum((double)ar[k].x), ri = wave_sum((double)ar[k].y);
      if (ln == 0) {
        red[wv][k] = make_double2(sr * us, si * us);
        red[wv][8 + k] = make_double2(rr * us, ri * us);
      }
    }
  if (norms) {
    aa = wave_sum(aa);
    bb.x = wave_sum(bb.x);
    bb.y = wave_sum(bb.y);
    if (ln == 0) {
      red[wv][16] = make_double2(aa, 0.0);
      red[wv][17] = bb;
    }
  }
  __syncthreads();
  const int t = threadIdx.x;
  int col = -1;
  if (t < 16 && (t & 7) < cnt) col = (t < 8 ? 0 : q) + c0 + (t & 7);
  if (norms && (t == 16 || t == 17)) col = 2 * q + (t - 16);
  if (col >= 0) {
    const double2 r = make_double2((red[0][t].x + red[1][t].x) + (red[2][t].x + red[3][t].x),
                                   (red[0][t].y + red[1][t].y) + (red[2][t].y + red[3][t].y));
    partial[(int64_t)col * nparts + bx] = r;
  }
}

// out[k] = sum_b partial[k * kRedBlocks + b]  (fixed tree per column)
__global__ __launch_bounds__(kThreads) void k_reduce_cols(const double2* __restrict__ partial, int nparts,
                                                          double2* __restrict__ out, const int* __restrict__ flag,
                                                          int64_t pstride, int64_t ostride,
                                                          const int* __restrict__ active) {
  const int z = blockIdx.z;
  if ((active && !active[z]) || (flag && flag[z] == 0)) return;
  partial += z * pstride;
  out += z * ostride;
  __shared__ double sh[4];
  const int k = blockIdx.x;
  double re = 0.0, im = 0.0;
  for (int b = threadIdx.x; b < nparts; b += blockDim.x) {
    re += partial[(int64_t)k * nparts + b].x;
    im += partial[(int64_t)k * nparts + b].y;
  }
  re = block_sum(re, sh);
  im = block_sum(im, sh);
  if (threadIdx.x == 0) out[k] = make_double2(re, im);
}


template <class T>
__global__ __launch_bounds__(kThreads) void k_norm2_partial(int64_t n, const T* __restrict__ w,
                                                            double* __restrict__ partial, int64_t wstride,
                                                            const int* __restrict__ active) {
  const int z = blockIdx.z;
  if (active && !active[z]) return;
  w += z * wstride;
  partial += (int64_t)z * gridDim.x;
  __shared__ double sh[4];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double2 v = ld2(w[i]);
    acc = fma(v.x, v.x, fma(v.y, v.y, acc));
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

__global__ __launch_bounds__(kThreads) void k_norm2_final(const double* __restrict__ partial,
                                                          double* __restrict__ out, const int* __restrict__ flag,
                                                          const int* __restrict__ active) {
  const int z = blockIdx.z;
  if ((active && !active[z]) || (flag && flag[z] == 0)) return;
  partial += (int64_t)z * kRedBlocks;
  out += z;
  __shared__ double sh[4];
  double acc = 0.0;
  for (int b = threadIdx.x; b < kRedBlocks; b += blockDim.x) acc += partial[b];
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) out[0] = sqrt(acc);
}

// v = w / nrm, each thread scale_rows<Ti, To>() consecutive rows (16-byte
// accesses when vec, else entry by entry)
template <class Ti, class To>
constexpr int scale_rows() {
  return rows_of<Ti>::R > rows_of<To>::R ? rows_of<Ti>::R : rows_of<To>::R;
}
template <class Ti, class To>
__global__ __launch_bounds__(kThreads) void k_scale_by_inv(int64_t n, const Ti* __restrict__ w,
                                                           const double* __restrict__ nrm, To* __restrict__ v,
                                                           int64_t wstride, int64_t vstride,
                                                           const int* __restrict__ active, int vec) {
  constexpr int R = scale_rows<Ti, To>();
  const int z = blockIdx.z;
  if (active && !active[z]) return;
  w += z * wstride;
  v += z * vstride;
  nrm += z;
  const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * R;
  if (i0 >= n) return;
  const double a = nrm[0];
  const double f = a > 0.0 ? 1.0 / a : 0.0;
  if (vec && i0 + R <= n) {
    constexpr int Gi = rows_of<Ti>::R, Go = rows_of<To>::R;
    const double fr = f * basis_unscale<Ti>();
    double2 x[R];
#pragma unroll
    for (int g = 0; g < R; g += Gi) ld_rows(w + i0 + g, x + g);
#pragma unroll
    for (int r = 0; r < R; ++r) x[r] = make_double2(x[r].x * fr, x[r].y * fr);
#pragma unroll
    for (int g = 0; g < R; g += Go) st_rows(v + i0 + g, x + g);
    return;
  }
  for (int r = 0; r < R && i0 + r < n; ++r) {
    const double2 x = ld2(w[i0 + r]);
    v[i0 + r] = st2<To>(make_double2(x.x * f, x.y * f));
  }
}

// v = w / ||w|| with ||w||^2 the sum of the kRedBlocks partial sums rpart,
// formed by every workgroup in k_norm2_final's order (so the same value
// everywhere, equal to k_norm2_final's); workgroup 0 stores ||w|| in
// out_norm.  Saves the dependent launch of k_norm2_final per Arnoldi step.
constexpr int kScaleGroups = 2;
template <class Ti, class To>
__global__ __launch_bounds__(kThreads) void k_scale_by_partials(int64_t n, const Ti* __restrict__ w,
                                                                const double* __restrict__ rpart,
                                                                double* __restrict__ out_norm, To* __restrict__ v,
                                                                int vec) {
  constexpr int R = scale_rows<Ti, To>();
  __shared__ double sh[4];
  __shared__ double nrm_s;
  double acc = 0.0;
  for (int b = threadIdx.x; b < kRedBlocks; b += blockDim.x) acc += rpart[b];
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) {
    nrm_s = sqrt(acc);
    if (blockIdx.x == 0) out_norm[0] = nrm_s;
  }
  __syncthreads();
  const double a = nrm_s;
  const double f = a > 0.0 ? 1.0 / a : 0.0;
  // kScaleGroups row groups per thread, a workgroup's width apart (the sum
  // above is formed once per workgroup, so fewer workgroups form it fewer times)
#pragma unroll
  for (int t = 0; t < kScaleGroups; ++t) {
    const int64_t i0 = (((int64_t)blockIdx.x * kScaleGroups + t) * blockDim.x + threadIdx.x) * R;
    if (i0 >= n) return;
    if (vec && i0 + R <= n) {
      constexpr int Gi = rows_of<Ti>::R, Go = rows_of<To>::R;
      const double fr = f * basis_unscale<Ti>();
      double2 x[R];
#pragma unroll
      for (int g = 0; g < R; g += Gi) ld_rows(w + i0 + g, x + g);
#pragma unroll
      for (int r = 0; r < R; ++r) x[r] = make_double2(x[r].x * fr, x[r].y * fr);
#pragma unroll
      for (int g = 0; g < R; g += Go) st_rows(v + i0 + g, x + g);
      continue;
    }
    for (int r = 0; r < R && i0 + r < n; ++r) {
      const double2 x = ld2(w[i0 + r]);
      v[i0 + r] = st2<To>(make_double2(x.x * f, x.y * f));
    }
  }
}

template <class Ti, class To>
__global__ __launch_bounds__(kThreads) void k_scale_host(int64_t n, const Ti* __restrict__ w, double a,
                                                         To* __restrict__ v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double2 x = ld2(w[i]);
  v[i] = st2<To>(make_double2(x.x * a, x.y * a));
}

template <class VT, class T>
__global__ __launch_bounds__(kThreads) void k_combine(int64_t n, const VT* __restrict__ V, int64_t ldv, int q,
                                                      const double2* __restrict__ y, T* __restrict__ u,
                                                      int64_t vstride, int64_t ystride, int64_t ustride,
                                                      const int* __restrict__ qs, const int* __restrict__ active) {
  const int z = blockIdx.z;
  if (active && !active[z]) return;
  V += z * vstride;
  y += z * ystride;
  u += z * ustride;
  if (qs) q = qs[z];
  __shared__ double2 ys[kMaxRestart + 1];
  if (threadIdx.x < q) ys[threadIdx.x] = y[threadIdx.x];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double2 acc = make_double2(0.0, 0.0);
  for (int k = 0; k < q; ++k) acc = cfma(ld2(V[(int64_t)k * ldv + i]), ys[k], acc);
  u[i] = st2<T>(acc);
}

// x += z   (x FP64, z in storage type)
template <class T>
__global__ __launch_bounds__(kThreads) void k_axpy(int64_t n, const T* __restrict__ zv, double2* __restrict__ x,
                                                   int64_t zstride, int64_t xstride, const int* __restrict__ active) {
  const int b = blockIdx.z;
  if (active && !active[b]) return;
  zv += b * zstride;
  x += b * xstride;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = cadd(x[i], ld2(zv[i]));
}

// w <- w - V h (FP64 arithmetic, stored in T) and rpart = per-block ||w||^2:
// the second CGS2 update fused with the norm of the new basis vector.


// ---- Hessenberg least squares on the device (one thread) ----
// Column j of H (row-major, leading dimension m) = h1 + h2 with H(j+1, j) =
// ||w||; applies the previous rotations, forms the new one, updates g and
// writes est[j] = |g(j+1)| / bnorm.  At j = 0, g is reset to (beta, 0, ...).
__device__ void givens_body(int j, int m, const double2* __restrict__ h1, const double2* __restrict__ h2,
                         const double* __restrict__ nrm, double2* __restrict__ H, double* __restrict__ cs,
                         double2* __restrict__ sn, double2* __restrict__ g, double beta, double bnorm,
                         double* __restrict__ est) {
  if (j == 0) {
    for (int i = 0; i <= m; ++i) g[i] = make_double2(0.0, 0.0);
    g[0] = make_double2(beta, 0.0);
  }
  for (int i = 0; i <= j; ++i) H[i * m + j] = cadd(h1[i], h2[i]);
  const double hn = nrm[0];
  for (int i = 0; i < j; ++i) {
    const double2 a = H[i * m + j], b = H[(i + 1) * m + j];
    const double c = cs[i];
    const double2 s = sn[i];
    H[i * m + j] = cadd(make_double2(c * a.x, c * a.y), cmul(s, b));
    const double2 sc = make_double2(s.x, -s.y);
    H[(i + 1) * m + j] = csub(make_double2(c * b.x, c * b.y), cmul(sc, a));
  }
  const double2 a = H[j * m + j];
  const double aa = sqrt(a.x * a.x + a.y * a.y);
  double c;
  double2 s, r;
  if (hn == 0.0) {
    c = 1.0; s = make_double2(0.0, 0.0); r = a;
  } else if (aa == 0.0) {
    c = 0.0; s = make_double2(1.0, 0.0); r = make_double2(hn, 0.0);
  } else {
    const double t = hypot(aa, hn);
    c = aa / t;
    const double2 ph = make_double2(a.x / aa, a.y / aa);
    s = make_double2(ph.x * hn / t, ph.y * hn / t);
    r = make_double2(ph.x * t, ph.y * t);
  }
  cs[j] = c;
  sn[j] = s;
  H[j * m + j] = r;
  const double2 gj = g[j];
  const double2 sc = make_double2(s.x, -s.y);
  const double2 ng = cmul(sc, gj);
  g[j + 1] = make_double2(-ng.x, -ng.y);
  g[j] = make_double2(c * gj.x, c * gj.y);
  est[j] = sqrt(g[j + 1].x * g[j + 1].x + g[j + 1].y * g[j + 1].y) / bnorm;
}

__global__ void k_givens(int j, int m, const double2* __restrict__ h1, const double2* __restrict__ h2,
                         const double* __restrict__ nrm, double2* __restrict__ H, double* __restrict__ cs,
                         double2* __restrict__ sn, double2* __restrict__ g, double beta, double bnorm,
                         double* __restrict__ est) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  givens_body(j, m, h1, h2, nrm, H, cs, sn, g, beta, bnorm, est);
}

// Small linear algebra of DCGS2 step j (one workgroup of 64 threads).  In:
// dots = [s = Q^H v (j), r = Q^H w (j), v^H v, v^H w] with Q the j finished
// basis vectors, v the pending vector (projected once), w the operator
// applied to v; Hraw the unrotated Hessenberg matrix (column-major, leading
// dimension m + 1) whose column j - 1 still holds the once-projected
// coefficients h and tnorm = ||t|| of the previous step (v = t / ||t||).
// With rho = ||v - Q s|| = sqrt(v^H v - |s|^2) (Pythagoras, Q orthonormal):
//   q_j = (v - Q s) / rho;  column j - 1 becomes h + ||t|| s, subdiagonal ||t|| rho;
//   A q_j = (w - Q H(0:j,0:j) s - q_j H(j,j-1) s_{j-1}) / rho, whose
//   coefficients are c = (r - H s) / rho and c_j = ((v^H w - s^H r) / rho
//   - H(j,j-1) s_{j-1}) / rho;  the next direction
//   t' = A q_j - Q c - q_j c_j = w / rho - kappa v / rho - Q g with
//   kappa = H(j,j-1) s_{j-1} / rho + c_j and g = H s / rho + c - kappa s / rho.
// Out: coef = [s (kMaxRestart), g (kMaxRestart), 1 / rho, -kappa / rho];
// Hraw columns j - 1 (final) and j (c, c_j; subdiagonal follows next step);
// the Givens rotation of the now final column j - 1 (estimate after j steps).
__global__ __launch_bounds__(64) void k_dcgs_coef(int j, int m, const double2* __restrict__ dots,
                                                  double2* __restrict__ Hraw, const double* __restrict__ tnorm,
                                                  double2* __restrict__ coef, double2* __restrict__ H,
                                                  double* __restrict__ cs, double2* __restrict__ sn,
                                                  double2* __restrict__ g, double beta, double bnorm,
                                                  double* __restrict__ est, double2* __restrict__ Sall,
                                                  double* __restrict__ rhoall, const double* __restrict__ betas,
                                                  const double* __restrict__ bnorms, int64_t dstride,
                                                  const int* __restrict__ active) {
  static_assert(kMaxRestart <= 64, "one lane per Hessenberg row");
  // system z of a batch (grid.z): per-system arrays at fixed strides; beta
  // and ||b|| from the device arrays when given
  const int zs = blockIdx.z;
  if (active && !active[zs]) return;
  if (betas) {
    beta = betas[zs];
    bnorm = bnorms[zs];
  }
  dots += zs * dstride;
  coef += zs * dstride;
  Hraw += (int64_t)zs * (m + 1) * m;
  H += (int64_t)zs * (m + 1) * m;
  tnorm += zs;
  cs += zs * (m + 1);
  sn += zs * (m + 1);
  g += zs * (m + 2);
  est += zs * (m + 1);
  __shared__ double2 ss[kMaxRestart], rr[kMaxRestart], hs[kMaxRestart], col[kMaxRestart + 1], snl[kMaxRestart];
  __shared__ double csl[kMaxRestart];
  __shared__ double sh_rho;
  __shared__ double2 sh_kappa;
  const int t = threadIdx.x, q = j, ld = m + 1;
  const double2 zero = make_double2(0.0, 0.0);
  const double2 st = t < q ? dots[t] : zero, rt = t < q ? dots[q + t] : zero;
  if (t < q) {
    ss[t] = st;
    rr[t] = rt;
  }
  // |s|^2 and s^H r over the wavefront
  const double s2 = wave_sum(st.x * st.x + st.y * st.y);
  const double2 sr = make_double2(wave_sum(st.x * rt.x + st.y * rt.y), wave_sum(st.x * rt.y - st.y * rt.x));
  const double rho2 = dots[2 * q].x - s2;
  const double rho = rho2 > 0.0 ? sqrt(rho2) : 0.0;
  const double ir = rho > 0.0 ? 1.0 / rho : 0.0;
  if (Sall) {   // the finishing transform of step j, for flexible cycles
    if (t < q) Sall[(int64_t)j * m + t] = st;
    if (t == 0) rhoall[j] = rho;
  }
  double hsubj = 0.0;      // final H(j, j-1)
  if (j >= 1) {
    // column j - 1 becomes h + ||t|| s with subdiagonal ||t|| rho (kept in LDS for the rotations)
    const double tn = tnorm[0];
    double2* hc = Hraw + (int64_t)(j - 1) * ld;
    if (t < j) {
      const double2 c = rfma(tn, st, hc[t]);
      hc[t] = c;
      col[t] = c;
    }
    hsubj = tn * rho;
    if (t == 0) hc[j] = make_double2(hsubj, 0.0);
    if (t < j - 1) {
      csl[t] = cs[t];
      snl[t] = sn[t];
    }
  }
  __syncthreads();
  // H s over the j x j leading block (column k has rows <= k + 1)
  if (t < q) {
    // eight independent loads in flight per round instead of one
    double2 acc = zero;
    for (int k0 = t > 0 ? t - 1 : 0; k0 < q; k0 += 8) {
      double2 h[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) h[u] = Hraw[(int64_t)min(k0 + u, q - 1) * ld + t];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (k0 + u < q) acc = cfma(h[u], ss[k0 + u], acc);
    }
    hs[t] = acc;
  }
  if (t == 0 && j >= 1) {
    // Givens rotations of the now final column j - 1 (earlier rotations, then its own),
    // the running entry kept in registers
    const int jj = j - 1;
    if (jj == 0) {
      for (int i = 0; i <= m; ++i) g[i] = zero;
      g[0] = make_double2(beta, 0.0);
    }
    double2 run = col[0];
    for (int i = 0; i < jj; ++i) {
      const double c = csl[i];
      const double2 sv = snl[i], b = col[i + 1];
      H[i * m + jj] = cadd(make_double2(c * run.x, c * run.y), cmul(sv, b));
      const double2 sc = make_double2(sv.x, -sv.y);
      run = csub(make_double2(c * b.x, c * b.y), cmul(sc, run));
    }
    const double aa = sqrt(run.x * run.x + run.y * run.y);
    double c;
    double2 sv, rr2;
    if (hsubj == 0.0) {
      c = 1.0; sv = zero; rr2 = run;
    } else if (aa == 0.0) {
      c = 0.0; sv = make_double2(1.0, 0.0); rr2 = make_double2(hsubj, 0.0);
    } else {
      const double tt = hypot(aa, hsubj);
      c = aa / tt;
      const double2 ph = make_double2(run.x / aa, run.y / aa);
      sv = make_double2(ph.x * hsubj / tt, ph.y * hsubj / tt);
      rr2 = make_double2(ph.x * tt, ph.y * tt);
    }
    cs[jj] = c;
    sn[jj] = sv;
    H[jj * m + jj] = rr2;
    const double2 gj = g[jj];
    const double2 ng = cmul(make_double2(sv.x, -sv.y), gj);
    g[jj + 1] = make_double2(-ng.x, -ng.y);
    g[jj] = make_double2(c * gj.x, c * gj.y);
    est[jj] = sqrt(ng.x * ng.x + ng.y * ng.y) / bnorm;
  }
  if (t == 0) {
    const double2 hsub = j >= 1 ? make_double2(hsubj * ss[j - 1].x, hsubj * ss[j - 1].y) : zero;
    const double2 vw = csub(dots[2 * q + 1], sr);
    const double2 cj = make_double2((vw.x * ir - hsub.x) * ir, (vw.y * ir - hsub.y) * ir);
    const double2 kappa = make_double2(hsub.x * ir + cj.x, hsub.y * ir + cj.y);
    Hraw[(int64_t)j * ld + j] = cj;
    sh_kappa = kappa;
    coef[2 * kMaxRestart] = make_double2(ir, 0.0);
    coef[2 * kMaxRestart + 1] = make_double2(-kappa.x * ir, -kappa.y * ir);
  }
  __syncthreads();
  if (t < q) {
    const double2 kappa = sh_kappa;
    const double2 c = make_double2((rr[t].x - hs[t].x) * ir, (rr[t].y - hs[t].y) * ir);
    Hraw[(int64_t)j * ld + t] = c;
    const double2 ks = cmul(kappa, ss[t]);
    coef[t] = ss[t];
    coef[kMaxRestart + t] = make_double2(hs[t].x * ir + c.x - ks.x * ir, hs[t].y * ir + c.y - ks.y * ir);
  }
}

// DCGS2 update, one read of V: v <- (v - V s) / rho (the finished basis
// vector j, in place) and w <- w / rho - (kappa / rho) v - V g (the next
// direction, in place), with rpart the per-block sums of |w|^2.  A thread
// takes R = rows_of<VT>::R consecutive rows with 16-byte accesses (vec as in
// k_mdot2) and the basis four vectors at a time.
template <class VT, class T>
__global__ __launch_bounds__(kThreads) void k_dcgs_update(int64_t n, const VT* __restrict__ V, int64_t ldv, int q,
                                                          const double2* __restrict__ coef, VT* __restrict__ v,
                                                          T* __restrict__ w, double* __restrict__ rpart,
                                                          int64_t vstride, int64_t wstride, int64_t cstride,
                                                          const int* __restrict__ active, int vec) {
  constexpr int R = rows_of<VT>::R;
  static_assert(rows_of<T>::R == R, "basis and direction row groups differ");
  const int zs = blockIdx.z;
  if (active && !active[zs]) return;
  V += zs * vstride;
  v += zs * vstride;
  w += zs * wstride;
  coef += zs * cstride;
  rpart += (int64_t)zs * gridDim.x;
  __shared__ double2 cs_[kMaxRestart], cg_[kMaxRestart];
  __shared__ double sh[4];
  const double us = basis_unscale<VT>();
  if (threadIdx.x < q) {
    // the basis is read unscaled: fold the factor into the coefficients
    const double2 a = coef[threadIdx.x], b = coef[kMaxRestart + threadIdx.x];
    cs_[threadIdx.x] = make_double2(a.x * us, a.y * us);
    cg_[threadIdx.x] = make_double2(b.x * us, b.y * us);
  }
  __syncthreads();
  const double ir = coef[2 * kMaxRestart].x;
  const double2 bv = coef[2 * kMaxRestart + 1];
  double acc = 0.0;
  for (int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * R; i0 < n;
       i0 += (int64_t)gridDim.x * blockDim.x * R) {
    double2 vi[R], wi[R], qa[R], ga[R];
    const bool fast = vec && i0 + R <= n;
    if (fast) {
      ld_rows(v + i0, vi);
      ld_rows(w + i0, wi);
#pragma unroll
      for (int r = 0; r < R; ++r) vi[r] = make_double2(vi[r].x * us, vi[r].y * us);
    } else {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        vi[r] = i0 + r < n ? ld2(v[i0 + r]) : make_double2(0.0, 0.0);
        wi[r] = i0 + r < n ? ld2(w[i0 + r]) : make_double2(0.0, 0.0);
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) qa[r] = ga[r] = make_double2(0.0, 0.0);
    if (fast) {
      int k = 0;
      for (; k + 4 <= q; k += 4) {
        double2 x[4][R];
#pragma unroll
        for (int u = 0; u < 4; ++u) ld_rows(V + (int64_t)(k + u) * ldv + i0, x[u]);
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int r = 0; r < R; ++r) {
            qa[r] = cfma(x[u][r], cs_[k + u], qa[r]);
            ga[r] = cfma(x[u][r], cg_[k + u], ga[r]);
          }
      }
      for (; k < q; ++k) {
        double2 x[R];
        ld_rows(V + (int64_t)k * ldv + i0, x);
#pragma unroll
        for (int r = 0; r < R; ++r) {
          qa[r] = cfma(x[r], cs_[k], qa[r]);
          ga[r] = cfma(x[r], cg_[k], ga[r]);
        }
      }
    } else {
      for (int k = 0; k < q; ++k)
#pragma unroll
        for (int r = 0; r < R; ++r)
          if (i0 + r < n) {
            const double2 x = raw2(V[(int64_t)k * ldv + i0 + r]);
            qa[r] = cfma(x, cs_[k], qa[r]);
            ga[r] = cfma(x, cg_[k], ga[r]);
          }
    }
    double2 vo[R], wo[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      vo[r] = make_double2((vi[r].x - qa[r].x) * ir, (vi[r].y - qa[r].y) * ir);
      const double2 bvi = cmul(bv, vi[r]);
      // |w|^2 of the value as stored
      wo[r] = ld2(st2<T>(make_double2(wi[r].x * ir + bvi.x - ga[r].x, wi[r].y * ir + bvi.y - ga[r].y)));
    }
    if (fast) {
      st_rows(v + i0, vo);
      st_rows(w + i0, wo);
    } else {
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (i0 + r < n) {
          v[i0 + r] = st2<VT>(vo[r]);
          w[i0 + r] = st2<T>(wo[r]);
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (i0 + r < n) acc = fma(wo[r].x, wo[r].x, fma(wo[r].y, wo[r].y, acc));
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) rpart[blockIdx.x] = acc;
}

// One right-hand side per workgroup z; per-system arrays at fixed strides,
// beta and bnorm from device arrays.
__global__ void k_givens_b(int j, int m, const double2* __restrict__ h1, const double2* __restrict__ h2,
                           const double* __restrict__ nrm, double2* __restrict__ H, double* __restrict__ cs,
                           double2* __restrict__ sn, double2* __restrict__ g, const double* __restrict__ beta,
                           const double* __restrict__ bnorm, double* __restrict__ est, int64_t hstride,
                           int64_t h2stride, const int* __restrict__ active) {
  const int z = blockIdx.z;
  if (threadIdx.x != 0 || (active && !active[z])) return;
  givens_body(j, m, h1 + z * hstride, h2 + z * h2stride, nrm + z, H + (int64_t)z * (m + 1) * m, cs + z * (m + 1),
              sn + z * (m + 1), g + z * (m + 2), beta[z], bnorm[z], est + z * (m + 1));
}

// y = H(0:k,0:k)^-1 g(0:k) (upper triangular), one thread
__device__ void backsolve_body(int k, int m, const double2* __restrict__ H, const double2* __restrict__ g,
                            double2* __restrict__ y) {
  for (int i = k - 1; i >= 0; --i) {
    double2 acc = g[i];
    for (int l = i + 1; l < k; ++l) acc = csub(acc, cmul(H[i * m + l], y[l]));
    const double2 d = H[i * m + i];
    const double den = d.x * d.x + d.y * d.y;
    // a zero pivot (a direction the preconditioner annihilated) contributes nothing
    y[i] = den > 0.0 ? cmul(acc, make_double2(d.x / den, -d.y / den)) : make_double2(0.0, 0.0);
  }
}

// the same with the triangle staged in LDS first (packed rows, loaded by
// the whole workgroup), so the serial recurrence reads no global memory
__global__ __launch_bounds__(64) void k_backsolve(int k, int m, const double2* __restrict__ H,
                                                  const double2* __restrict__ g, double2* __restrict__ y) {
  __shared__ double2 T[kMaxRestart * (kMaxRestart + 1) / 2];
  __shared__ double2 gs[kMaxRestart], ys[kMaxRestart];
  // row i of the triangle (columns i..k-1) starts at i k - i (i - 1) / 2
  for (int i = 0; i < k; ++i)
    for (int l = i + threadIdx.x; l < k; l += blockDim.x) T[i * k - i * (i - 1) / 2 + (l - i)] = H[i * m + l];
  for (int i = threadIdx.x; i < k; i += blockDim.x) gs[i] = g[i];
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int i = k - 1; i >= 0; --i) {
    const double2* Ti = T + (i * k - i * (i - 1) / 2);
    double2 acc = gs[i];
    for (int l = i + 1; l < k; ++l) acc = csub(acc, cmul(Ti[l - i], ys[l]));
    const double2 d = Ti[0];
    const double den = d.x * d.x + d.y * d.y;
    // a zero pivot (a direction the preconditioner annihilated) contributes nothing
    ys[i] = den > 0.0 ? cmul(acc, make_double2(d.x / den, -d.y / den)) : make_double2(0.0, 0.0);
    y[i] = ys[i];
  }
}

__global__ void k_backsolve_b(const int* __restrict__ ks, int m, const double2* __restrict__ H,
                              const double2* __restrict__ g, double2* __restrict__ y, int64_t ystride,
                              const int* __restrict__ active) {
  const int z = blockIdx.z;
  if (threadIdx.x != 0 || (active && !active[z])) return;
  backsolve_body(ks[z], m, H + (int64_t)z * (m + 1) * m, g + z * (m + 2), y + z * ystride);
}

// ---- batched right-hand sides: the matrix / block inverses are read once
// per launch for up to kBatchChunk systems (vectors of system r at r * ld).

// z_r = Minv r_r for the active systems, one wavefront per block.
template <class T, class MT, class RT>
__global__ __launch_bounds__(kThreads) void k_block_apply_b(int64_t nb, const int* __restrict__ blk_ptr,
                                                            const int* __restrict__ blk_dofs,
                                                            const MT* __restrict__ minv, int nrhs, int64_t rstride,
                                                            const RT* __restrict__ r, int64_t zstride,
                                                            T* __restrict__ z, const int* __restrict__ active) {
  __shared__ T rl[4][kBatchChunk][kMaxBlock];
  const int w = threadIdx.x >> 6, i = threadIdx.x & 63;
  const int64_t k = (int64_t)blockIdx.x * 4 + w;
  int b0 = 0, sz = 0, dof = -1;
  if (k < nb) {
    b0 = blk_ptr[k];
    sz = blk_ptr[k + 1] - b0;
    if (i < sz) dof = blk_dofs[b0 + i];
  }
  const MT* Mk = minv + k * kMaxBlock * kMaxBlock;
  for (int c0 = 0; c0 < nrhs; c0 += kBatchChunk) {
    const int cn = min(kBatchChunk, nrhs - c0);
#pragma unroll
    for (int q = 0; q < kBatchChunk; ++q) {
      const bool on = q < cn && dof >= 0 && (!active || active[c0 + q]);
      rl[w][q][i] = on ? st2<T>(ld2(r[(int64_t)(c0 + q) * rstride + dof])) : zero2<T>();
    }
    __syncthreads();
    if (dof >= 0) {
      T acc[kBatchChunk];
#pragma unroll
      for (int q = 0; q < kBatchChunk; ++q) acc[q] = zero2<T>();
      for (int j = 0; j < sz; ++j) {
        const T mij = as_vec(ld_stream(Mk + j * kMaxBlock + i));
#pragma unroll
        for (int q = 0; q < kBatchChunk; ++q)
          if (q < cn) acc[q] = cfmaT(mij, rl[w][q][j], acc[q]);
      }
#pragma unroll
      for (int q = 0; q < kBatchChunk; ++q)
        if (q < cn && (!active || active[c0 + q])) z[(int64_t)(c0 + q) * zstride + dof] = acc[q];
    }
    __syncthreads();
  }
}

// Batched block-Jacobi apply on the matrix cores, for complex-half
// inverses and complex-half (scaled) inputs: per 64-DOF block and chunk of 8
// systems, Z = M R with M = Mr + i Mi (64 x 64) and R = Rr + i Ri (64 x 8)
// is the real product [Zr Zi] = Mr [Rr Ri] + Mi [-Ri Rr] (64 x 64 times
// 64 x 16), eight v_mfma_f32_16x16x16_f16 per 16-row tile.  Half x half
// products are exact in float32 and the sums are float32, as in
// k_block_apply_b; only the order of the sums differs.  One wavefront per
// block, 4 blocks per workgroup; R is staged in LDS.  Fragment layout of
// v_mfma_f32_16x16x16_f16: lane l supplies A(l % 16, 4 (l / 16) + u) and
// B(4 (l / 16) + u, l % 16), u = 0..3, and receives D(4 (l / 16) + u, l % 16).
// The inverses' columns past the block size are zero (k_block_invert).
typedef _Float16 h4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(kThreads) void k_block_apply_mfma(int64_t nb, const int* __restrict__ blk_ptr,
                                                               const int* __restrict__ blk_dofs,
                                                               const uint32_t* __restrict__ minv, int nrhs,
                                                               int64_t rstride, const hbasis* __restrict__ r,
                                                               int64_t zstride, float2* __restrict__ z,
                                                               const int* __restrict__ active, int interleave) {
  __shared__ uint32_t rl[4][kBatchChunk][kMaxBlock];
  __shared__ int dl[4][kMaxBlock];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int64_t k = (int64_t)blockIdx.x * 4 + w;
  int b0 = 0, sz = 0;
  if (k < nb) {
    b0 = blk_ptr[k];
    sz = blk_ptr[k + 1] - b0;
  }
  dl[w][l] = l < sz ? blk_dofs[b0 + l] : -1;
  const uint32_t* Mk = minv + (k < nb ? k : 0) * kMaxBlock * kMaxBlock;
  const int n = l & 15, q = n & 7, kq = (l >> 4) * 4;
  const bool imag_col = n >= 8;
  // the block's A fragments (16 KB per wavefront) are issued before the
  // right-hand sides are gathered and stay in registers for every chunk
  uint32_t mw[4][4][4];
#pragma unroll
  for (int ks = 0; ks < 4; ++ks)
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int u = 0; u < 4; ++u) mw[ks][t][u] = ld_stream(Mk + (ks * 16 + kq + u) * kMaxBlock + t * 16 + n);
  for (int c0 = 0; c0 < nrhs; c0 += kBatchChunk) {
    const int cn = min(kBatchChunk, nrhs - c0);
    __syncthreads();   // dl written / previous chunk's rl consumed
#pragma unroll
    for (int s = 0; s < kBatchChunk; ++s) {
      const int dof = dl[w][l];
      const bool on = s < cn && dof >= 0 && (!active || active[c0 + s]);
      rl[w][s][l] = on ? r[(int64_t)(c0 + s) * rstride + dof].b : 0u;
    }
    __syncthreads();
    if (k >= nb) continue;
    f4_t acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = (f4_t){0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int k0 = ks * 16;
      h4_t b1, b2;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const uint32_t x = rl[w][q][k0 + kq + u];
        const _Float16 re = __builtin_bit_cast(_Float16, (unsigned short)(x & 0xffffu));
        const _Float16 im = __builtin_bit_cast(_Float16, (unsigned short)(x >> 16));
        b1[u] = imag_col ? im : re;
        b2[u] = imag_col ? re : -im;
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        h4_t ar, ai;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const uint32_t m = mw[ks][t][u];
          ar[u] = __builtin_bit_cast(_Float16, (unsigned short)(m & 0xffffu));
          ai[u] = __builtin_bit_cast(_Float16, (unsigned short)(m >> 16));
        }
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x16f16(ar, b1, acc[t], 0, 0, 0);
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x16f16(ai, b2, acc[t], 0, 0, 0);
      }
    }
    // lane n < 8 holds the real parts of system n, lane n + 8 the imaginary
    // parts: pair them, undo the inputs' 2^14 scale
    constexpr float us = 1.0f / 16384.0f;
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const float other = __shfl_xor(acc[t][u], 8, 64);
        const int row = t * 16 + kq + u;
        const int dof = dl[w][row];
        if (!imag_col && q < cn && dof >= 0 && (!active || active[c0 + q])) {
          // interleaved: the chunk's 8 systems side by side per row (see k_spmv_b_il)
          const int64_t o = interleave ? ((int64_t)(c0 / kBatchChunk) * zstride + dof) * kBatchChunk + q
                                       : (int64_t)(c0 + q) * zstride + dof;
          z[o] = make_float2(acc[t][u] * us, other * us);
        }
      }
  }
}

// y_r = M~ x_r (penalty-free operator), or y_r = b_r - M~ x_r if b; 8 lanes per row.
template <class T>
__global__ __launch_bounds__(kThreads) void k_spmv_b(int64_t n, const int* __restrict__ rowptr,
                                                     const int* __restrict__ col, const T* __restrict__ val, int nrhs,
                                                     int64_t ld, const T* __restrict__ x, const T* __restrict__ b,
                                                     T* __restrict__ y, const int* __restrict__ active) {
  const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kLanes;
  const int lane = threadIdx.x % kLanes;
  for (int c0 = 0; c0 < nrhs; c0 += kBatchChunk) {
    const int cn = min(kBatchChunk, nrhs - c0);
    bool on[kBatchChunk];
    T acc[kBatchChunk];
#pragma unroll
    for (int q = 0; q < kBatchChunk; ++q) {
      on[q] = q < cn && (!active || active[c0 + q]);
      acc[q] = zero2<T>();
    }
    if (row < n) {
      for (int p = rowptr[row] + lane; p < rowptr[row + 1]; p += kLanes) {
        const T v = val[p];
        const int c = col[p];
#pragma unroll
        for (int q = 0; q < kBatchChunk; ++q)
          if (on[q]) acc[q] = cfmaT(v, x[(int64_t)(c0 + q) * ld + c], acc[q]);
      }
    }
#pragma unroll
    for (int q = 0; q < kBatchChunk; ++q)
      for (int o = kLanes / 2; o > 0; o >>= 1) {
        acc[q].x += __shfl_xor(acc[q].x, o, kLanes);
        acc[q].y += __shfl_xor(acc[q].y, o, kLanes);
      }
    if (row < n && lane == 0) {
#pragma unroll
      for (int q = 0; q < kBatchChunk; ++q)
        if (on[q]) {
          const int64_t o = (int64_t)(c0 + q) * ld + row;
          y[o] = b ? st2<T>(csub(ld2(b[o]), ld2(acc[q]))) : acc[q];
        }
    }
  }
}

// ---- several frequencies in one batch.  On the penalty-free operator every
// stored entry is P + c(omega) Q with P, Q real: c = -i omega on the A-A
// entries (K_nu - i omega M_sigma), c = i / omega on the V-V entries
// ((i/omega) S_sigma), and Q = 0 on the A-V couplings (-B_sigma), so the
// row class decides c.  k_factor_pq recovers {P, Q} from one operator's
// equilibrated complex128 values (val = s_i s_j (P + c0 Q)); k_spmv_mf reads
// the factored matrix once for a chunk of systems of different frequencies:
// y_r = s_r (P + c_r Q) u_r with u_r = s_r x_r (k_scale_sys), s_r the
// equilibration of system r's operator; 8 lanes per row, complex64.
__global__ __launch_bounds__(kThreads) void k_factor_pq(int64_t n, int64_t ne, const int* __restrict__ rowptr,
                                                        const int* __restrict__ col, const double2* __restrict__ val,
                                                        const double* __restrict__ s, double omega,
                                                        float2* __restrict__ pq) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double si = s[i];
  for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) {
    const double d = 1.0 / (si * s[col[p]]);
    const double re = val[p].x * d, im = val[p].y * d;
    pq[p] = make_float2((float)re, (float)(i < ne ? -im / omega : im * omega));
  }
}

__global__ __launch_bounds__(kThreads) void k_scale_sys(int64_t n, const float2* __restrict__ x, int64_t ld,
                                                        const mf_sys* __restrict__ sys, float2* __restrict__ u,
                                                        const int* __restrict__ active) {
  const int z = blockIdx.z;
  if (active && !active[z]) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float f = (float)sys[z].s[i];
  const float2 v = x[(int64_t)z * ld + i];
  u[(int64_t)z * ld + i] = make_float2(v.x * f, v.y * f);
}

__global__ __launch_bounds__(kThreads) void k_spmv_mf(int64_t n, int64_t ne, const int* __restrict__ rowptr,
                                                      const int* __restrict__ col, const float2* __restrict__ pq,
                                                      int nrhs, int64_t ld, const float2* __restrict__ u,
                                                      float2* __restrict__ y, const mf_sys* __restrict__ sys,
                                                      const int* __restrict__ active) {
  const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kLanes;
  const int lane = threadIdx.x % kLanes;
  for (int c0 = 0; c0 < nrhs; c0 += kBatchChunk) {
    const int cn = min(kBatchChunk, nrhs - c0);
    bool on[kBatchChunk];
    float2 ap[kBatchChunk], aq[kBatchChunk];
#pragma unroll
    for (int q = 0; q < kBatchChunk; ++q) {
      on[q] = q < cn && (!active || active[c0 + q]);
      ap[q] = aq[q] = make_float2(0.f, 0.f);
    }
    if (row < n) {
      for (int p = rowptr[row] + lane; p < rowptr[row + 1]; p += kLanes) {
        const float2 v = pq[p];
        const int c = col[p];
#pragma unroll
        for (int q = 0; q < kBatchChunk; ++q)
          if (on[q]) {
            const float2 x = u[(int64_t)(c0 + q) * ld + c];
            ap[q].x = fmaf(v.x, x.x, ap[q].x);
            ap[q].y = fmaf(v.x, x.y, ap[q].y);
            aq[q].x = fmaf(v.y, x.x, aq[q].x);
            aq[q].y = fmaf(v.y, x.y, aq[q].y);
          }
      }
    }
#pragma unroll
    for (int q = 0; q < kBatchChunk; ++q)
      for (int o = kLanes / 2; o > 0; o >>= 1) {
        ap[q].x += __shfl_xor(ap[q].x, o, kLanes);
        ap[q].y += __shfl_xor(ap[q].y, o, kLanes);
        aq[q].x += __shfl_xor(aq[q].x, o, kLanes);
        aq[q].y += __shfl_xor(aq[q].y, o, kLanes);
      }
    if (row < n && lane == 0) {
#pragma unroll
      for (int q = 0; q < kBatchChunk; ++q)
        if (on[q]) {
          const mf_sys& sq = sys[c0 + q];
          const float w = row < ne ? sq.w_a : sq.w_v, f = (float)sq.s[row];
          // (P u) + i w (Q u), then the row scaling
          y[(int64_t)(c0 + q) * ld + row] =
              make_float2((ap[q].x - w * aq[q].y) * f, (ap[q].y + w * aq[q].x) * f);
        }
    }
  }
}

// k_spmv_b for complex64 with the input interleaved per chunk of 8 systems:
// x of system c0 + q at row c is xil[((c0 / 8) ld + c) 8 + q], so one
// 64-byte load per matrix entry serves the whole chunk (the systems' own
// vectors would be 8 separate gathers).  Output per system at stride ld.
__global__ __launch_bounds__(kThreads) void k_spmv_b_il(int64_t n, const int* __restrict__ rowptr,
                                                        const int* __restrict__ col, const float2* __restrict__ val,
                                                        int nrhs, int64_t ld, const float2* __restrict__ xil,
                                                        float2* __restrict__ y, const int* __restrict__ active) {
  static_assert(kBatchChunk == 8, "four 16-byte loads per entry");
  const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kLanes;
  const int lane = threadIdx.x % kLanes;
  for (int c0 = 0; c0 < nrhs; c0 += kBatchChunk) {
    const int cn = min(kBatchChunk, nrhs - c0);
    const float4* __restrict__ xc = reinterpret_cast<const float4*>(xil + (int64_t)(c0 / kBatchChunk) * ld * kBatchChunk);
    float2 acc[kBatchChunk];
#pragma unroll
    for (int q = 0; q < kBatchChunk; ++q) acc[q] = make_float2(0.f, 0.f);
    if (row < n) {
      for (int p = rowptr[row] + lane; p < rowptr[row + 1]; p += kLanes) {
        const float2 v = val[p];
        const float4* xp = xc + (int64_t)col[p] * (kBatchChunk / 2);
        const float4 a[4] = {xp[0], xp[1], xp[2], xp[3]};
#pragma unroll
        for (int h = 0; h < 4; ++h) {
          acc[2 * h] = cfmaT(v, make_float2(a[h].x, a[h].y), acc[2 * h]);
          acc[2 * h + 1] = cfmaT(v, make_float2(a[h].z, a[h].w), acc[2 * h + 1]);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < kBatchChunk; ++q)
      for (int o = kLanes / 2; o > 0; o >>= 1) {
        acc[q].x += __shfl_xor(acc[q].x, o, kLanes);
        acc[q].y += __shfl_xor(acc[q].y, o, kLanes);
      }
    if (row < n && lane == 0) {
#pragma unroll
      for (int q = 0; q < kBatchChunk; ++q)
        if (q < cn && (!active || active[c0 + q])) y[(int64_t)(c0 + q) * ld + row] = acc[q];
    }
  }
}

// out_r = (T) in_r
template <class T>
__global__ __launch_bounds__(kThreads) void k_convert_b(int64_t n, const double2* __restrict__ in, int64_t istride,
                                                        T* __restrict__ out, int64_t ostride) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[blockIdx.z * ostride + i] = st2<T>(in[blockIdx.z * istride + i]);
}

// out = (complex64) in
__global__ __launch_bounds__(kThreads) void k_to_c64(int64_t n, const double2* __restrict__ in,
                                                     float2* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = make_float2((float)in[i].x, (float)in[i].y);
}

__global__ __launch_bounds__(kThreads) void k_diag_scale(int64_t n, const double2* __restrict__ in,
                                                         const double* __restrict__ s, int divide,
                                                         double2* __restrict__ out, int64_t istride, int64_t ostride) {
  in += blockIdx.z * istride;
  out += blockIdx.z * ostride;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double f = divide ? 1.0 / s[i] : s[i];
  const double2 v = in[i];
  out[i] = make_double2(v.x * f, v.y * f);
}

__global__ __launch_bounds__(kThreads) void k_zero(int64_t n, double2* __restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = make_double2(0.0, 0.0);
}

// One workgroup per conductor component: mass-weighted mean of V over it.
__global__ __launch_bounds__(kThreads) void k_vmean(int64_t nc, const int* __restrict__ comp,
                                                    const double* __restrict__ lumped, const double2* __restrict__ V,
                                                    double2* __restrict__ mean) {
  __shared__ double sh[4];
  const int c = blockIdx.x;
  double re = 0.0, im = 0.0, den = 0.0;
  for (int64_t i = threadIdx.x; i < nc; i += blockDim.x)
    if (comp[i] == c) {
      const double m = lumped[i];
      re = fma(m, V[i].x, re);
      im = fma(m, V[i].y, im);
      den += m;
    }
  re = block_sum(re, sh);
  im = block_sum(im, sh);
  den = block_sum(den, sh);
  if (threadIdx.x == 0) mean[c] = make_double2(re / den, im / den);
}

__global__ __launch_bounds__(kThreads) void k_vmean_sub(int64_t nc, const int* __restrict__ comp,
                                                        const double2* __restrict__ mean, double2* __restrict__ V) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nc) V[i] = csub(V[i], mean[comp[i]]);
}

// partial sums of a_i * b_i (unconjugated)
__global__ __launch_bounds__(kThreads) void k_udot_partial(int64_t n, const double2* __restrict__ a,
                                                           const double2* __restrict__ b,
                                                           double2* __restrict__ partial) {
  __shared__ double sh[4];
  double2 acc = make_double2(0.0, 0.0);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    acc = cfma(a[i], b[i], acc);
  const double re = block_sum(acc.x, sh);
  const double im = block_sum(acc.y, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = make_double2(re, im);
}

// Per-tetrahedron fields of one solution x = (A, V) of a configuration whose
// conductor-node numbering is vmap (-1: no V there, taken as 0).  The lowest-
// order edge field E_h = i w A_h + grad V_h on K is sum_a lambda_a u_a with
// u_a = sum_b c_ab grad(lambda_b), c_ab = -c_ba the local edge coefficient of
// the edge (a, b) (Whitney functions lambda_a grad lambda_b - lambda_b grad
// lambda_a); grad V_h lies in the same space with c_ab = V_b - V_a.  curl A_h
// = sum 2 A_ab grad(lambda_a) x grad(lambda_b).
__device__ __forceinline__ void tet_fields(const double g[4][3], const int e6[6], double sg[6], const int n4[4],
                                           const double2* __restrict__ x, int64_t ne, const int* __restrict__ vmap,
                                           double omega, double2 u[4][3], double2 cu[3]) {
  constexpr int ea[6] = {0, 0, 0, 1, 1, 2};
  constexpr int eb[6] = {1, 2, 3, 2, 3, 3};
  double2 v[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int c = vmap[n4[a]];
    v[a] = c >= 0 ? x[ne + c] : make_double2(0.0, 0.0);
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int j = 0; j < 3; ++j) u[a][j] = make_double2(0.0, 0.0);
#pragma unroll
  for (int j = 0; j < 3; ++j) cu[j] = make_double2(0.0, 0.0);
#pragma unroll
  for (int l = 0; l < 6; ++l) {
    const int a = ea[l], b = eb[l];
    const double2 A = x[e6[l]];
    const double2 Al = make_double2(sg[l] * A.x, sg[l] * A.y);          // local-orientation A
    // c_ab = i w A_ab + V_b - V_a
    const double2 c = make_double2(-omega * Al.y + v[b].x - v[a].x, omega * Al.x + v[b].y - v[a].y);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      u[a][j] = rfma(g[b][j], c, u[a][j]);
      u[b][j] = rfma(-g[a][j], c, u[b][j]);
    }
    const double cx = g[a][1] * g[b][2] - g[a][2] * g[b][1];
    const double cy = g[a][2] * g[b][0] - g[a][0] * g[b][2];
    const double cz = g[a][0] * g[b][1] - g[a][1] * g[b][0];
    cu[0] = rfma(2.0 * cx, Al, cu[0]);
    cu[1] = rfma(2.0 * cy, Al, cu[1]);
    cu[2] = rfma(2.0 * cz, Al, cu[2]);
  }
}

// out[l] partials: sum over tetrahedra whose (nu, sigma) differ between the
// two configurations of  i w dnu |K| curl A_d . curl A_0  -  dsig int_K E_d . E_0,
// with int_K lambda_a lambda_b = |K| (1 + delta_ab) / 20.  Grid-stride over
// tetrahedra; most of them are skipped after reading their region.
__global__ __launch_bounds__(kThreads) void k_dz_volume(
    int64_t nt, const double* __restrict__ xyz, const int* __restrict__ tet, const int* __restrict__ region,
    const uint8_t* __restrict__ signbits, const int* __restrict__ tet2edge, const double* __restrict__ nu_d,
    const double* __restrict__ sig_d, const double* __restrict__ nu_0, const double* __restrict__ sig_0, double omega,
    int64_t ne, const double2* __restrict__ xd, const int* __restrict__ vmap_d, int nl, const double2* __restrict__ x0,
    int64_t ld0, const int* __restrict__ vmap_0, double2* __restrict__ partial) {
  __shared__ double sh[4];
  double2 acc[kMaxDzCols];
#pragma unroll
  for (int l = 0; l < kMaxDzCols; ++l) acc[l] = make_double2(0.0, 0.0);
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nt; t += (int64_t)gridDim.x * blockDim.x) {
    const int r = region[t];
    const double dnu = nu_d[r] - nu_0[r], dsig = sig_d[r] - sig_0[r];
    if (dnu == 0.0 && dsig == 0.0) continue;
    const int4 nd = reinterpret_cast<const int4*>(tet)[t];
    const int n4[4] = {nd.x, nd.y, nd.z, nd.w};
    double p[4][3];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int j = 0; j < 3; ++j) p[k][j] = xyz[3 * (int64_t)n4[k] + j];
    double e1[3], e2[3], e3[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      e1[j] = p[1][j] - p[0][j];
      e2[j] = p[2][j] - p[0][j];
      e3[j] = p[3][j] - p[0][j];
    }
    const double c23[3] = {e2[1] * e3[2] - e2[2] * e3[1], e2[2] * e3[0] - e2[0] * e3[2], e2[0] * e3[1] - e2[1] * e3[0]};
    const double c31[3] = {e3[1] * e1[2] - e3[2] * e1[1], e3[2] * e1[0] - e3[0] * e1[2], e3[0] * e1[1] - e3[1] * e1[0]};
    const double c12[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
    const double det = e1[0] * c23[0] + e1[1] * c23[1] + e1[2] * c23[2];
    const double id = 1.0 / det;
    const double vol = fabs(det) * (1.0 / 6.0);
    double g[4][3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      g[1][j] = c23[j] * id;
      g[2][j] = c31[j] * id;
      g[3][j] = c12[j] * id;
      g[0][j] = -(g[1][j] + g[2][j] + g[3][j]);
    }
    int e6[6];
    double sg[6];
    const uint8_t sb = signbits[t];
#pragma unroll
    for (int l = 0; l < 6; ++l) {
      e6[l] = tet2edge[6 * t + l];
      sg[l] = ((sb >> l) & 1) ? -1.0 : 1.0;
    }
    double2 ud[4][3], cd[3];
    tet_fields(g, e6, sg, n4, xd, ne, vmap_d, omega, ud, cd);
    double2 sd[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) sd[j] = cadd(cadd(ud[0][j], ud[1][j]), cadd(ud[2][j], ud[3][j]));
#pragma unroll
    for (int l = 0; l < kMaxDzCols; ++l) {
      if (l >= nl) break;
      double2 u0[4][3], c0[3];
      tet_fields(g, e6, sg, n4, x0 + (int64_t)l * ld0, ne, vmap_0, omega, u0, c0);
      double2 ee = make_double2(0.0, 0.0), cc = make_double2(0.0, 0.0);
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const double2 s0 = cadd(cadd(u0[0][j], u0[1][j]), cadd(u0[2][j], u0[3][j]));
        ee = cfma(sd[j], s0, ee);
#pragma unroll
        for (int a = 0; a < 4; ++a) ee = cfma(ud[a][j], u0[a][j], ee);
        cc = cfma(cd[j], c0[j], cc);
      }
      // i w dnu |K| cc - dsig |K|/20 ee
      const double fe = -dsig * vol * (1.0 / 20.0), fc = omega * dnu * vol;
      acc[l].x += fe * ee.x - fc * cc.y;
      acc[l].y += fe * ee.y + fc * cc.x;
    }
  }
#pragma unroll
  for (int l = 0; l < kMaxDzCols; ++l) {
    if (l >= nl) break;
    const double re = block_sum(acc[l].x, sh);
    const double im = block_sum(acc[l].y, sh);
    if (threadIdx.x == 0) partial[(int64_t)l * gridDim.x + blockIdx.x] = make_double2(re, im);
  }
}

__global__ __launch_bounds__(kThreads) void k_edge_field(int64_t ne, const int* __restrict__ edge_v,
                                                         const double2* __restrict__ x, double omega,
                                                         double2* __restrict__ E) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  const double2 a = x[e];
  double2 v = make_double2(-omega * a.y, omega * a.x);
  const int lo = edge_v[2 * e], hi = edge_v[2 * e + 1];
  if (lo >= 0 && hi >= 0) v = cadd(v, csub(x[ne + hi], x[ne + lo]));
  E[e] = v;
}

}  // namespace

// ---------------------------------------------------------------------------
// launch wrappers
// ---------------------------------------------------------------------------
void launch_element(int64_t nt, int64_t nct, const double* xyz, const int* tet, const int* region,
                    const uint8_t* signbits, const int* cidx, const double* nu_reg, const double* sig_reg,
                    double omega, double delta_v, double2* ebuf, double* wbuf, double* vol4, hipStream_t st) {
  k_element<<<blocks_for(nt), kThreads, 0, st>>>(nt, nct, xyz, tet, region, signbits, cidx, nu_reg, sig_reg, omega,
                                                 delta_v, ebuf, wbuf, vol4);
}
void launch_gather_c(int64_t n, const int* ptr, const int* list, const double2* buf, double2* out, hipStream_t st) {
  k_gather_c<<<blocks_for(n), kThreads, 0, st>>>(n, ptr, list, buf, out);
}
void launch_gather_r(int64_t n, const int* ptr, const int* list, const double* buf, double* out, hipStream_t st) {
  k_gather_r<<<blocks_for(n), kThreads, 0, st>>>(n, ptr, list, buf, out);
}
void launch_gather_r2c(int64_t n, int64_t ntot, const int* ptr, const int* list, const double* buf, double2* out,
                       hipStream_t st) {
  k_gather_r2c<<<blocks_for(ntot), kThreads, 0, st>>>(n, ntot, ptr, list, buf, out);
}
void launch_permute_r(int64_t n, const int* perm, const double* in, double* out, hipStream_t st) {
  k_permute_r<<<blocks_for(n), kThreads, 0, st>>>(n, perm, in, out);
}
void launch_d0tau(int64_t nv, const double* d0, double tau, double* d0tau, hipStream_t st) {
  k_d0tau<<<blocks_for(nv), kThreads, 0, st>>>(nv, d0, tau, d0tau);
}
void launch_equilibrate(int64_t n, int64_t ne, const int* diagpos, const double2* val, const int* wrowptr,
                        const int* wcol, const double* wval, const double* d0tau, double* s, int* status,
                        hipStream_t st) {
  k_equilibrate<<<blocks_for(n), kThreads, 0, st>>>(n, ne, diagpos, val, wrowptr, wcol, wval, d0tau, s, status);
}
void launch_scale_rows(int64_t n, const int* rowptr, const int* col, double2* val, const double* s, hipStream_t st) {
  k_scale_rows<<<blocks_for(n), kThreads, 0, st>>>(n, rowptr, col, val, s);
}
void launch_scale_w(int64_t ne, const int* wrowptr, double* wval, const double* s, hipStream_t st) {
  k_scale_w<<<blocks_for(ne), kThreads, 0, st>>>(ne, wrowptr, wval, s);
}
void launch_block_invert(int64_t nb, const int* blk_ptr, const int* blk_dofs, const int* blk_of, const int* loc_of,
                         const int* rowptr, const int* col, const double2* val, int64_t ne, const int* wrowptr,
                         const int* wcol, const double* wval, const double* d0tau, double* gscr, double2* minv,
                         int* status, hipStream_t st) {
  if (nb <= 0) return;
  k_block_gauge<<<(unsigned)nb, kMaxBlock, 0, st>>>(blk_ptr, blk_dofs, ne, wrowptr, wcol, wval, d0tau, gscr);
  k_block_invert<<<(unsigned)nb, kMaxBlock, 0, st>>>(blk_ptr, blk_dofs, blk_of, loc_of, rowptr, col, val, gscr, minv,
                                                      status);
}
void launch_rhs_elem(int64_t nt, const double* xyz, const int* tet, const uint8_t* signbits, const double* J,
                     double* rbuf, hipStream_t st) {
  k_rhs_elem<<<blocks_for(nt), kThreads, 0, st>>>(nt, xyz, tet, signbits, J, rbuf);
}
void launch_wt(int64_t nv, const int* wtrowptr, const int* wtcol, const double* wtval, const double* d0tau,
               const double2* x, double2* t, hipStream_t st) {
  k_wt<<<blocks_for(nv * kLanes), kThreads, 0, st>>>(nv, wtrowptr, wtcol, wtval, d0tau, x, t);
}
template <class T>
void launch_spmv(int64_t ns, const int* sptr, const int* srow, const int* scol, const T* sval, int64_t ne,
                 const int* wrowptr, const int* wcol, const double* wval, const double2* t, const T* x,
                 const double2* b, T* y, hipStream_t st, int grid, int schedule, const int* xcd_groups,
                 const int* scplx) {
  const unsigned full = blocks_for(ns * kSellC);
  unsigned g = grid > 0 && (unsigned)grid < full ? (unsigned)grid : full;
  if (schedule && (g < (unsigned)kXcds || !xcd_groups)) schedule = 0;
  k_spmv_sell<T><<<g, kThreads, 0, st>>>(ns, sptr, srow, scol, sval, x, b, y, schedule, xcd_groups, scplx);
  if (wrowptr)
    k_gauge_add<T><<<blocks_for(ne * kLanes), kThreads, 0, st>>>(ne, wrowptr, wcol, wval, t, b ? -1.0 : 1.0, y);
}
int spmv_full_grid(int64_t ns) { return (int)blocks_for(ns * kSellC); }
void launch_sell_gather(int64_t tot, int64_t ns, const int* sptr, const int* src, const double2* val, double2* sval,
                        float2* sval32, int* scplx, hipStream_t st) {
  k_sell_values<<<blocks_for(ns * kSellC), kThreads, 0, st>>>(ns, sptr, src, val, sval, sval32, scplx);
}
template <class T, class MT, class RT>
void launch_block_apply(int64_t nb, const int* blk_ptr, const int* blk_dofs, const MT* minv, const RT* r, T* z,
                        hipStream_t st) {
  k_block_apply<T, MT, RT><<<blocks_for(nb, 4), kThreads, 0, st>>>(nb, blk_ptr, blk_dofs, minv, r, z);
}
int mdot2_parts(int64_t n) {
  // tiles of the widest row groups (4 rows per thread); every workgroup gets
  // the same number of tiles (the smaller groups split each tile in two)
  const int64_t tiles = (n + 4 * kThreads - 1) / (4 * kThreads);
  const int64_t per = (tiles + kDot2MaxBlocks - 1) / kDot2MaxBlocks;
  const int64_t parts = per > 0 ? (tiles + per - 1) / per : 1;
  return (int)(parts > 0 ? parts : 1);
}
int mdot_parts(int64_t n) { return (int)((n + 2 * kThreads - 1) / (2 * kThreads)); }
template <class T>
void launch_mdot(int64_t n, const T* V, int64_t ldv, int q, const T* w, double2* partial, hipStream_t st,
                 int want_norm, const int* flag) {
  dim3 grid(mdot_parts(n), (q + 7) / 8);
  k_mdot<T><<<grid, kThreads, 0, st>>>(n, V, ldv, q, w, partial, want_norm, flag, 0, 0, 0, nullptr);
}
void launch_reduce_cols(int q, int nparts, const double2* partial, double2* out, hipStream_t st, const int* flag) {
  k_reduce_cols<<<q, kThreads, 0, st>>>(partial, nparts, out, flag, 0, 0, nullptr);
}
template <class T>
void launch_norm2(int64_t n, const T* w, double* partial, double* out_norm, hipStream_t st) {
  k_norm2_partial<T><<<kRedBlocks, kThreads, 0, st>>>(n, w, partial, 0, nullptr);
  k_norm2_final<<<1, kThreads, 0, st>>>(partial, out_norm, nullptr, nullptr);
}
// every vector 16-byte aligned and the system strides multiples of R rows
int vec_ok(int R, const void* a, const void* b, int64_t sa, int64_t sb) {
  return (((uintptr_t)a | (uintptr_t)b) & 15) == 0 && sa % R == 0 && sb % R == 0;
}
template <class Ti, class To>
void launch_scale_by_inv(int64_t n, const Ti* w, const double* norm, To* v, hipStream_t st) {
  constexpr int R = scale_rows<Ti, To>();
  k_scale_by_inv<Ti, To><<<blocks_for((n + R - 1) / R), kThreads, 0, st>>>(n, w, norm, v, 0, 0, nullptr,
                                                                           vec_ok(R, w, v, 0, 0));
}
template <class Ti, class To>
void launch_scale_host(int64_t n, const Ti* w, double a, To* v, hipStream_t st) {
  k_scale_host<Ti, To><<<blocks_for(n), kThreads, 0, st>>>(n, w, a, v);
}
template <class VT, class T>
void launch_combine(int64_t n, const VT* V, int64_t ldv, int q, const double2* y, T* u, hipStream_t st) {
  k_combine<VT, T><<<blocks_for(n), kThreads, 0, st>>>(n, V, ldv, q, y, u, 0, 0, 0, nullptr, nullptr);
}
template <class T>
void launch_axpy(int64_t n, const T* z, double2* x, hipStream_t st) {
  k_axpy<T><<<blocks_for(n), kThreads, 0, st>>>(n, z, x, 0, 0, nullptr);
}
// whether the row-group accesses of k_mdot2 / k_dcgs_update may be used:
// every vector of every system 16-byte aligned
template <class VT>
int rows_aligned(const void* V, const void* v, const void* w, int64_t ldv, int64_t vstride, int64_t wstride) {
  constexpr int R = rows_of<VT>::R;
  return (((uintptr_t)V | (uintptr_t)v | (uintptr_t)w) & 15) == 0 && ldv % R == 0 && vstride % R == 0 &&
         wstride % R == 0;
}
template <class VT, class T>
void launch_mdot2(int64_t n, const VT* V, int64_t ldv, int q, const VT* v, const T* w, double2* partial,
                  hipStream_t st) {
  dim3 grid(mdot2_parts(n), q > 0 ? (q + 7) / 8 : 1);
  k_mdot2<VT, T><<<grid, kThreads, 0, st>>>(n, V, ldv, q, v, w, partial, 0, 0, 0, nullptr,
                                            rows_aligned<VT>(V, v, w, ldv, 0, 0));
}
void launch_dcgs_coef(int j, int m, const double2* dots, double2* Hraw, const double* tnorm, double2* coef,
                      double2* H, double* cs, double2* sn, double2* g, double beta, double bnorm, double* est,
                      double2* Sall, double* rhoall, hipStream_t st) {
  k_dcgs_coef<<<1, 64, 0, st>>>(j, m, dots, Hraw, tnorm, coef, H, cs, sn, g, beta, bnorm, est, Sall, rhoall,
                                nullptr, nullptr, 0, nullptr);
}
void launch_dcgs_coef_dev(int j, int m, const double2* dots, double2* Hraw, const double* tnorm, double2* coef,
                          double2* H, double* cs, double2* sn, double2* g, const double* beta, const double* bnorm,
                          double* est, double2* Sall, double* rhoall, hipStream_t st) {
  k_dcgs_coef<<<1, 64, 0, st>>>(j, m, dots, Hraw, tnorm, coef, H, cs, sn, g, 0.0, 0.0, est, Sall, rhoall, beta,
                                bnorm, 0, nullptr);
}
__global__ void k_set2(double a, double b, double* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    out[0] = a;
    out[1] = b;
  }
}
void launch_set2(double a, double b, double* out, hipStream_t st) { k_set2<<<1, 64, 0, st>>>(a, b, out); }
// Flexible cycles: the basis vector q_j = (v_j - sum_{i<j} s_i^(j) q_i) / rho_j
// was finished after z_j = B_j v_j was formed, so the columns matching the
// Hessenberg matrix are Zt_j = (Z_j - sum_{i<j} s_i^(j) Zt_i) / rho_j.  Turn
// the coefficients y on Zt (k of them) into coefficients on the stored Z.
__global__ void k_flex_coeffs(int k, int m, const double2* __restrict__ Sall, const double* __restrict__ rhoall,
                              double2* __restrict__ y) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int jj = k - 1; jj >= 0; --jj) {
    const double r = rhoall[jj];
    const double2 u = r > 0.0 ? make_double2(y[jj].x / r, y[jj].y / r) : make_double2(0.0, 0.0);
    y[jj] = u;
    for (int i = 0; i < jj; ++i) y[i] = csub(y[i], cmul(u, Sall[(int64_t)jj * m + i]));
  }
}
void launch_flex_coeffs(int k, int m, const double2* Sall, const double* rhoall, double2* y, hipStream_t st) {
  k_flex_coeffs<<<1, 64, 0, st>>>(k, m, Sall, rhoall, y);
}
template <class VT, class T>
void launch_dcgs_update(int64_t n, const VT* V, int64_t ldv, int q, const double2* coef, VT* v, T* w, double* rpart,
                        double* out_norm, hipStream_t st) {
  k_dcgs_update<VT, T><<<kRedBlocks, kThreads, 0, st>>>(n, V, ldv, q, coef, v, w, rpart, 0, 0, 0, nullptr,
                                                        rows_aligned<VT>(V, v, w, ldv, 0, 0));
  if (out_norm) k_norm2_final<<<1, kThreads, 0, st>>>(rpart, out_norm, nullptr, nullptr);
}
template <class Ti, class To>
void launch_scale_by_partials(int64_t n, const Ti* w, const double* rpart, double* out_norm, To* v, hipStream_t st) {
  constexpr int R = scale_rows<Ti, To>();
  k_scale_by_partials<Ti, To><<<blocks_for((n + R - 1) / R, kThreads * kScaleGroups), kThreads, 0, st>>>(
      n, w, rpart, out_norm, v, vec_ok(R, w, v, 0, 0));
}
template <class VT, class T>
void launch_mdot2_b(int64_t n, const VT* V, int64_t ldv, int64_t vstride, int q, const VT* v, const T* w,
                    int64_t wstride, double2* partial, int64_t pstride, const int* active, int nrhs, hipStream_t st) {
  dim3 grid(mdot2_parts(n), q > 0 ? (q + 7) / 8 : 1, nrhs);
  k_mdot2<VT, T><<<grid, kThreads, 0, st>>>(n, V, ldv, q, v, w, partial, vstride, wstride, pstride, active,
                                            rows_aligned<VT>(V, v, w, ldv, vstride, wstride));
}
void launch_dcgs_coef_b(int j, int m, const double2* dots, int64_t dstride, double2* Hraw, const double* tnorm,
                        double2* coef, double2* H, double* cs, double2* sn, double2* g, const double* beta,
                        const double* bnorm, double* est, const int* active, int nrhs, hipStream_t st) {
  k_dcgs_coef<<<dim3(1, 1, nrhs), 64, 0, st>>>(j, m, dots, Hraw, tnorm, coef, H, cs, sn, g, 0.0, 1.0, est, nullptr,
                                               nullptr, beta, bnorm, dstride, active);
}
template <class VT, class T>
void launch_dcgs_update_b(int64_t n, const VT* V, int64_t ldv, int64_t vstride, int q, const double2* coef,
                          int64_t cstride, VT* v, T* w, int64_t wstride, double* rpart, double* out_norm,
                          const int* active, int nrhs, hipStream_t st) {
  k_dcgs_update<VT, T><<<dim3(kRedBlocks, 1, nrhs), kThreads, 0, st>>>(
      n, V, ldv, q, coef, v, w, rpart, vstride, wstride, cstride, active, rows_aligned<VT>(V, v, w, ldv, vstride, wstride));
  k_norm2_final<<<dim3(1, 1, nrhs), kThreads, 0, st>>>(rpart, out_norm, nullptr, active);
}
void launch_givens(int j, int m, const double2* h1, const double2* h2, const double* nrm, double2* H, double* cs,
                   double2* sn, double2* g, double beta, double bnorm, double* est, hipStream_t st) {
  k_givens<<<1, 64, 0, st>>>(j, m, h1, h2, nrm, H, cs, sn, g, beta, bnorm, est);
}
void launch_backsolve(int k, int m, const double2* H, const double2* g, double2* y, hipStream_t st) {
  k_backsolve<<<1, 64, 0, st>>>(k, m, H, g, y);
}
// ---- batched launch wrappers (grid.z = system index)
template <class T, class MT, class RT>
void launch_block_apply_b(int64_t nb, const int* blk_ptr, const int* blk_dofs, const MT* minv, int nrhs,
                          int64_t rstride, const RT* r, int64_t zstride, T* z, const int* active, hipStream_t st) {
  k_block_apply_b<T, MT, RT><<<blocks_for(nb, 4), kThreads, 0, st>>>(nb, blk_ptr, blk_dofs, minv, nrhs, rstride, r, zstride,
                                                              z, active);
}
template <class T>
void launch_spmv_b(int64_t n, const int* rowptr, const int* col, const T* val, int nrhs, int64_t ld, const T* x,
                   const T* b, T* y, const int* active, hipStream_t st) {
  k_spmv_b<T><<<blocks_for(n * kLanes), kThreads, 0, st>>>(n, rowptr, col, val, nrhs, ld, x, b, y, active);
}
void launch_reduce_cols_b(int q, int nparts, const double2* partial, int64_t pstride, double2* out, int64_t ostride,
                          const int* flag, const int* active, int nrhs, hipStream_t st) {
  dim3 grid(q, 1, nrhs);
  k_reduce_cols<<<grid, kThreads, 0, st>>>(partial, nparts, out, flag, pstride, ostride, active);
}
template <class T>
void launch_norm2_b(int64_t n, const T* w, int64_t wstride, double* partial, double* out_norm, const int* active,
                    int nrhs, hipStream_t st) {
  dim3 grid(kRedBlocks, 1, nrhs);
  k_norm2_partial<T><<<grid, kThreads, 0, st>>>(n, w, partial, wstride, active);
  dim3 g1(1, 1, nrhs);
  k_norm2_final<<<g1, kThreads, 0, st>>>(partial, out_norm, nullptr, active);
}
template <class Ti, class To>
void launch_scale_by_inv_b(int64_t n, const Ti* w, int64_t wstride, const double* norm, To* v, int64_t vstride,
                           const int* active, int nrhs, hipStream_t st) {
  constexpr int R = scale_rows<Ti, To>();
  dim3 grid(blocks_for((n + R - 1) / R), 1, nrhs);
  k_scale_by_inv<Ti, To><<<grid, kThreads, 0, st>>>(n, w, norm, v, wstride, vstride, active,
                                                    vec_ok(R, w, v, wstride, vstride));
}
void launch_givens_b(int j, int m, const double2* h1, const double2* h2, int64_t hstride, int64_t h2stride,
                     const double* nrm, double2* H, double* cs, double2* sn, double2* g, const double* beta,
                     const double* bnorm, double* est, const int* active, int nrhs, hipStream_t st) {
  dim3 grid(1, 1, nrhs);
  k_givens_b<<<grid, 64, 0, st>>>(j, m, h1, h2, nrm, H, cs, sn, g, beta, bnorm, est, hstride, h2stride, active);
}
void launch_backsolve_b(const int* ks, int m, const double2* H, const double2* g, double2* y, int64_t ystride,
                        const int* active, int nrhs, hipStream_t st) {
  dim3 grid(1, 1, nrhs);
  k_backsolve_b<<<grid, 64, 0, st>>>(ks, m, H, g, y, ystride, active);
}
template <class VT, class T>
void launch_combine_b(int64_t n, const VT* V, int64_t ldv, int64_t vstride, const int* qs, const double2* y,
                      int64_t ystride, T* u, int64_t ustride, const int* active, int nrhs, hipStream_t st) {
  dim3 grid(blocks_for(n), 1, nrhs);
  k_combine<VT, T><<<grid, kThreads, 0, st>>>(n, V, ldv, 0, y, u, vstride, ystride, ustride, qs, active);
}
template <class T>
void launch_axpy_b(int64_t n, const T* z, int64_t zstride, double2* x, int64_t xstride, const int* active, int nrhs,
                   hipStream_t st) {
  dim3 grid(blocks_for(n), 1, nrhs);
  k_axpy<T><<<grid, kThreads, 0, st>>>(n, z, x, zstride, xstride, active);
}
void launch_diag_scale_b(int64_t n, const double2* in, int64_t istride, const double* s, int divide, double2* out,
                         int64_t ostride, int nrhs, hipStream_t st) {
  dim3 grid(blocks_for(n), 1, nrhs);
  k_diag_scale<<<grid, kThreads, 0, st>>>(n, in, s, divide, out, istride, ostride);
}
template <class T>
void launch_to_storage_b(int64_t n, const double2* in, int64_t istride, T* out, int64_t ostride, int nrhs,
                         hipStream_t st) {
  dim3 grid(blocks_for(n), 1, nrhs);
  k_convert_b<T><<<grid, kThreads, 0, st>>>(n, in, istride, out, ostride);
}
void launch_to_c64(int64_t n, const double2* in, float2* out, hipStream_t st) {
  k_to_c64<<<blocks_for(n), kThreads, 0, st>>>(n, in, out);
}
#define EDDY_INST(T)                                                                                              \
  template void launch_spmv<T>(int64_t, const int*, const int*, const int*, const T*, int64_t, const int*,       \
                               const int*, const double*, const double2*, const T*, const double2*, T*,          \
                               hipStream_t, int, int, const int*, const int*);                                   \
  template void launch_block_apply<T, T, T>(int64_t, const int*, const int*, const T*, const T*, T*, hipStream_t); \
  template void launch_mdot<T>(int64_t, const T*, int64_t, int, const T*, double2*, hipStream_t, int, const int*); \
  template void launch_norm2<T>(int64_t, const T*, double*, double*, hipStream_t);                                \
  template void launch_scale_by_inv<T, T>(int64_t, const T*, const double*, T*, hipStream_t);                     \
  template void launch_scale_host<double2, T>(int64_t, const double2*, double, T*, hipStream_t);                  \
  template void launch_combine<T, T>(int64_t, const T*, int64_t, int, const double2*, T*, hipStream_t);           \
  template void launch_axpy<T>(int64_t, const T*, double2*, hipStream_t);
EDDY_INST(double2)
EDDY_INST(float2)
#undef EDDY_INST
template void launch_mdot2<double2, double2>(int64_t, const double2*, int64_t, int, const double2*, const double2*,
                                             double2*, hipStream_t);
template void launch_mdot2<float2, float2>(int64_t, const float2*, int64_t, int, const float2*, const float2*,
                                           double2*, hipStream_t);
template void launch_mdot2<hbasis, float2>(int64_t, const hbasis*, int64_t, int, const hbasis*, const float2*,
                                           double2*, hipStream_t);
template void launch_dcgs_update<double2, double2>(int64_t, const double2*, int64_t, int, const double2*, double2*,
                                                   double2*, double*, double*, hipStream_t);
template void launch_dcgs_update<float2, float2>(int64_t, const float2*, int64_t, int, const double2*, float2*,
                                                 float2*, double*, double*, hipStream_t);
template void launch_dcgs_update<hbasis, float2>(int64_t, const hbasis*, int64_t, int, const double2*, hbasis*,
                                                 float2*, double*, double*, hipStream_t);
template void launch_scale_by_inv<float2, hbasis>(int64_t, const float2*, const double*, hbasis*, hipStream_t);
template void launch_scale_by_partials<float2, hbasis>(int64_t, const float2*, const double*, double*, hbasis*,
                                                       hipStream_t);
template void launch_scale_by_partials<float2, float2>(int64_t, const float2*, const double*, double*, float2*,
                                                       hipStream_t);
template void launch_scale_by_partials<double2, double2>(int64_t, const double2*, const double*, double*, double2*,
                                                         hipStream_t);
template void launch_scale_host<double2, hbasis>(int64_t, const double2*, double, hbasis*, hipStream_t);
template void launch_combine<hbasis, float2>(int64_t, const hbasis*, int64_t, int, const double2*, float2*,
                                             hipStream_t);
template void launch_block_apply<float2, uint32_t, hbasis>(int64_t, const int*, const int*, const uint32_t*,
                                                           const hbasis*, float2*, hipStream_t);
template void launch_mdot2_b<double2, double2>(int64_t, const double2*, int64_t, int64_t, int, const double2*, const double2*,
                                      int64_t, double2*, int64_t, const int*, int, hipStream_t);
template void launch_mdot2_b<float2, float2>(int64_t, const float2*, int64_t, int64_t, int, const float2*, const float2*,
                                     int64_t, double2*, int64_t, const int*, int, hipStream_t);
template void launch_dcgs_update_b<double2, double2>(int64_t, const double2*, int64_t, int64_t, int, const double2*, int64_t,
                                            double2*, double2*, int64_t, double*, double*, const int*, int,
                                            hipStream_t);
template void launch_dcgs_update_b<float2, float2>(int64_t, const float2*, int64_t, int64_t, int, const double2*, int64_t,
                                           float2*, float2*, int64_t, double*, double*, const int*, int,
                                           hipStream_t);
#define EDDY_INST_B(T)                                                                                            \
  template void launch_block_apply_b<T, T, T>(int64_t, const int*, const int*, const T*, int, int64_t, const T*,  \
                                              int64_t, T*, const int*, hipStream_t);                              \
  template void launch_spmv_b<T>(int64_t, const int*, const int*, const T*, int, int64_t, const T*, const T*, T*,  \
                                 const int*, hipStream_t);                                                        \
  template void launch_norm2_b<T>(int64_t, const T*, int64_t, double*, double*, const int*, int, hipStream_t);      \
  template void launch_scale_by_inv_b<T, T>(int64_t, const T*, int64_t, const double*, T*, int64_t, const int*,  \
                                            int, hipStream_t);                                                    \
  template void launch_combine_b<T, T>(int64_t, const T*, int64_t, int64_t, const int*, const double2*, int64_t,  \
                                       T*, int64_t, const int*, int, hipStream_t);                                \
  template void launch_axpy_b<T>(int64_t, const T*, int64_t, double2*, int64_t, const int*, int, hipStream_t);      \
  template void launch_to_storage_b<T>(int64_t, const double2*, int64_t, T*, int64_t, int, hipStream_t);
EDDY_INST_B(double2)
EDDY_INST_B(float2)
#undef EDDY_INST_B
template void launch_block_apply<float2, uint32_t, float2>(int64_t, const int*, const int*, const uint32_t*,
                                                           const float2*, float2*, hipStream_t);
template void launch_block_apply_b<float2, uint32_t, float2>(int64_t, const int*, const int*, const uint32_t*, int,
                                                             int64_t, const float2*, int64_t, float2*, const int*,
                                                             hipStream_t);
template void launch_block_apply_b<float2, uint32_t, hbasis>(int64_t, const int*, const int*, const uint32_t*, int,
                                                             int64_t, const hbasis*, int64_t, float2*, const int*,
                                                             hipStream_t);
void launch_block_apply_mfma(int64_t nb, const int* blk_ptr, const int* blk_dofs, const uint32_t* minv, int nrhs,
                             int64_t rstride, const hbasis* r, int64_t zstride, float2* z, const int* active,
                             int interleave, hipStream_t st) {
  k_block_apply_mfma<<<blocks_for(nb, 4), kThreads, 0, st>>>(nb, blk_ptr, blk_dofs, minv, nrhs, rstride, r, zstride,
                                                             z, active, interleave);
}
void launch_spmv_b_il(int64_t n, const int* rowptr, const int* col, const float2* val, int nrhs, int64_t ld,
                      const float2* xil, float2* y, const int* active, hipStream_t st) {
  k_spmv_b_il<<<blocks_for(n * kLanes), kThreads, 0, st>>>(n, rowptr, col, val, nrhs, ld, xil, y, active);
}
template void launch_scale_by_inv_b<double2, float2>(int64_t, const double2*, int64_t, const double*, float2*, int64_t,
                                                     const int*, int, hipStream_t);
template void launch_scale_by_inv_b<double2, hbasis>(int64_t, const double2*, int64_t, const double*, hbasis*, int64_t,
                                                     const int*, int, hipStream_t);
template void launch_scale_by_inv_b<float2, hbasis>(int64_t, const float2*, int64_t, const double*, hbasis*, int64_t,
                                                    const int*, int, hipStream_t);
template void launch_combine_b<hbasis, float2>(int64_t, const hbasis*, int64_t, int64_t, const int*, const double2*,
                                               int64_t, float2*, int64_t, const int*, int, hipStream_t);
template void launch_mdot2_b<hbasis, float2>(int64_t, const hbasis*, int64_t, int64_t, int, const hbasis*,
                                             const float2*, int64_t, double2*, int64_t, const int*, int, hipStream_t);
template void launch_dcgs_update_b<hbasis, float2>(int64_t, const hbasis*, int64_t, int64_t, int, const double2*,
                                                   int64_t, hbasis*, float2*, int64_t, double*, double*, const int*,
                                                   int, hipStream_t);
__global__ __launch_bounds__(kThreads) void k_to_c16(int64_t n, const double2* __restrict__ in,
                                                     uint32_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = pack_h2(in[i].x, in[i].y);
}
void launch_to_c16(int64_t n, const double2* in, uint32_t* out, hipStream_t st) {
  k_to_c16<<<blocks_for(n), kThreads, 0, st>>>(n, in, out);
}
void launch_face(int64_t nf, const double* xyz, const int* face, const int* face_region, const double* nu_reg,
                 const double* sig_reg, double omega, double2* fbuf, double* area3, hipStream_t st) {
  if (nf <= 0) return;
  k_face<<<blocks_for(nf), kThreads, 0, st>>>(nf, xyz, face, face_region, nu_reg, sig_reg, omega, fbuf, area3);
}
void launch_factor_pq(int64_t n, int64_t ne, const int* rowptr, const int* col, const double2* val, const double* s,
                      double omega, float2* pq, hipStream_t st) {
  k_factor_pq<<<blocks_for(n), kThreads, 0, st>>>(n, ne, rowptr, col, val, s, omega, pq);
}
void launch_spmv_mf(int64_t n, int64_t ne, const int* rowptr, const int* col, const float2* pq, int nrhs, int64_t ld,
                    const float2* x, float2* u, float2* y, const mf_sys* sys, const int* active, hipStream_t st) {
  k_scale_sys<<<dim3(blocks_for(n), 1, nrhs), kThreads, 0, st>>>(n, x, ld, sys, u, active);
  k_spmv_mf<<<blocks_for(n * kLanes), kThreads, 0, st>>>(n, ne, rowptr, col, pq, nrhs, ld, u, y, sys, active);
}
void launch_diag_scale(int64_t n, const double2* in, const double* s, int divide, double2* out, hipStream_t st) {
  k_diag_scale<<<blocks_for(n), kThreads, 0, st>>>(n, in, s, divide, out, 0, 0);
}
void launch_zero(int64_t n, double2* x, hipStream_t st) { k_zero<<<blocks_for(n), kThreads, 0, st>>>(n, x); }
void launch_vmean(int64_t nc, int ncomp, const int* comp, const double* lumped, double2* V, double2* scratch,
                  hipStream_t st) {
  if (ncomp <= 0 || nc <= 0) return;
  k_vmean<<<ncomp, kThreads, 0, st>>>(nc, comp, lumped, V, scratch);
  k_vmean_sub<<<blocks_for(nc), kThreads, 0, st>>>(nc, comp, scratch, V);
}
void launch_dz_volume(int64_t nt, const double* xyz, const int* tet, const int* region, const uint8_t* signbits,
                      const int* tet2edge, const double* nu_d, const double* sig_d, const double* nu_0,
                      const double* sig_0, double omega, int64_t ne, const double2* xd, const int* vmap_d, int nl,
                      const double2* x0, int64_t ld0, const int* vmap_0, double2* partial, double2* out,
                      hipStream_t st) {
  k_dz_volume<<<kRedBlocks, kThreads, 0, st>>>(nt, xyz, tet, region, signbits, tet2edge, nu_d, sig_d, nu_0, sig_0,
                                               omega, ne, xd, vmap_d, nl, x0, ld0, vmap_0, partial);
  k_reduce_cols<<<nl, kThreads, 0, st>>>(partial, kRedBlocks, out, nullptr, 0, 0, nullptr);
}
void launch_udot(int64_t n, const double2* a, const double2* b, double2* partial, double2* out, hipStream_t st) {
  k_udot_partial<<<kRedBlocks, kThreads, 0, st>>>(n, a, b, partial);
  k_reduce_cols<<<1, kThreads, 0, st>>>(partial, kRedBlocks, out, nullptr, 0, 0, nullptr);
}
void launch_edge_divergence(int64_t nv, const int* wtrowptr, const int* wtcol, const int* edges, const double2* b,
                            double2* d, hipStream_t st) {
  k_edge_divergence<<<blocks_for(nv), kThreads, 0, st>>>(nv, wtrowptr, wtcol, edges, b, d);
}
void launch_lap_diag(int64_t nv, const int* wtrowptr, const int* wtcol, const double* wtval, const int* edges,
                     const double* s, double* diag, hipStream_t st) {
  k_lap_diag<<<blocks_for(nv), kThreads, 0, st>>>(nv, wtrowptr, wtcol, wtval, edges, s, diag);
}
void launch_lap_assemble(int64_t nv, const int* wtrowptr, const int* wtcol, const double* wtval, const int* edges,
                         const double* s, const int* lrowptr, const int* lcol, double* lval, hipStream_t st) {
  k_lap_assemble<<<blocks_for(nv), kThreads, 0, st>>>(nv, wtrowptr, wtcol, wtval, edges, s, lrowptr, lcol, lval);
}
void launch_lap_spmv_dot(int64_t nv, const int* lrowptr, const int* lcol, const double* lval, const double2* p,
                         double2* q, double2* partial, hipStream_t st) {
  k_lap_spmv_dot<<<kRedBlocks, kThreads, 0, st>>>(nv, lrowptr, lcol, lval, p, q, partial);
}
void launch_cg_update(int64_t n, const double2* rz, const double2* pq_part, const double2* p, const double2* q,
                      const double* diag, double2* psi, double2* r, double2* z, double2* partial, hipStream_t st) {
  k_cg_update<<<kRedBlocks, kThreads, 0, st>>>(n, rz, pq_part, p, q, diag, psi, r, z, partial);
}
void launch_jacobi(int64_t n, const double2* r, const double* diag, double2* z, hipStream_t st) {
  k_jacobi<<<blocks_for(n), kThreads, 0, st>>>(n, r, diag, z);
}
void launch_cg_dir(int64_t n, const double2* rz_part, const double2* rz_old, double2* rz_new, const double2* z,
                   double2* p, hipStream_t st) {
  k_cg_dir<<<blocks_for(n), kThreads, 0, st>>>(n, rz_part, rz_old, rz_new, z, p);
}
void launch_project(int64_t ne, int64_t nc, const int* edges, const int* cond_nodes, const double2* psi, double omega,
                    double2* x, hipStream_t st) {
  k_project<<<blocks_for(ne + nc), kThreads, 0, st>>>(ne, nc, edges, cond_nodes, psi, omega, x);
}
void launch_edge_field(int64_t ne, const int* edge_v, const double2* x, double omega, double2* E, hipStream_t st) {
  k_edge_field<<<blocks_for(ne), kThreads, 0, st>>>(ne, edge_v, x, omega, E);
}

}  // namespace eddy
