// Learned coarse correction: subdomain statistics, features and targets,
// the graph network (bf16 operands on MFMA, float32 accumulation) forward,
// backward and Adam, and the per-subdomain scaling of the preconditioned
// vector.  The definitions (features, targets, network, rounding points) are
// those stated in gnn.h and eddy.h.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"
#include "gnn.h"

namespace eddy {
namespace {

#include "devmath.h"

typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

// float32 -> bfloat16 bits, round to nearest, ties to even (finite inputs)
__device__ __forceinline__ uint16_t f2bf(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// C [M x N] (float32, row stride ldc) = A [M x K] B [K x N] with bf16
// operands fetched by a(i, k), b(k, j) (bit patterns).  M, N, K multiples of
// 16; the 16 x 16 output tiles are spread over the workgroup's wavefronts.
// v_mfma_f32_16x16x16_bf16: lane l supplies A(l % 16, 4 (l / 16) + u) and
// B(4 (l / 16) + u, l % 16), u = 0..3, and receives D(4 (l / 16) + u, l % 16).
template <class FA, class FB>
__device__ void gemm(int M, int N, int K, FA a, FB b, float* C, int ldc) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  const int tn = N / 16, ntile = (M / 16) * tn;
  const int r = lane & 15, kq = (lane >> 4) * 4;
  for (int t = wave; t < ntile; t += nw) {
    const int i0 = (t / tn) * 16, j0 = (t % tn) * 16;
    f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += 16) {
      bf16x4_t av, bv;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        av[u] = (short)a(i0 + r, k0 + kq + u);
        bv[u] = (short)b(k0 + kq + u, j0 + r);
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) C[(i0 + kq + u) * ldc + j0 + r] = acc[u];
  }
}

struct Scratch {
  float *Z0, *Z1, *Z2, *H, *Tf, *dH, *Gt, *Y;
  uint16_t *Xb, *Hb1, *Hb2, *Hb3, *Tb, *dZb, *dTb, *dYb;
};
__device__ Scratch carve(float* base) {
  constexpr int PW = kGnnP * kGnnWidth;
  Scratch s;
  s.Z0 = base; s.Z1 = base + PW; s.Z2 = base + 2 * PW; s.H = base + 3 * PW; s.Tf = base + 4 * PW;
  s.dH = base + 5 * PW; s.Gt = base + 6 * PW; s.Y = base + 7 * PW;
  uint16_t* h = (uint16_t*)(base + 7 * PW + kGnnP * kGnnFout);
  s.Xb = h; h += kGnnP * kGnnFin;
  s.Hb1 = h; h += PW; s.Hb2 = h; h += PW; s.Hb3 = h; h += PW; s.Tb = h; h += PW; s.dZb = h; h += PW;
  s.dTb = h; h += PW; s.dYb = h;
  return s;
}

// Forward pass of one sample (module doc of the oracle; same rounding points).
__device__ void forward(const float* __restrict__ th, const uint16_t* __restrict__ Ab, const float* __restrict__ X,
                        Scratch& s) {
  constexpr int W = kGnnWidth, P = kGnnP;
  const int t = threadIdx.x, nt = blockDim.x;
  for (int e = t; e < P * kGnnFin; e += nt) s.Xb[e] = f2bf(X[e]);
  __syncthreads();
  auto Aop = [&](int i, int k) { return Ab[i * P + k]; };
  // layer 0
  gemm(P, W, kGnnFin, [&](int i, int k) { return s.Xb[i * kGnnFin + k]; },
       [&](int k, int j) { return f2bf(th[kGnnOffW0 + k * W + j]); }, s.Tf, W);
  __syncthreads();
  for (int e = t; e < P * W; e += nt) s.Tb[e] = f2bf(s.Tf[e]);
  __syncthreads();
  gemm(P, W, P, Aop, [&](int k, int j) { return s.Tb[k * W + j]; }, s.Z0, W);
  __syncthreads();
  for (int e = t; e < P * W; e += nt) {
    const float z = s.Z0[e] + th[kGnnOffB0 + (e % W)];
    s.Z0[e] = z;
    const float h = z > 0.f ? z : 0.f;
    s.H[e] = h;
    s.Hb1[e] = f2bf(h);
  }
  __syncthreads();
  // layers 1, 2 (residual)
  for (int l = 1; l <= 2; ++l) {
    const uint16_t* Hb = l == 1 ? s.Hb1 : s.Hb2;
    uint16_t* Hn = l == 1 ? s.Hb2 : s.Hb3;
    float* Z = l == 1 ? s.Z1 : s.Z2;
    const int oW = l == 1 ? kGnnOffW1 : kGnnOffW2, ob = l == 1 ? kGnnOffB1 : kGnnOffB2;
    gemm(P, W, W, [&](int i, int k) { return Hb[i * W + k]; },
         [&](int k, int j) { return f2bf(th[oW + k * W + j]); }, s.Tf, W);
    __syncthreads();
    for (int e = t; e < P * W; e += nt) s.Tb[e] = f2bf(s.Tf[e]);
    __syncthreads();
    gemm(P, W, P, Aop, [&](int k, int j) { return s.Tb[k * W + j]; }, Z, W);
    __syncthreads();
    for (int e = t; e < P * W; e += nt) {
      const float z = Z[e] + th[ob + (e % W)];
      Z[e] = z;
      const float h = (z > 0.f ? z : 0.f) + s.H[e];
      s.H[e] = h;
      Hn[e] = f2bf(h);
    }
    __syncthreads();
  }
  // output layer
  gemm(P, kGnnFout, W, [&](int i, int k) { return s.Hb3[i * W + k]; },
       [&](int k, int j) { return f2bf(th[kGnnOffW3 + k * kGnnFout + j]); }, s.Tf, kGnnFout);
  __syncthreads();
  for (int e = t; e < P * kGnnFout; e += nt) s.Tb[e] = f2bf(s.Tf[e]);
  __syncthreads();
  gemm(P, kGnnFout, P, Aop, [&](int k, int j) { return s.Tb[k * kGnnFout + j]; }, s.Y, kGnnFout);
  __syncthreads();
  for (int e = t; e < P * kGnnFout; e += nt) s.Y[e] += th[kGnnOffB3 + (e % kGnnFout)];
  __syncthreads();
}

__global__ __launch_bounds__(kThreads) void k_gnn_forward(const float* __restrict__ th,
                                                          const uint16_t* __restrict__ Ab,
                                                          const float* __restrict__ X, float* __restrict__ Y,
                                                          float* __restrict__ scratch) {
  const int smp = blockIdx.x;
  Scratch s = carve(scratch + (int64_t)smp * kGnnScratch);
  forward(th, Ab, X + (int64_t)smp * kGnnP * kGnnFin, s);
  for (int e = threadIdx.x; e < kGnnP * kGnnFout; e += blockDim.x) Y[(int64_t)smp * kGnnP * kGnnFout + e] = s.Y[e];
}

// Forward, loss and backward of one sample per workgroup; per-sample
// gradients into grads[smp][kGnnParams], loss into loss[smp].
__global__ __launch_bounds__(kThreads) void k_gnn_sample(const float* __restrict__ th, const uint16_t* __restrict__ Ab,
                                                         const float* __restrict__ Xall,
                                                         const float* __restrict__ call,
                                                         const float* __restrict__ wall, float* __restrict__ scratch,
                                                         float* __restrict__ grads, float* __restrict__ loss) {
  constexpr int W = kGnnWidth, P = kGnnP, FO = kGnnFout;
  const int smp = blockIdx.x, t = threadIdx.x, nt = blockDim.x;
  Scratch s = carve(scratch + (int64_t)smp * kGnnScratch);
  const float* cs = call + (int64_t)smp * P * 2;
  const float* w = wall + (int64_t)smp * P;
  float* g = grads + (int64_t)smp * kGnnParams;
  forward(th, Ab, Xall + (int64_t)smp * P * kGnnFin, s);
  // loss and dY (float32), dY rounded for the GEMMs
  double lacc = 0.0;
  for (int e = t; e < P * FO; e += nt) {
    const int p = e / FO, j = e % FO;
    float d = 0.f;
    if (j < 2) {
      const float diff = s.Y[e] - cs[p * 2 + j];
      lacc += (double)w[p] * diff * diff;
      d = 2.f * w[p] * diff;
    }
    s.Tf[e] = d;
    s.dYb[e] = f2bf(d);
  }
  __syncthreads();
  // output layer: b3, dT3 = bf16(A dY), dW3 = Hb3^T dT3, dH = dT3 W3^T
  for (int j = t; j < FO; j += nt) {
    float acc = 0.f;
    for (int p = 0; p < P; ++p) acc += s.Tf[p * FO + j];
    g[kGnnOffB3 + j] = j < 2 ? acc : 0.f;
  }
  auto Aop = [&](int i, int k) { return Ab[i * P + k]; };
  gemm(P, FO, P, Aop, [&](int k, int j) { return s.dYb[k * FO + j]; }, s.Gt, FO);
  __syncthreads();
  for (int e = t; e < P * FO; e += nt) s.dTb[e] = f2bf(s.Gt[e]);
  __syncthreads();
  gemm(W, FO, P, [&](int i, int k) { return s.Hb3[k * W + i]; }, [&](int k, int j) { return s.dTb[k * FO + j]; },
       s.Gt, FO);
  __syncthreads();
  for (int e = t; e < W * FO; e += nt) g[kGnnOffW3 + e] = (e % FO) < 2 ? s.Gt[e] : 0.f;
  gemm(P, W, FO, [&](int i, int k) { return s.dTb[i * FO + k]; },
       [&](int k, int j) { return f2bf(th[kGnnOffW3 + j * FO + k]); }, s.dH, W);
  __syncthreads();
  // layers 2, 1
  for (int l = 2; l >= 1; --l) {
    const float* Z = l == 2 ? s.Z2 : s.Z1;
    const uint16_t* Hb = l == 2 ? s.Hb2 : s.Hb1;
    const int oW = l == 2 ? kGnnOffW2 : kGnnOffW1, ob = l == 2 ? kGnnOffB2 : kGnnOffB1;
    for (int e = t; e < P * W; e += nt) {
      const float dz = Z[e] > 0.f ? s.dH[e] : 0.f;
      s.Tf[e] = dz;
      s.dZb[e] = f2bf(dz);
    }
    __syncthreads();
    for (int j = t; j < W; j += nt) {
      float acc = 0.f;
      for (int p = 0; p < P; ++p) acc += s.Tf[p * W + j];
      g[ob + j] = acc;
    }
    gemm(P, W, P, Aop, [&](int k, int j) { return s.dZb[k * W + j]; }, s.Gt, W);
    __syncthreads();
    for (int e = t; e < P * W; e += nt) s.dTb[e] = f2bf(s.Gt[e]);
    __syncthreads();
    gemm(W, W, P, [&](int i, int k) { return Hb[k * W + i]; }, [&](int k, int j) { return s.dTb[k * W + j]; },
         s.Gt, W);
    __syncthreads();
    for (int e = t; e < W * W; e += nt) g[oW + e] = s.Gt[e];
    // dH += dT W^T (the residual path keeps dH)
    gemm(P, W, W, [&](int i, int k) { return s.dTb[i * W + k]; },
         [&](int k, int j) { return f2bf(th[oW + j * W + k]); }, s.Gt, W);
    __syncthreads();
    for (int e = t; e < P * W; e += nt) s.dH[e] += s.Gt[e];
    __syncthreads();
  }
  // layer 0
  for (int e = t; e < P * W; e += nt) {
    const float dz = s.Z0[e] > 0.f ? s.dH[e] : 0.f;
    s.Tf[e] = dz;
    s.dZb[e] = f2bf(dz);
  }
  __syncthreads();
  for (int j = t; j < W; j += nt) {
    float acc = 0.f;
    for (int p = 0; p < P; ++p) acc += s.Tf[p * W + j];
    g[kGnnOffB0 + j] = acc;
  }
  gemm(P, W, P, Aop, [&](int k, int j) { return s.dZb[k * W + j]; }, s.Gt, W);
  __syncthreads();
  for (int e = t; e < P * W; e += nt) s.dTb[e] = f2bf(s.Gt[e]);
  __syncthreads();
  gemm(kGnnFin, W, P, [&](int i, int k) { return s.Xb[k * kGnnFin + i]; },
       [&](int k, int j) { return s.dTb[k * W + j]; }, s.Gt, W);
  __syncthreads();
  for (int e = t; e < kGnnFin * W; e += nt) g[kGnnOffW0 + e] = s.Gt[e];
  // the loss (block sum in a fixed order)
  __shared__ double shd[4];
  const double L = block_sum(lacc, shd);
  if (t == 0) loss[smp] = (float)L;
}

// Batch-mean gradient (fixed order over samples) and one Adam step.
__global__ __launch_bounds__(kThreads) void k_gnn_adam(int nsamp, const float* __restrict__ grads,
                                                       float* __restrict__ th, float* __restrict__ m,
                                                       float* __restrict__ v, float* __restrict__ gmean, int step,
                                                       float lr) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kGnnParams) return;
  float acc = 0.f;
  for (int s = 0; s < nsamp; ++s) acc += grads[(int64_t)s * kGnnParams + i];
  const float gi = acc / (float)nsamp;
  if (gmean) gmean[i] = gi;
  if (lr == 0.f) return;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / (1.f - powf(b1, (float)step));
  const float vh = vi / (1.f - powf(b2, (float)step));
  th[i] -= lr * mh / (sqrtf(vh) + eps);
}

// Per-subdomain sums: workgroup (x, p) covers part x of subdomain p's range.
template <class T>
__global__ __launch_bounds__(kThreads) void k_gnn_stats(const int* __restrict__ perm, const int* __restrict__ sub_ptr,
                                                        const T* __restrict__ r, const T* __restrict__ z,
                                                        const T* __restrict__ e, const T* __restrict__ eb,
                                                        const double* __restrict__ rs, const double* __restrict__ es,
                                                        double2* __restrict__ partial) {
  const int p = blockIdx.y, part = blockIdx.x;
  const int q0 = sub_ptr[p], q1 = sub_ptr[p + 1];
  double rr = 0, zz = 0, ee = 0;
  double2 zr = make_double2(0, 0), zd = make_double2(0, 0);
  for (int q = q0 + part * blockDim.x + threadIdx.x; q < q1; q += gridDim.x * blockDim.x) {
    const int i = perm[q];
    double2 ri = ld2(r[i]);
    const double2 zi = ld2(z[i]);
    if (rs) ri = make_double2(ri.x * rs[i], ri.y * rs[i]);
    rr = fma(ri.x, ri.x, fma(ri.y, ri.y, rr));
    zz = fma(zi.x, zi.x, fma(zi.y, zi.y, zz));
    zr = cfma_conj(zi, ri, zr);
    if (e) {
      double2 ei = ld2(e[i]);
      if (eb) ei = csub(ei, ld2(eb[i]));
      if (es) ei = make_double2(ei.x / es[i], ei.y / es[i]);
      ee = fma(ei.x, ei.x, fma(ei.y, ei.y, ee));
      zd = cfma_conj(zi, csub(ei, zi), zd);
    }
  }
  __shared__ double sh[4];
  const double v[7] = {rr, zz, zr.x, zr.y, zd.x, zd.y, ee};
  double out[7];
#pragma unroll
  for (int k = 0; k < 7; ++k) out[k] = block_sum(v[k], sh);
  if (threadIdx.x == 0) {
    double2* o = partial + ((int64_t)p * gridDim.x + part) * 4;
    o[0] = make_double2(out[0], out[1]);
    o[1] = make_double2(out[2], out[3]);
    o[2] = make_double2(out[4], out[5]);
    o[3] = make_double2(out[6], 0.0);
  }
}

// Reduce the parts (fixed order): sums[p*4 + 0] = (|r|^2, |z|^2), [1] = z^H r,
// [2] = z^H (e - z), [3] = (|e|^2, 0).
__global__ void k_gnn_stats_reduce(int nparts, const double2* __restrict__ partial, double2* __restrict__ sums) {
  const int p = threadIdx.x;
  if (p >= kGnnP) return;
  double2 acc[4] = {make_double2(0, 0), make_double2(0, 0), make_double2(0, 0), make_double2(0, 0)};
  for (int x = 0; x < nparts; ++x)
    for (int k = 0; k < 4; ++k) acc[k] = cadd(acc[k], partial[((int64_t)p * nparts + x) * 4 + k]);
  for (int k = 0; k < 4; ++k) sums[p * 4 + k] = acc[k];
}

__global__ void k_gnn_features(const double2* __restrict__ sums, const float* __restrict__ static4, int with_targets,
                               float* __restrict__ X, float* __restrict__ cstar, float* __restrict__ w) {
  const int p = threadIdx.x;
  __shared__ double tot[3];
  if (p == 0) {
    double a = 0, b = 0, c = 0;
    for (int k = 0; k < kGnnP; ++k) {
      a += sums[k * 4].x;
      b += sums[k * 4].y;
      c += sums[k * 4 + 3].x;
    }
    tot[0] = a; tot[1] = b; tot[2] = c;
  }
  __syncthreads();
  if (p >= kGnnP) return;
  const double rr = sums[p * 4].x, zz = sums[p * 4].y;
  const double2 zr = sums[p * 4 + 1], zd = sums[p * 4 + 2];
  const double sq = sqrt((double)kGnnP);
  float* x = X + p * kGnnFin;
  x[0] = (float)(tot[0] > 0 ? sqrt(rr / tot[0]) * sq : 0.0);
  x[1] = (float)(tot[1] > 0 ? sqrt(zz / tot[1]) * sq : 0.0);
  const double den = sqrt(zz) * sqrt(rr);
  x[2] = (float)(den > 0 ? zr.x / den : 0.0);
  x[3] = (float)(den > 0 ? zr.y / den : 0.0);
  for (int k = 0; k < 4; ++k) x[4 + k] = static4[p * 4 + k];
  for (int k = 8; k < kGnnFin; ++k) x[k] = 0.f;
  if (with_targets) {
    cstar[p * 2] = (float)(zz > 0 ? zd.x / zz : 0.0);
    cstar[p * 2 + 1] = (float)(zz > 0 ? zd.y / zz : 0.0);
    w[p] = (float)(tot[2] > 0 ? zz / tot[2] : 0.0);
  }
}

template <class T>
__global__ __launch_bounds__(kThreads) void k_gnn_scale(const int* __restrict__ perm, const int* __restrict__ sub_ptr,
                                                        const float* __restrict__ Y, T* __restrict__ z) {
  const int p = blockIdx.y;
  const int q0 = sub_ptr[p], q1 = sub_ptr[p + 1];
  const double2 f = make_double2(1.0 + (double)Y[p * kGnnFout], (double)Y[p * kGnnFout + 1]);
  for (int q = q0 + blockIdx.x * blockDim.x + threadIdx.x; q < q1; q += gridDim.x * blockDim.x) {
    const int i = perm[q];
    z[i] = st2<T>(cmul(f, ld2(z[i])));
  }
}

}  // namespace

int gnn_scratch_floats() { return kGnnScratch; }
template <class T>
void launch_gnn_stats(const int* perm, const int* sub_ptr, const T* r, const T* z, const T* e, const T* eb,
                      const double* rs, const double* es, double2* partial, double2* out, hipStream_t st) {
  k_gnn_stats<T><<<dim3(kGnnStatParts, kGnnP), kThreads, 0, st>>>(perm, sub_ptr, r, z, e, eb, rs, es, partial);
  k_gnn_stats_reduce<<<1, kGnnP, 0, st>>>(kGnnStatParts, partial, out);
}
void launch_gnn_features(const double2* sums, const float* static4, int with_targets, float* X, float* cstar,
                         float* w, hipStream_t st) {
  k_gnn_features<<<1, kGnnP, 0, st>>>(sums, static4, with_targets, X, cstar, w);
}
void launch_gnn_forward(int nsamp, const float* theta, const uint16_t* ahat, const float* X, float* Y,
                        float* scratch, hipStream_t st) {
  k_gnn_forward<<<nsamp, kThreads, 0, st>>>(theta, ahat, X, Y, scratch);
}
void launch_gnn_train(int nsamp, float* theta, float* m, float* v, const uint16_t* ahat, const float* X,
                      const float* cstar, const float* w, float* scratch, float* grads, float* loss, float* gmean,
                      int step, float lr, hipStream_t st) {
  k_gnn_sample<<<nsamp, kThreads, 0, st>>>(theta, ahat, X, cstar, w, scratch, grads, loss);
  k_gnn_adam<<<(kGnnParams + kThreads - 1) / kThreads, kThreads, 0, st>>>(nsamp, grads, theta, m, v, gmean, step, lr);
}
template <class T>
void launch_gnn_scale(const int* perm, const int* sub_ptr, const float* Y, T* z, hipStream_t st) {
  k_gnn_scale<T><<<dim3(16, kGnnP), kThreads, 0, st>>>(perm, sub_ptr, Y, z);
}
template void launch_gnn_stats<double2>(const int*, const int*, const double2*, const double2*, const double2*,
                                        const double2*, const double*, const double*, double2*, double2*,
                                        hipStream_t);
template void launch_gnn_stats<float2>(const int*, const int*, const float2*, const float2*, const float2*,
                                       const float2*, const double*, const double*, double2*, double2*, hipStream_t);
// out = s b - y (the equilibrated residual from M~ x~ = y)
__global__ __launch_bounds__(kThreads) void k_scaled_residual(int64_t n, const double2* __restrict__ b,
                                                              const double* __restrict__ s,
                                                              const double2* __restrict__ y,
                                                              double2* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[i] = make_double2(s[i] * b[i].x - y[i].x, s[i] * b[i].y - y[i].y);
}
void launch_scaled_residual(int64_t n, const double2* b, const double* s, const double2* y, double2* out,
                            hipStream_t st) {
  k_scaled_residual<<<blocks_for(n), kThreads, 0, st>>>(n, b, s, y, out);
}
template void launch_gnn_scale<double2>(const int*, const int*, const float*, double2*, hipStream_t);
template void launch_gnn_scale<float2>(const int*, const int*, const float*, float2*, hipStream_t);

}  // namespace eddy
