// Device helpers shared by the HIP translation units (complex arithmetic on
// double2/float2, deterministic wave/block reductions).  Included inside an
// anonymous namespace by each .hip file.
#pragma once

constexpr int kThreads = 256;

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// acc + conj(a) * b
__device__ __forceinline__ double2 cfma_conj(double2 a, double2 b, double2 acc) {
  return make_double2(fma(a.x, b.x, fma(a.y, b.y, acc.x)), fma(a.x, b.y, fma(-a.y, b.x, acc.y)));
}
// acc + a * b
__device__ __forceinline__ double2 cfma(double2 a, double2 b, double2 acc) {
  return make_double2(fma(a.x, b.x, fma(-a.y, b.y, acc.x)), fma(a.x, b.y, fma(a.y, b.x, acc.y)));
}
// acc + r * b (r real)
__device__ __forceinline__ double2 rfma(double r, double2 b, double2 acc) {
  return make_double2(fma(r, b.x, acc.x), fma(r, b.y, acc.y));
}

inline unsigned blocks_for(int64_t n, int per = kThreads) {
  int64_t b = (n + per - 1) / per;
  return (unsigned)(b < 1 ? 1 : b);
}

// Sum over the 64 lanes of a wavefront (fixed butterfly).
__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Deterministic sum over a 256-thread block (fixed shuffle tree, then the 4
// wave totals in order).  Result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) sh[w] = v;
  __syncthreads();
  double r = 0;
  if (threadIdx.x == 0) r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  __syncthreads();
  return r;
}


// Loads of data read exactly once (matrix values and indices): non-temporal,
// so that they do not evict reused data (the gathered vector) from the L2.
typedef double v2d_t __attribute__((ext_vector_type(2)));
typedef float v2f_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ int ld_stream(const int* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ float ld_stream(const float* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ double ld_stream(const double* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ double2 ld_stream(const double2* p) {
  const v2d_t v = __builtin_nontemporal_load(reinterpret_cast<const v2d_t*>(p));
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ float2 ld_stream(const float2* p) {
  const v2f_t v = __builtin_nontemporal_load(reinterpret_cast<const v2f_t*>(p));
  return make_float2(v.x, v.y);
}

// Complex half precision (block inverses of the mixed16 mode): real part in
// the low 16 bits, imaginary part in the high 16 bits, IEEE binary16 each.
__device__ __forceinline__ uint32_t ld_stream(const uint32_t* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ float2 unpack_h2(uint32_t b) {
  const _Float16 lo = __builtin_bit_cast(_Float16, (unsigned short)(b & 0xffffu));
  const _Float16 hi = __builtin_bit_cast(_Float16, (unsigned short)(b >> 16));
  return make_float2((float)lo, (float)hi);
}
__device__ __forceinline__ uint32_t pack_h2(double re, double im) {
  const unsigned short lo = __builtin_bit_cast(unsigned short, (_Float16)re);
  const unsigned short hi = __builtin_bit_cast(unsigned short, (_Float16)im);
  return (uint32_t)lo | ((uint32_t)hi << 16);
}
// a stored matrix entry as a vector of the arithmetic type
__device__ __forceinline__ double2 as_vec(double2 v) { return v; }
__device__ __forceinline__ float2 as_vec(float2 v) { return v; }
__device__ __forceinline__ float2 as_vec(uint32_t v) { return unpack_h2(v); }

// ---- storage-type helpers: complex128 (double2) or complex64 (float2) ----
__device__ __forceinline__ double2 ld2(double2 a) { return a; }
__device__ __forceinline__ double2 ld2(float2 a) { return make_double2(a.x, a.y); }
template <class T> __device__ __forceinline__ T st2(double2 a);
template <> __device__ __forceinline__ double2 st2<double2>(double2 a) { return a; }
template <> __device__ __forceinline__ float2 st2<float2>(double2 a) { return make_float2((float)a.x, (float)a.y); }
__device__ __forceinline__ double2 ld2(hbasis a) {
  const float2 f = unpack_h2(a.b);
  return make_double2((double)f.x * (1.0 / 16384.0), (double)f.y * (1.0 / 16384.0));
}
template <> __device__ __forceinline__ hbasis st2<hbasis>(double2 a) {
  return hbasis{pack_h2(a.x * 16384.0, a.y * 16384.0)};
}
template <class T> __device__ __forceinline__ T zero2();
template <> __device__ __forceinline__ double2 zero2<double2>() { return make_double2(0.0, 0.0); }
template <> __device__ __forceinline__ float2 zero2<float2>() { return make_float2(0.f, 0.f); }
// acc + a * b in the storage precision
template <class T> __device__ __forceinline__ T cfmaT(T a, T b, T acc) {
  acc.x = fma(a.x, b.x, fma(-a.y, b.y, acc.x));
  acc.y = fma(a.x, b.y, fma(a.y, b.x, acc.y));
  return acc;
}


// ---- row groups: rows_of<T>::R consecutive entries of one vector moved
// with 16-byte accesses (the first entry 16-byte aligned).  Complex-half
// entries come back as stored, i.e. times 2^14; basis_unscale<T>() is the
// factor that undoes it (1 for the other types), applied by the caller
// once per sum instead of once per entry.
template <class T> struct rows_of;
template <> struct rows_of<double2> { static constexpr int R = 2; };
template <> struct rows_of<float2> { static constexpr int R = 4; };
template <> struct rows_of<hbasis> { static constexpr int R = 4; };
template <class T> __device__ __forceinline__ constexpr double basis_unscale() { return 1.0; }
template <> __device__ __forceinline__ constexpr double basis_unscale<hbasis>() { return 1.0 / 16384.0; }
__device__ __forceinline__ double2 raw2(double2 a) { return a; }
__device__ __forceinline__ double2 raw2(float2 a) { return make_double2(a.x, a.y); }
__device__ __forceinline__ double2 raw2(hbasis a) {
  const float2 f = unpack_h2(a.b);
  return make_double2(f.x, f.y);
}
__device__ __forceinline__ void ld_rows(const double2* __restrict__ p, double2* o) {
  o[0] = p[0];
  o[1] = p[1];
}
__device__ __forceinline__ void ld_rows(const float2* __restrict__ p, double2* o) {
  const float4 a = reinterpret_cast<const float4*>(p)[0], b = reinterpret_cast<const float4*>(p)[1];
  o[0] = make_double2(a.x, a.y);
  o[1] = make_double2(a.z, a.w);
  o[2] = make_double2(b.x, b.y);
  o[3] = make_double2(b.z, b.w);
}
__device__ __forceinline__ void ld_rows(const hbasis* __restrict__ p, double2* o) {
  const uint4 u = *reinterpret_cast<const uint4*>(p);
  o[0] = raw2(hbasis{u.x});
  o[1] = raw2(hbasis{u.y});
  o[2] = raw2(hbasis{u.z});
  o[3] = raw2(hbasis{u.w});
}
// stores take true values (complex-half entries are scaled here)
__device__ __forceinline__ void st_rows(double2* __restrict__ p, const double2* x) {
  p[0] = x[0];
  p[1] = x[1];
}
__device__ __forceinline__ void st_rows(float2* __restrict__ p, const double2* x) {
  reinterpret_cast<float4*>(p)[0] = make_float4((float)x[0].x, (float)x[0].y, (float)x[1].x, (float)x[1].y);
  reinterpret_cast<float4*>(p)[1] = make_float4((float)x[2].x, (float)x[2].y, (float)x[3].x, (float)x[3].y);
}
__device__ __forceinline__ void st_rows(hbasis* __restrict__ p, const double2* x) {
  *reinterpret_cast<uint4*>(p) = make_uint4(st2<hbasis>(x[0]).b, st2<hbasis>(x[1]).b, st2<hbasis>(x[2]).b,
                                            st2<hbasis>(x[3]).b);
}
// the same row groups as complex64 (complex-half and complex64 storage only)
__device__ __forceinline__ void ld_rows(const float2* __restrict__ p, float2* o) {
  const float4 a = reinterpret_cast<const float4*>(p)[0], b = reinterpret_cast<const float4*>(p)[1];
  o[0] = make_float2(a.x, a.y);
  o[1] = make_float2(a.z, a.w);
  o[2] = make_float2(b.x, b.y);
  o[3] = make_float2(b.z, b.w);
}
__device__ __forceinline__ void ld_rows(const hbasis* __restrict__ p, float2* o) {
  const uint4 u = *reinterpret_cast<const uint4*>(p);
  o[0] = unpack_h2(u.x);
  o[1] = unpack_h2(u.y);
  o[2] = unpack_h2(u.z);
  o[3] = unpack_h2(u.w);
}
__device__ __forceinline__ float2 rawf(float2 a) { return a; }
__device__ __forceinline__ float2 rawf(hbasis a) { return unpack_h2(a.b); }
__device__ __forceinline__ float2 cfma_conj(float2 a, float2 b, float2 acc) {
  acc.x = fmaf(a.x, b.x, fmaf(a.y, b.y, acc.x));
  acc.y = fmaf(a.x, b.y, fmaf(-a.y, b.x, acc.y));
  return acc;
}
// per-thread partial sums of the fused dots: complex64 when the direction is
// complex64 (a thread sums a few row groups; every wider sum is FP64)
template <class T> struct dot_acc { using type = double2; };
template <> struct dot_acc<float2> { using type = float2; };
__device__ __forceinline__ void to_acc(double2 a, double2& o) { o = a; }
__device__ __forceinline__ void to_acc(double2 a, float2& o) { o = make_float2((float)a.x, (float)a.y); }
__device__ __forceinline__ double2 raw_as(double2 a, double2) { return a; }
__device__ __forceinline__ double2 raw_as(float2 a, double2) { return raw2(a); }
__device__ __forceinline__ double2 raw_as(hbasis a, double2) { return raw2(a); }
__device__ __forceinline__ float2 raw_as(float2 a, float2) { return a; }
__device__ __forceinline__ float2 raw_as(hbasis a, float2) { return rawf(a); }
