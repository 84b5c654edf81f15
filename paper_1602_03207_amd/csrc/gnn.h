// Launch wrappers of the learned coarse correction (gnn.hip).  All launches
// are asynchronous on `st`; sizes are fixed by the constants in internal.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace eddy {

// Per-subdomain sums over the DOFs of each subdomain, in the block order
// (perm = block DOF list, sub_ptr[P+1] = ranges in it): for each subdomain
// |r|^2, |z|^2, conj(z).r, and, if e != nullptr, conj(z).(e - z) and |e|^2,
// with r_i taken as r_i rs_i and e_i as (e_i - eb_i) / es_i where rs, eb, es
// are non-null.
// out: kGnnP x 4 double2 [rr, zz, zr, zd] + one double2 (sum |e|^2) at index
// 4 * kGnnP.  partial: kGnnP * kGnnStatParts * 5 double2.
constexpr int kGnnStatParts = 64;
template <class T>
void launch_gnn_stats(const int* perm, const int* sub_ptr, const T* r, const T* z, const T* e, const T* eb,
                      const double* rs, const double* es, double2* partial, double2* out, hipStream_t st);
// out = s b - y
void launch_scaled_residual(int64_t n, const double2* b, const double* s, const double2* y, double2* out,
                            hipStream_t st);
// words of per-sample scratch of the network kernels
int gnn_scratch_floats();
// Features X [P x Fin] (float32) from the sums and the static columns
// (static4 [P x 4]); with targets, c* [P x 2] and w [P] (float32).
void launch_gnn_features(const double2* sums, const float* static4, int with_targets, float* X, float* cstar,
                         float* w, hipStream_t st);
// Network forward for nsamp samples (X, Y at stride P x Fin / P x Fout):
// Y = f(theta; A_hat, X).  scratch: nsamp * kGnnScratch floats.
void launch_gnn_forward(int nsamp, const float* theta, const uint16_t* ahat, const float* X, float* Y,
                        float* scratch, hipStream_t st);
// Training: per-sample forward, loss and backward (grads [nsamp x kGnnParams],
// loss [nsamp]), then the batch-mean gradient (written to gmean if non-null)
// and one Adam step on theta, m, v (skipped if lr == 0).
void launch_gnn_train(int nsamp, float* theta, float* m, float* v, const uint16_t* ahat, const float* X,
                      const float* cstar, const float* w, float* scratch, float* grads, float* loss, float* gmean,
                      int step, float lr, hipStream_t st);
// z[perm[q]] *= (1 + c_p) over subdomain p's range (c_p = Y[p][0] + i Y[p][1]).
template <class T>
void launch_gnn_scale(const int* perm, const int* sub_ptr, const float* Y, T* z, hipStream_t st);

}  // namespace eddy
