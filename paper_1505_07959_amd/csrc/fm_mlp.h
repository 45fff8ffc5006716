// Internal declarations of the learned-coarse kernels (mlp.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fm {

int mlp_param_count();

// Y (S x 8) = net(X (S x 6)); acts (S x 192: h1|h2|h3) may be null.
hipError_t mlp_forward(const float* theta, const float* norm, const float* X, int64_t S, float* Y, float* acts,
                       hipStream_t st);
// per-sample loss Ls (S) and dL/dY (S x 8); Lsum (1) = sum of Ls when non-null
hipError_t mlp_loss(const float* Y, const float* cbase, const double* G, const double* bD, const double* fD,
                    const double* fn, float rho, int64_t S, float* dY, double* Ls, double* Lsum, hipStream_t st);
// grad (9288) of the batch loss; deltas: scratch S x 192
hipError_t mlp_backward(const float* theta, const float* norm, const float* X, const float* acts, const float* dY,
                        int64_t S, float* deltas, float* grad, hipStream_t st);
hipError_t mlp_adam(float* theta, const float* g, float* m, float* v, int64_t count, int t, float lr, float b1,
                    float b2, float eps, hipStream_t st);

// One fitting sample: basis X, X K^j (j = 1..3), K^j (j = 1..3), target f
// (all FP64 np x np), Euler coefficients ce; results go to row `out`.
struct FeatItem {
  const double* x;
  const double* xk[3];
  const double* k[3];
  const double* f;
  double ce[8];
  int np;
  int n;
  int64_t out;
};
// G (rows x 64), bD (rows x 8), fD (rows), fn (rows); part: nitems*nblk*46 doubles
hipError_t features(const FeatItem* items, int nitems, double* part, int nblk, double* G, double* bD, double* fD,
                    double* fn, hipStream_t st);
// out[0..3] = tr(M^j) / n, j = 1..4 (M2 = M M)
hipError_t trace_moments(const double* M, const double* M2, int n, int np, double* out, hipStream_t st);

}  // namespace fm
