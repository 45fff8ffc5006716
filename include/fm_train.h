/*
 * fm_train.h -- learned coarse propagator of libfm: network kernels, fitting
 * features and model installation.
 *
 * The classical parareal algorithm (Sec. 2, Alg. 1 of Chehab & Petcu) accepts
 * any cheap coarse propagator G.  The library's learned G is the polynomial
 * step X+ = X p(K) + q(K), K = h (A - I) X (inverse homotopy) or
 * K = h (A X - I) (steady inverse flow X' = X - X A X, centred on its root),
 * p and q cubic with coefficients c = c_Euler + y, c_Euler = (1, -1, 0, ...)
 * (forward Euler), where y (8 values) comes from a network of the inputs
 * x = (t, h, mu_1..mu_4), mu_j = tr((A - I)^j) / n: standardised
 * z = (x - mean) / std, three tanh layers of width 64, linear output.
 * Weights: 9288 values, layer by layer, W (out x in, row-major) then b.
 *
 * All pointers below are device pointers (FP32 network data, FP64 fitting
 * data) unless marked host; arrays are row-major with the sample index
 * slowest.  Calls are asynchronous on hip_stream except where noted.
 * Errors: FM_ERR_INVALID for NULL pointers / negative sizes, FM_ERR_DEVICE
 * for launch failures (see fm_last_error()).
 */
#ifndef FM_TRAIN_H
#define FM_TRAIN_H

#include "fm.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Number of network parameters (9288). */
int32_t fm_mlp_param_count(void);

/* Y (S x 8) = network(X (S x 6)) with weights theta (9288) and norm
 * (12: mean[6] then std[6]).  acts: NULL or S x 192 (the three hidden layers,
 * kept for fm_mlp_backward). */
fm_status fm_mlp_forward(const float* theta, const float* norm, const float* X, int64_t S, float* Y, float* acts,
                         void* hip_stream);

/* Fitting loss of the step family for coefficients c = cbase + Y:
 *   L_s = (Y_s^T G_s Y_s - 2 bD_s^T Y_s + fD_s) / fn_s + rho |c_s,4..7|^2,
 * with the defect data written relative to cbase (bD = b - G cbase,
 * fD = f - 2 b^T cbase + cbase^T G cbase; G S x 64, bD S x 8, fD and fn S, FP64)
 * as produced by fm_learned_features.  Writes dY = dL/dY / S (S x 8), the
 * per-sample losses Ls (S, FP64) and, if Lsum is not NULL, their sum (1). */
fm_status fm_mlp_loss(const float* Y, const float* cbase, const double* G, const double* bD, const double* fD,
                      const double* fn, float rho, int64_t S, float* dY, double* Ls, double* Lsum,
                      void* hip_stream);

/* grad (9288) = d(sum_s L_s / S)/d theta by back-propagation of dY through the
 * network evaluated by fm_mlp_forward (its X and acts); deltas: scratch
 * S x 192.  The sample sums run in 32 parallel classes whose partial sums sit
 * in a fixed device array of the library: calls on one GPU must not overlap. */
fm_status fm_mlp_backward(const float* theta, const float* norm, const float* X, const float* acts,
                          const float* dY, int64_t S, float* deltas, float* grad, void* hip_stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) at 1-based step t. */
fm_status fm_mlp_adam(float* theta, const float* grad, float* m, float* v, int64_t count, int32_t t, float lr,
                      void* hip_stream);

/* Fitting data of the step family for state/target pairs, one per problem b
 * of the flow: the basis E = (X, X K, X K^2, X K^3, I, K, K^2, K^3), K as
 * above, built with FP64 products; D = FX - sum_a cE_a E_a (cE: Euler coefficients).
 * Row row0 + b of the outputs receives G_ab = <E_a, E_b>_F (64), bD_a =
 * <E_a, D>_F (8), fD = ||D||_F^2 and fn = ||FX||_F^2.  X, FX: host arrays of
 * device n x n FP64 matrices.  Only for the inverse flows. */
fm_status fm_learned_features(fm_flow f, double h, const double* const* X, const double* const* FX, double* G,
                              double* bD, double* fD, double* fn, int64_t row0, void* hip_stream);

/* mu_j = tr((A - I)^j) / n, j = 1..4, of every problem (host out, batch x 4;
 * synchronous). */
fm_status fm_trace_moments(fm_flow f, double* mu_host, void* hip_stream);

/* Install network weights (host theta[9288], host norm[12]) as the flow's
 * learned coarse step (the same as option coarse_model=<file>). */
fm_status fm_flow_set_coarse_model(fm_flow f, int32_t kind, const double* theta_host, const double* norm_host);

#ifdef __cplusplus
}
#endif

#endif /* FM_TRAIN_H */
