// Kernels of the learned coarse step: the coefficient network (forward, loss,
// backward, Adam) in FP32, the FP64 fitting features of the polynomial step
// family, and the trace moments of A - I.
//
// Network: z = (x - mean) / std (x = (t, h, mu1..mu4)), three tanh hidden
// layers of width 64, linear output of 8; flat weights layer by layer
// (W out x in row-major, then b).  One thread evaluates one sample with all
// weights staged in LDS (37 KB, broadcast reads).  Weight gradients are sums
// over samples: WG_CH sample classes (s mod WG_CH) are summed in parallel,
// one parameter per thread in sample order, then the class sums are added
// in class order (deterministic, no atomics).
#include "fm_common.h"
#include "fm_mlp.h"

namespace fm {
namespace {

constexpr int NI = 6, NH = 64, NO = 8;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + NH * NI;
constexpr int OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH;
constexpr int OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NH * NH;
constexpr int OFF_W4 = OFF_B3 + NH, OFF_B4 = OFF_W4 + NO * NH;
constexpr int NPARAM = OFF_B4 + NO;
static_assert(NPARAM == 9288, "parameter count");

constexpr int MT = 128;  // threads (samples) per block

__device__ __forceinline__ void load_weights(float* w, const float* __restrict__ theta) {
  for (int i = threadIdx.x; i < NPARAM; i += blockDim.x) w[i] = theta[i];
  __syncthreads();
}

// acts layout per sample: h1[64] h2[64] h3[64]
__global__ __launch_bounds__(MT) void k_mlp_fwd(const float* __restrict__ theta, const float* __restrict__ norm,
                                                const float* __restrict__ X, int64_t S, float* __restrict__ Y,
                                                float* __restrict__ acts) {
  __shared__ float w[NPARAM];
  load_weights(w, theta);
  const int64_t s = blockIdx.x * (int64_t)MT + threadIdx.x;
  if (s >= S) return;
  float z[NI], a[NH], b[NH];
  for (int i = 0; i < NI; ++i) z[i] = (X[s * NI + i] - norm[i]) / norm[NI + i];
  for (int o = 0; o < NH; ++o) {
    float v = w[OFF_B1 + o];
    for (int i = 0; i < NI; ++i) v += w[OFF_W1 + o * NI + i] * z[i];
    a[o] = tanhf(v);
  }
  if (acts) for (int o = 0; o < NH; ++o) acts[s * 3 * NH + o] = a[o];
  for (int o = 0; o < NH; ++o) {
    float v = w[OFF_B2 + o];
    for (int i = 0; i < NH; ++i) v += w[OFF_W2 + o * NH + i] * a[i];
    b[o] = tanhf(v);
  }
  if (acts) for (int o = 0; o < NH; ++o) acts[s * 3 * NH + NH + o] = b[o];
  for (int o = 0; o < NH; ++o) {
    float v = w[OFF_B3 + o];
    for (int i = 0; i < NH; ++i) v += w[OFF_W3 + o * NH + i] * b[i];
    a[o] = tanhf(v);
  }
  if (acts) for (int o = 0; o < NH; ++o) acts[s * 3 * NH + 2 * NH + o] = a[o];
  for (int o = 0; o < NO; ++o) {
    float v = w[OFF_B4 + o];
    for (int i = 0; i < NH; ++i) v += w[OFF_W4 + o * NH + i] * a[i];
    Y[s * NO + o] = v;
  }
}

// Per-sample loss and dL/dY for c = cbase + Y with the defect data written
// relative to cbase: G (8x8), bD = b - G cbase, fD = f - 2 b.cbase + cbase.G.cbase
// (all FP64), fn = f:
//   L_s = (dc^T G dc - 2 bD^T dc + fD) / fn + rho |c_q|^2,  dc = Y,
//   dL/dY = [2 (G dc - bD) / fn + 2 rho Dq c] / S.
__global__ void k_mlp_loss(const float* __restrict__ Y, const float* __restrict__ cbase,
                           const double* __restrict__ G, const double* __restrict__ bD,
                           const double* __restrict__ fD, const double* __restrict__ fn, float rho, int64_t S,
                           float* __restrict__ dY, double* __restrict__ Ls) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= S) return;
  double dc[NO], c[NO];
  for (int a = 0; a < NO; ++a) {
    dc[a] = Y[s * NO + a];
    c[a] = cbase[s * NO + a] + dc[a];
  }
  const double* g = G + s * 64;
  double quad = 0.0, lin = 0.0, pen = 0.0;
  double gd[NO];
  for (int a = 0; a < NO; ++a) {
    double v = 0.0;
    for (int b2 = 0; b2 < NO; ++b2) v += g[a * NO + b2] * dc[b2];
    gd[a] = v;
    quad += dc[a] * v;
    lin += bD[s * NO + a] * dc[a];
  }
  for (int a = 4; a < NO; ++a) pen += c[a] * c[a];
  const double f = fn[s];
  Ls[s] = (quad - 2.0 * lin + fD[s]) / f + rho * pen;
  for (int a = 0; a < NO; ++a) {
    double d = 2.0 * (gd[a] - bD[s * NO + a]) / f;
    if (a >= 4) d += 2.0 * rho * c[a];
    dY[s * NO + a] = (float)(d / (double)S);
  }
}

// Per-sample back-propagated deltas of the hidden layers: d3, d2, d1 (S x 64 each).
__global__ __launch_bounds__(MT) void k_mlp_delta(const float* __restrict__ theta, const float* __restrict__ acts,
                                                  const float* __restrict__ dY, int64_t S,
                                                  float* __restrict__ deltas) {
  __shared__ float w[NPARAM];
  load_weights(w, theta);
  const int64_t s = blockIdx.x * (int64_t)MT + threadIdx.x;
  if (s >= S) return;
  const float* h = acts + s * 3 * NH;
  float d[NH], e[NH];
  for (int i = 0; i < NH; ++i) {
    float v = 0.f;
    for (int o = 0; o < NO; ++o) v += dY[s * NO + o] * w[OFF_W4 + o * NH + i];
    d[i] = v * (1.f - h[2 * NH + i] * h[2 * NH + i]);
  }
  for (int i = 0; i < NH; ++i) deltas[s * 3 * NH + 2 * NH + i] = d[i];
  for (int i = 0; i < NH; ++i) {
    float v = 0.f;
    for (int o = 0; o < NH; ++o) v += d[o] * w[OFF_W3 + o * NH + i];
    e[i] = v * (1.f - h[NH + i] * h[NH + i]);
  }
  for (int i = 0; i < NH; ++i) deltas[s * 3 * NH + NH + i] = e[i];
  for (int i = 0; i < NH; ++i) {
    float v = 0.f;
    for (int o = 0; o < NH; ++o) v += e[o] * w[OFF_W2 + o * NH + i];
    d[i] = v * (1.f - h[i] * h[i]);
  }
  for (int i = 0; i < NH; ++i) deltas[s * 3 * NH + i] = d[i];
}

// Weight gradients as sums over samples:
//   layer l: gW[o][i] = sum_s delta_l[s][o] * in_l[s][i], gb[o] = sum_s delta_l[s][o]
// with in_1 = z (standardised inputs), in_l = h_{l-1}; delta_4 = dY.
// Stage 1, grid (parameter blocks, WG_CH): block (b, c) sums samples
// s = c, c + WG_CH, ... for its parameters into g_wgrad_part[c][p]; the
// threads of a block read neighbouring entries of one sample row at a time.
// Stage 2 adds the WG_CH partial sums of each parameter in class order.
// The partial sums live in a fixed device array: backward calls on one GPU
// must not overlap.
constexpr int WG_CH = 32;
__device__ double g_wgrad_part[WG_CH * NPARAM];

__global__ __launch_bounds__(256) void k_mlp_wgrad_part(const float* __restrict__ norm, const float* __restrict__ X,
                                                        const float* __restrict__ acts,
                                                        const float* __restrict__ deltas,
                                                        const float* __restrict__ dY, int64_t S) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (p >= NPARAM) return;
  int layer, o, i;
  bool bias;
  if (p < OFF_B1) { layer = 1; o = p / NI; i = p % NI; bias = false; }
  else if (p < OFF_W2) { layer = 1; o = p - OFF_B1; i = 0; bias = true; }
  else if (p < OFF_B2) { layer = 2; o = (p - OFF_W2) / NH; i = (p - OFF_W2) % NH; bias = false; }
  else if (p < OFF_W3) { layer = 2; o = p - OFF_B2; i = 0; bias = true; }
  else if (p < OFF_B3) { layer = 3; o = (p - OFF_W3) / NH; i = (p - OFF_W3) % NH; bias = false; }
  else if (p < OFF_W4) { layer = 3; o = p - OFF_B3; i = 0; bias = true; }
  else if (p < OFF_B4) { layer = 4; o = (p - OFF_W4) / NH; i = (p - OFF_W4) % NH; bias = false; }
  else { layer = 4; o = p - OFF_B4; i = 0; bias = true; }
  double acc = 0.0;
  for (int64_t s = c; s < S; s += WG_CH) {
    const float dv = layer == 4 ? dY[s * NO + o] : deltas[s * 3 * NH + (layer - 1) * NH + o];
    float in = 1.f;
    if (!bias) {
      if (layer == 1) in = (X[s * NI + i] - norm[i]) / norm[NI + i];
      else in = acts[s * 3 * NH + (layer - 2) * NH + i];
    }
    acc += (double)dv * (double)in;
  }
  g_wgrad_part[(int64_t)c * NPARAM + p] = acc;
}

__global__ __launch_bounds__(256) void k_mlp_wgrad_sum(float* __restrict__ grad) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NPARAM) return;
  double acc = 0.0;
  for (int c = 0; c < WG_CH; ++c) acc += g_wgrad_part[(int64_t)c * NPARAM + p];
  grad[p] = (float)acc;
}

__global__ void k_adam(float* __restrict__ theta, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t count, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  theta[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Fixed-order sum of per-sample losses: one block.
__global__ void k_sum(const double* __restrict__ x, int64_t S, double* __restrict__ out) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < S; i += 256) s += x[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

// ---- fitting features ------------------------------------------------------
// For one sample: basis E = (X, X K, X K^2, X K^3, I, K, K^2, K^3) (FP64,
// np x np), target F, Euler member cE; D = F - sum_a cE_a E_a.
// Outputs G_ab = <E_a, E_b>, bD_a = <E_a, D>, fD = <D, D>, fn = <F, F>.
// grid = (nblk, nitems); partial sums of the 36 + 8 + 2 = 46 products per block.
constexpr int NFEAT = 46;

__global__ __launch_bounds__(256) void k_features_part(const FeatItem* __restrict__ items, double* __restrict__ part) {
  const FeatItem it = items[blockIdx.y];
  double acc[NFEAT];
  for (int q = 0; q < NFEAT; ++q) acc[q] = 0.0;
  const int np = it.np, n = it.n;
  const int64_t count = (int64_t)np * np;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / np, c = e % np;
    double E[8];
    E[0] = it.x[e];
    E[1] = it.xk[0][e];
    E[2] = it.xk[1][e];
    E[3] = it.xk[2][e];
    E[4] = (r == c && r < n) ? 1.0 : 0.0;
    E[5] = it.k[0][e];
    E[6] = it.k[1][e];
    E[7] = it.k[2][e];
    const double F = it.f[e];
    double D = F;
    for (int a = 0; a < 8; ++a) D -= it.ce[a] * E[a];
    int q = 0;
    for (int a = 0; a < 8; ++a)
      for (int b = a; b < 8; ++b) acc[q++] += E[a] * E[b];
    for (int a = 0; a < 8; ++a) acc[q++] += E[a] * D;
    acc[q++] += D * D;
    acc[q++] += F * F;
  }
  __shared__ double sh[256];
  for (int q = 0; q < NFEAT; ++q) {
    sh[threadIdx.x] = acc[q];
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
      if ((int)threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * NFEAT + q] = sh[0];
    __syncthreads();
  }
}

// grid = nitems: reduce the partials of item j in block order and scatter
// into the output arrays at row it.out.
__global__ void k_features_reduce(const FeatItem* __restrict__ items, const double* __restrict__ part, int nblk,
                                  double* __restrict__ G, double* __restrict__ bD, double* __restrict__ fD,
                                  double* __restrict__ fn) {
  const FeatItem it = items[blockIdx.x];
  const int q = threadIdx.x;
  if (q >= NFEAT) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += part[((int64_t)blockIdx.x * nblk + b) * NFEAT + q];
  const int64_t row = it.out;
  if (q < 36) {
    int a = 0, qq = q;
    while (qq >= 8 - a) { qq -= 8 - a; ++a; }
    const int b = a + qq;
    G[row * 64 + a * 8 + b] = s;
    G[row * 64 + b * 8 + a] = s;
  } else if (q < 44) {
    bD[row * 8 + (q - 36)] = s;
  } else if (q == 44) {
    fD[row] = s;
  } else {
    fn[row] = s;
  }
}

// tr(M), tr(M^2), tr(M^3), tr(M^4) from M and M2 = M M (np x np, FP64):
// tr(M^3) = sum_ij M2_ij M_ji, tr(M^4) = sum_ij M2_ij M2_ji.  One block.
__global__ void k_trace_moments(const double* __restrict__ M, const double* __restrict__ M2, int n, int np,
                                double* __restrict__ out) {
  __shared__ double sh[256];
  double acc[4] = {0, 0, 0, 0};
  for (int64_t e = threadIdx.x; e < (int64_t)n * n; e += 256) {
    const int64_t i = e / n, j = e % n;
    const double mij = M[i * np + j], mji = M[j * np + i];
    const double m2ij = M2[i * np + j], m2ji = M2[j * np + i];
    if (i == j) {
      acc[0] += mij;
      acc[1] += m2ij;
    }
    acc[2] += m2ij * mji;
    acc[3] += m2ij * m2ji;
  }
  for (int q = 0; q < 4; ++q) {
    sh[threadIdx.x] = acc[q];
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
      if ((int)threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[q] = sh[0] / n;
    __syncthreads();
  }
}

}  // namespace

int mlp_param_count() { return NPARAM; }

hipError_t mlp_forward(const float* theta, const float* norm, const float* X, int64_t S, float* Y, float* acts,
                       hipStream_t st) {
  if (S <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_fwd, dim3((S + MT - 1) / MT), dim3(MT), 0, st, theta, norm, X, S, Y, acts);
  return hipGetLastError();
}

hipError_t mlp_loss(const float* Y, const float* cbase, const double* G, const double* bD, const double* fD,
                    const double* fn, float rho, int64_t S, float* dY, double* Ls, double* Lsum, hipStream_t st) {
  if (S <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_loss, dim3((S + 255) / 256), dim3(256), 0, st, Y, cbase, G, bD, fD, fn, rho, S, dY, Ls);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !Lsum) return e;
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, st, Ls, S, Lsum);
  return hipGetLastError();
}

hipError_t mlp_backward(const float* theta, const float* norm, const float* X, const float* acts, const float* dY,
                        int64_t S, float* deltas, float* grad, hipStream_t st) {
  if (S <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_delta, dim3((S + MT - 1) / MT), dim3(MT), 0, st, theta, acts, dY, S, deltas);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mlp_wgrad_part, dim3((NPARAM + 255) / 256, WG_CH), dim3(256), 0, st, norm, X, acts, deltas,
                     dY, S);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mlp_wgrad_sum, dim3((NPARAM + 255) / 256), dim3(256), 0, st, grad);
  return hipGetLastError();
}

hipError_t mlp_adam(float* theta, const float* g, float* m, float* v, int64_t count, int t, float lr, float b1,
                    float b2, float eps, hipStream_t st) {
  const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
  hipLaunchKernelGGL(k_adam, dim3((count + 255) / 256), dim3(256), 0, st, theta, g, m, v, count, lr, b1, b2, eps,
                     c1, c2);
  return hipGetLastError();
}

hipError_t features(const FeatItem* items, int nitems, double* part, int nblk, double* G, double* bD, double* fD,
                    double* fn, hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_features_part, dim3(nblk, nitems), dim3(256), 0, st, items, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_features_reduce, dim3(nitems), dim3(64), 0, st, items, part, nblk, G, bD, fD, fn);
  return hipGetLastError();
}

hipError_t trace_moments(const double* M, const double* M2, int n, int np, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_trace_moments, dim3(1), dim3(256), 0, st, M, M2, n, np, out);
  return hipGetLastError();
}

}  // namespace fm
