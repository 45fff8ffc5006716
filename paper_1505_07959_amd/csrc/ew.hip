// Elementwise and reduction kernels of libfm: staging of A, identity/copies,
// the FP64 parareal correction with its increment norms, and deterministic
// FP64 dot products for the refinement.  All are HBM-bound streams; they use
// grid-stride loops over 16-byte-aligned FP64 data and fixed-order reductions
// (one partial per block, reduced by a single block in block order).
#include "fm_common.h"

namespace fm {
namespace {

constexpr int EW_THREADS = 256;

inline int ew_grid(int64_t count) {
  int64_t g = (count + EW_THREADS * 4 - 1) / (EW_THREADS * 4);
  if (g < 1) g = 1;
  if (g > 8192) g = 8192;
  return (int)g;
}

__global__ void k_stage_pad(double* __restrict__ dst, int np, const double* __restrict__ src, int64_t n,
                            int64_t ld) {
  const int64_t total = (int64_t)np * np;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / np, j = e % np;
    dst[e] = (i < n && j < n) ? src[i * ld + j] : 0.0;
  }
}

template <class T>
__device__ __forceinline__ T cvt(double v) { return (T)v; }
template <>
__device__ __forceinline__ __bf16 cvt<__bf16>(double v) { return (__bf16)(float)v; }
template <>
__device__ __forceinline__ _Float16 cvt<_Float16>(double v) { return (_Float16)(float)v; }

// operand-type store; SPLIT: hi plane at e, lo plane at e + plane
template <class T, bool SPLIT>
__device__ __forceinline__ void st_cvt(T* dst, int64_t e, int64_t plane, double v) {
  const T hi = cvt<T>(v);
  dst[e] = hi;
  if constexpr (SPLIT) dst[e + plane] = cvt<T>(v - (double)(float)hi);
}

template <class T, bool SPLIT = false>
__global__ void k_convert(T* __restrict__ dst, const double* __restrict__ src, double shift, int n, int np) {
  const int64_t total = (int64_t)np * np;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / np, j = e % np;
    double v = src[e];
    if (i == j && i < n) v += shift;
    st_cvt<T, SPLIT>(dst, e, total, v);
  }
}

template <class T, bool SPLIT = false>
__global__ void k_prep(const PrepItem* __restrict__ items, const int* __restrict__ live) {
  const PrepItem it = items[blockIdx.y];
  if (live != nullptr && live[it.inst] == 0) return;
  T* y = (T*)it.y;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < it.count; e += (int64_t)gridDim.x * blockDim.x) {
    const double v = it.u[e];
    if (it.fo) it.fo[e] = v;
    st_cvt<T, SPLIT>(y, e, it.count, v);
  }
}

__global__ void k_cast(const CastItem* __restrict__ items) {
  const CastItem it = items[blockIdx.y];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  if (it.narrow) {
    const double* s = (const double*)it.src;
    float* d = (float*)it.dst;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < it.count; e += stride) d[e] = (float)s[e];
  } else {
    const float* s = (const float*)it.src;
    double* d = (double*)it.dst;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < it.count; e += stride) d[e] = (double)s[e];
  }
}

template <class T>
__global__ void k_fill(T* __restrict__ dst, int64_t count) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = cvt<T>(0.25 + 0.001 * (double)((e * 2654435761ll) % 1000));
}

__global__ void k_identity(double* __restrict__ dst, int n, int np) {
  const int64_t total = (int64_t)np * np;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / np, j = e % np;
    dst[e] = (i == j && i < n) ? 1.0 : 0.0;
  }
}

__global__ void k_copy_in(double* __restrict__ dst, int np, const double* __restrict__ src, int n) {
  const int64_t total = (int64_t)np * np;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / np, j = e % np;
    dst[e] = (i < n && j < n) ? src[i * n + j] : 0.0;
  }
}

__global__ void k_copy_out(double* __restrict__ dst, int n, const double* __restrict__ src, int np) {
  const int64_t total = (int64_t)n * n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / n, j = e % n;
    dst[e] = src[i * np + j];
  }
}

__global__ void k_pad_copy(const PadItem* __restrict__ items, int pad) {
  const PadItem it = items[blockIdx.y];
  if (pad) {
    const int64_t total = (int64_t)it.np * it.np;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
      const int64_t i = e / it.np, j = e % it.np;
      it.dst[e] = (i < it.n && j < it.n) ? it.src[i * it.n + j] : 0.0;
    }
  } else {
    const int64_t total = (int64_t)it.n * it.n;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
      const int64_t i = e / it.n, j = e % it.n;
      it.dst[e] = it.src[i * it.np + j];
    }
  }
}

__global__ void k_copy(double* __restrict__ dst, const double* __restrict__ src, int64_t count) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = src[e];
}

// Block-wide sum in a fixed order (tree over the 256 lanes).
__device__ __forceinline__ double block_sum(double v, double* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
#pragma unroll
  for (int s = EW_THREADS / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] += sh[t + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// grid = (nblk, nitems).  U^{k+1}_{n+1} = F + (G_new - G_old), in FP64 and in
// this association, so that G_new == G_old bitwise gives F bitwise.
__global__ void k_correction(const CorrItem* __restrict__ items, double* __restrict__ part,
                             const int* __restrict__ live) {
  __shared__ double sh[EW_THREADS];
  const CorrItem it = items[blockIdx.y];
  const int nblk = gridDim.x;
  double dd = 0.0, uu = 0.0, bad = 0.0;
  if (live == nullptr || live[it.inst] != 0)
  for (int64_t e = blockIdx.x * (int64_t)EW_THREADS + threadIdx.x; e < it.count; e += (int64_t)nblk * EW_THREADS) {
    const double gn = it.gnew[e];
    const double un = it.f[e] + (gn - it.gold[e]);
    const double d = un - it.u[e];
    it.u[e] = un;
    it.gold[e] = gn;
    dd += d * d;
    uu += un * un;
    if (!isfinite(un)) bad = 1.0;
  }
  dd = block_sum(dd, sh);
  uu = block_sum(uu, sh);
  bad = block_sum(bad, sh);
  if (threadIdx.x == 0) {
    double* p = part + ((int64_t)it.slot * nblk + blockIdx.x) * 3;
    p[0] = dd;
    p[1] = uu;
    p[2] = bad;
  }
}

// grid = nitems; sums nblk partial triples of item j in block order.
__global__ void k_reduce_triples(const double* __restrict__ part, int nblk, double* __restrict__ out) {
  __shared__ double sh[EW_THREADS];
  const double* p = part + (int64_t)blockIdx.x * nblk * 3;
  double a = 0, b = 0, c = 0;
  for (int i = threadIdx.x; i < nblk; i += EW_THREADS) {
    a += p[3 * i];
    b += p[3 * i + 1];
    c += p[3 * i + 2];
  }
  a = block_sum(a, sh);
  b = block_sum(b, sh);
  c = block_sum(c, sh);
  if (threadIdx.x == 0) {
    out[3 * blockIdx.x] = a;
    out[3 * blockIdx.x + 1] = b;
    out[3 * blockIdx.x + 2] = c;
  }
}

__global__ void k_dot_part(const double* __restrict__ a, const double* __restrict__ b, int64_t count,
                           double* __restrict__ part) {
  __shared__ double sh[EW_THREADS];
  double s = 0.0;
  for (int64_t e = blockIdx.x * (int64_t)EW_THREADS + threadIdx.x; e < count; e += (int64_t)gridDim.x * EW_THREADS)
    s += a[e] * b[e];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void k_sum_part(const double* __restrict__ part, int nblk, double* __restrict__ out) {
  __shared__ double sh[EW_THREADS];
  double s = 0.0;
  for (int i = threadIdx.x; i < nblk; i += EW_THREADS) s += part[i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) out[0] = s;
}

__global__ void k_axpy_dev(double* __restrict__ y, const double* __restrict__ x, const double* __restrict__ alpha,
                           double sign, int64_t count) {
  const double a = sign * alpha[0];
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x)
    y[e] += a * x[e];
}

// grid = (nblk, nitems)
__global__ void k_dots_part(const DotItem* __restrict__ items, double* __restrict__ part) {
  __shared__ double sh[EW_THREADS];
  const DotItem it = items[blockIdx.y];
  double s = 0.0;
  if (it.mode == 1) {
    for (int64_t e = blockIdx.x * (int64_t)EW_THREADS + threadIdx.x; e < it.count; e += (int64_t)gridDim.x * EW_THREADS)
      s += isfinite(it.a[e]) ? 0.0 : 1.0;
  } else if (it.sub) {
    for (int64_t e = blockIdx.x * (int64_t)EW_THREADS + threadIdx.x; e < it.count; e += (int64_t)gridDim.x * EW_THREADS)
      s += (it.a[e] - it.sub[e]) * (it.b[e] - it.sub[e]);
  } else {
    for (int64_t e = blockIdx.x * (int64_t)EW_THREADS + threadIdx.x; e < it.count; e += (int64_t)gridDim.x * EW_THREADS)
      s += it.a[e] * it.b[e];
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = s;
}

// grid = nitems
__global__ void k_dots_reduce(const DotItem* __restrict__ items, const double* __restrict__ part, int nblk,
                              double* __restrict__ out) {
  __shared__ double sh[EW_THREADS];
  double s = 0.0;
  for (int i = threadIdx.x; i < nblk; i += EW_THREADS) s += part[(int64_t)blockIdx.x * nblk + i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) out[items[blockIdx.x].slot] = s;
}

__global__ void k_cg_init(const CgItem* __restrict__ items) {
  const CgItem it = items[blockIdx.y];
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < it.count; e += (int64_t)gridDim.x * blockDim.x) {
    const double v = it.ap[e];
    it.h[e] = 0.0;
    it.r[e] = v;
    it.p[e] = v;
  }
}

__global__ void k_add(const CgItem* __restrict__ items) {
  const CgItem it = items[blockIdx.y];
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < it.count; e += (int64_t)gridDim.x * blockDim.x)
    it.h[e] += it.ap[e];
}

__global__ void k_cg_step1(const CgItem* __restrict__ items, const double* __restrict__ rr,
                           const double* __restrict__ pap) {
  const CgItem it = items[blockIdx.y];
  const double den = pap[it.slot];
  const double a = den != 0.0 ? rr[it.slot] / den : 0.0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < it.count; e += (int64_t)gridDim.x * blockDim.x) {
    it.h[e] += a * it.p[e];
    it.r[e] -= a * it.ap[e];
  }
}

__global__ void k_cg_step2(const CgItem* __restrict__ items, const double* __restrict__ rr_new,
                           const double* __restrict__ rr) {
  const CgItem it = items[blockIdx.y];
  const double den = rr[it.slot];
  const double b = den != 0.0 ? rr_new[it.slot] / den : 0.0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < it.count; e += (int64_t)gridDim.x * blockDim.x)
    it.p[e] = it.r[e] + b * it.p[e];
}


__global__ void k_lincomb(LinItem it) {
  for (int64_t e = blockIdx.x * (int64_t)EW_THREADS + threadIdx.x; e < it.count; e += (int64_t)gridDim.x * EW_THREADS) {
    if (it.mode == LIN_SCALE) {
      it.out1[e] = it.scale * it.z[e];
      continue;
    }
    if (it.mode == LIN_AXPY) {
      it.out1[e] = it.z[e] + it.scale * it.c[e];
      continue;
    }
    double p = 0.0, f = 0.0;
    for (int j = 0; j < it.s; ++j) {
      const double a = it.alpha[j];
      p += a * it.q[j][e];
      if (it.mode == LIN_SWEEP) f += a * it.fq[j][e];
    }
    const double z = it.z[e];
    it.out1[e] = z - p;
    if (it.mode == LIN_SWEEP) it.out2[e] = it.c ? f + it.c[e] : f;
  }
}


// max_i sum_j |a_ij| of an n x n row-major matrix (leading dimension ld), one
// block; rows are summed in column order, the maximum is order independent.
__global__ void k_norm_inf(const double* __restrict__ a, int64_t n, int64_t ld, double* __restrict__ out) {
  __shared__ double sh[EW_THREADS];
  double m = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += EW_THREADS) {
    double r = 0.0;
    for (int64_t j = 0; j < n; ++j) r += fabs(a[i * ld + j]);
    m = fmax(m, r);
  }
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int s = EW_THREADS / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

// The real form of the sine/cosine system of Sec. 3, Example 3 (X0 = 0):
// out = [[0, -c A], [c A, 0]], 2n x 2n row-major (leading dimension 2n).
__global__ void k_rotation_generator(double* __restrict__ out, const double* __restrict__ a, int64_t n, int64_t ld,
                                     double c) {
  const int64_t m = 2 * n, total = m * m;
  for (int64_t e = blockIdx.x * (int64_t)EW_THREADS + threadIdx.x; e < total; e += (int64_t)gridDim.x * EW_THREADS) {
    const int64_t i = e / m, j = e % m;
    double v = 0.0;
    if (i < n && j >= n) v = -c * a[i * ld + (j - n)];
    else if (i >= n && j < n) v = c * a[(i - n) * ld + j];
    out[e] = v;
  }
}

}  // namespace

hipError_t launch_dots(const DotItem* items, int nitems, double* part, int nblk, double* out, hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_dots_part, dim3(nblk, nitems), dim3(EW_THREADS), 0, st, items, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_dots_reduce, dim3(nitems), dim3(EW_THREADS), 0, st, items, part, nblk, out);
  return hipGetLastError();
}

hipError_t launch_cg_init(const CgItem* items, int nitems, hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cg_init, dim3(64, nitems), dim3(EW_THREADS), 0, st, items);
  return hipGetLastError();
}

hipError_t launch_add(const CgItem* items, int nitems, hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_add, dim3(64, nitems), dim3(EW_THREADS), 0, st, items);
  return hipGetLastError();
}

hipError_t launch_cg_step1(const CgItem* items, int nitems, const double* rr, const double* pap, hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cg_step1, dim3(64, nitems), dim3(EW_THREADS), 0, st, items, rr, pap);
  return hipGetLastError();
}

hipError_t launch_cg_step2(const CgItem* items, int nitems, const double* rr_new, const double* rr,
                           hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cg_step2, dim3(64, nitems), dim3(EW_THREADS), 0, st, items, rr_new, rr);
  return hipGetLastError();
}

hipError_t stage_pad_f64(double* dst, int np, const double* src, int64_t n, int64_t ld, hipStream_t st) {
  hipLaunchKernelGGL(k_stage_pad, dim3(ew_grid((int64_t)np * np)), dim3(EW_THREADS), 0, st, dst, np, src, n, ld);
  return hipGetLastError();
}

hipError_t convert_f64(void* dst, int dt, const double* src, double shift, int n, int np, hipStream_t st) {
  dim3 g(ew_grid((int64_t)np * np)), b(EW_THREADS);
  switch (dt) {
    case DT_F64: hipLaunchKernelGGL(k_convert<double>, g, b, 0, st, (double*)dst, src, shift, n, np); break;
    case DT_F32: hipLaunchKernelGGL(k_convert<float>, g, b, 0, st, (float*)dst, src, shift, n, np); break;
    case DT_BF16: hipLaunchKernelGGL(k_convert<__bf16>, g, b, 0, st, (__bf16*)dst, src, shift, n, np); break;
    case DT_F16: hipLaunchKernelGGL(k_convert<_Float16>, g, b, 0, st, (_Float16*)dst, src, shift, n, np); break;
    case DT_BF16X3:
      hipLaunchKernelGGL((k_convert<__bf16, true>), g, b, 0, st, (__bf16*)dst, src, shift, n, np);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t convert_split_f64(void* dst, int dt, const double* src, double shift, int n, int np, hipStream_t st) {
  dim3 g(ew_grid((int64_t)np * np)), b(EW_THREADS);
  switch (dt) {
    case DT_BF16:
      hipLaunchKernelGGL((k_convert<__bf16, true>), g, b, 0, st, (__bf16*)dst, src, shift, n, np);
      break;
    case DT_F16:
      hipLaunchKernelGGL((k_convert<_Float16, true>), g, b, 0, st, (_Float16*)dst, src, shift, n, np);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t fill_pattern(void* dst, int dt, int64_t count, hipStream_t st) {
  dim3 g(ew_grid(count)), b(EW_THREADS);
  switch (dt) {
    case DT_F64: hipLaunchKernelGGL(k_fill<double>, g, b, 0, st, (double*)dst, count); break;
    case DT_F32: hipLaunchKernelGGL(k_fill<float>, g, b, 0, st, (float*)dst, count); break;
    case DT_BF16: hipLaunchKernelGGL(k_fill<__bf16>, g, b, 0, st, (__bf16*)dst, count); break;
    case DT_F16: hipLaunchKernelGGL(k_fill<_Float16>, g, b, 0, st, (_Float16*)dst, count); break;
    case DT_BF16X3: hipLaunchKernelGGL(k_fill<__bf16>, g, b, 0, st, (__bf16*)dst, 2 * count); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t set_identity(double* dst, int n, int np, hipStream_t st) {
  hipLaunchKernelGGL(k_identity, dim3(ew_grid((int64_t)np * np)), dim3(EW_THREADS), 0, st, dst, n, np);
  return hipGetLastError();
}

hipError_t copy_in(double* dst, int np, const double* src, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_copy_in, dim3(ew_grid((int64_t)np * np)), dim3(EW_THREADS), 0, st, dst, np, src, n);
  return hipGetLastError();
}

hipError_t copy_out(double* dst, int n, const double* src, int np, hipStream_t st) {
  hipLaunchKernelGGL(k_copy_out, dim3(ew_grid((int64_t)n * n)), dim3(EW_THREADS), 0, st, dst, n, src, np);
  return hipGetLastError();
}

hipError_t launch_pad_copy(const PadItem* items, int nitems, int pad, hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pad_copy, dim3(64, nitems), dim3(EW_THREADS), 0, st, items, pad);
  return hipGetLastError();
}

hipError_t copy_f64(double* dst, const double* src, int64_t count, hipStream_t st) {
  hipLaunchKernelGGL(k_copy, dim3(ew_grid(count)), dim3(EW_THREADS), 0, st, dst, src, count);
  return hipGetLastError();
}

hipError_t launch_correction(const CorrItem* items, int nitems, double* part, int nblk, const int* live,
                             hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_correction, dim3(nblk, nitems), dim3(EW_THREADS), 0, st, items, part, live);
  return hipGetLastError();
}

hipError_t launch_prep(const PrepItem* items, int nitems, int dt, const int* live, hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  dim3 g(64, nitems), b(EW_THREADS);
  switch (dt) {
    case DT_F64: hipLaunchKernelGGL(k_prep<double>, g, b, 0, st, items, live); break;
    case DT_F32: hipLaunchKernelGGL(k_prep<float>, g, b, 0, st, items, live); break;
    case DT_BF16: hipLaunchKernelGGL(k_prep<__bf16>, g, b, 0, st, items, live); break;
    case DT_F16: hipLaunchKernelGGL(k_prep<_Float16>, g, b, 0, st, items, live); break;
    case DT_BF16X3: hipLaunchKernelGGL((k_prep<__bf16, true>), g, b, 0, st, items, live); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_cast(const CastItem* items, int nitems, hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cast, dim3(256, nitems), dim3(EW_THREADS), 0, st, items);
  return hipGetLastError();
}

hipError_t launch_reduce_pairs(const double* part, int nitems, int nblk, double* out, hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_triples, dim3(nitems), dim3(EW_THREADS), 0, st, part, nblk, out);
  return hipGetLastError();
}

hipError_t launch_dot(const double* a, const double* b, int64_t count, double* part, int nblk, double* out,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_dot_part, dim3(nblk), dim3(EW_THREADS), 0, st, a, b, count, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sum_part, dim3(1), dim3(EW_THREADS), 0, st, part, nblk, out);
  return hipGetLastError();
}

hipError_t launch_axpy_dev(double* y, const double* x, const double* alpha_d, double sign, int64_t count,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_axpy_dev, dim3(ew_grid(count)), dim3(EW_THREADS), 0, st, y, x, alpha_d, sign, count);
  return hipGetLastError();
}

hipError_t launch_lincomb(const LinItem& it, hipStream_t st) {
  if (it.count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_lincomb, dim3(ew_grid(it.count)), dim3(EW_THREADS), 0, st, it);
  return hipGetLastError();
}

hipError_t launch_norm_inf(const double* a, int64_t n, int64_t ld, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_norm_inf, dim3(1), dim3(EW_THREADS), 0, st, a, n, ld, out);
  return hipGetLastError();
}

hipError_t launch_rotation_generator(double* out, const double* a, int64_t n, int64_t ld, double c, hipStream_t st) {
  hipLaunchKernelGGL(k_rotation_generator, dim3(ew_grid(4 * n * n)), dim3(EW_THREADS), 0, st, out, a, n, ld, c);
  return hipGetLastError();
}

}  // namespace fm
