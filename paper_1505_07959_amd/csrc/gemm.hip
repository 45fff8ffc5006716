// Grouped, persistent MFMA GEMM for gfx950 with the propagators' epilogues
// fused in.  C = A * B for square np x np row-major operands, one launch over
// a list of independent products (all time slices of all problems of one
// parareal stage).
//
// Design (CDNA4):
//  * 256 threads = 4 wavefronts in a 2 x 2 grid, each owning a (BM/2) x
//    (BM/2) block of C built from MFMA tiles; the 256-wide 16-bit tiles use
//    512 threads = 8 wavefronts in a 2 x 4 grid (128 x 64 per wave, two
//    waves per SIMD, half the L2 traffic per flop of the 128-wide tiles):
//      FP64  v_mfma_f64_16x16x4f64     (16x16 blocks, FP64 accumulate)
//      FP32  v_mfma_f32_32x32x2f32     (32x32 blocks)
//      BF16  v_mfma_f32_32x32x16_bf16  (32x32 blocks, FP32 accumulate)
//      FP16  v_mfma_f32_32x32x16_f16
//  * Operand tiles are staged through LDS, double-buffered with one barrier
//    per K tile; global loads of tile k+1 are in flight during the MFMAs of
//    tile k.  A is kept row-major (k contiguous, rows padded by 16 bytes so the
//    128-bit fragment reads of 8 consecutive rows hit distinct banks); B is
//    stored k-grouped, [BK/V][BN][V], so each lane's V consecutive k values
//    of one column are one contiguous 16/32-byte read.  The transposition of
//    B happens in registers between the global load and the LDS store.
//  * Within one instruction lane group q contributes k = q*V .. q*V+V-1 of
//    the chunk (for FP64/FP32 spread over 4 instructions); the summation order
//    over k is the same for every tile shape, so results do not depend on
//    the chosen configuration.
//  * Persistent grid: each workgroup loops over output tiles.  Tiles are
//    split into 8 contiguous ranges, one per XCD (workgroups are dispatched
//    round-robin over the 8 XCDs), so concurrently running tiles of a
//    product share an L2; within a product tiles are visited in groups of 8
//    tile rows.
//  * No atomics and a fixed reduction order: the kernels are deterministic,
//    which the parareal exactness property relies on.
#include "fm_common.h"

#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>
#include <utility>

namespace fm {
namespace {

typedef float f2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f16v __attribute__((ext_vector_type(16)));
typedef double d2 __attribute__((ext_vector_type(2)));
typedef double d4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));

template <int DT> struct Tr;
template <> struct Tr<DT_F64> {
  using T = double; using Acc = double; using AccV = d4;
  using G16 = d2;   // one 16-byte global chunk
  using LV = d4;    // one lane's k-vector
  using FV = d2;    // one pipeline step's fragment (2 k-values)
  static constexpr int MI = 16, V = 4, NACC = 4;
};
template <> struct Tr<DT_F32> {
  using T = float; using Acc = float; using AccV = f16v;
  using G16 = f4; using LV = f4; using FV = f2;
  static constexpr int MI = 32, V = 4, NACC = 16;
};
template <> struct Tr<DT_BF16> {
  using T = __bf16; using Acc = float; using AccV = f16v;
  using G16 = bf8; using LV = bf8; using FV = bf8;
  static constexpr int MI = 32, V = 8, NACC = 16;
};
template <> struct Tr<DT_F16> {
  using T = _Float16; using Acc = float; using AccV = f16v;
  using G16 = h8; using LV = h8; using FV = h8;
  static constexpr int MI = 32, V = 8, NACC = 16;
};
// split BF16: every operand matrix is two BF16 planes (hi, then lo at +np^2)
template <> struct Tr<DT_BF16X3> {
  using T = __bf16; using Acc = float; using AccV = f16v;
  using G16 = bf8; using LV = bf8; using FV = bf8;
  static constexpr int MI = 32, V = 8, NACC = 16;
};

// Calls f(std::integral_constant<int, I>()) for I = 0, 1, ... in order.
template <class F, int... I>
__device__ __forceinline__ void static_for(std::integer_sequence<int, I...>, F&& f) {
  (f(std::integral_constant<int, I>()), ...);
}

// K segments of a product: 1, or 3 for split BF16 (A_hi B_hi, A_hi B_lo, A_lo B_hi)
template <int DT> constexpr int nseg() { return DT == DT_BF16X3 ? 3 : 1; }

template <int DT>
__device__ __forceinline__ void mma(typename Tr<DT>::AccV& acc, const typename Tr<DT>::LV& a,
                                    const typename Tr<DT>::LV& b) {
  if constexpr (DT == DT_F64) {
#pragma unroll
    for (int t = 0; t < 4; ++t) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t], b[t], acc, 0, 0, 0);
  } else if constexpr (DT == DT_F32) {
#pragma unroll
    for (int t = 0; t < 4; ++t) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[t], b[t], acc, 0, 0, 0);
  } else if constexpr (DT == DT_BF16 || DT == DT_BF16X3) {
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
  } else {
    acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, acc, 0, 0, 0);
  }
}

// One k-step of the FP64 / FP32 MFMA (scalar operands per lane).
template <int DT, class S>
__device__ __forceinline__ void mma1(typename Tr<DT>::AccV& acc, S a, S b) {
  if constexpr (DT == DT_F64) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  else acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
}

// Row/column (within the MI x MI block) of accumulator register v of `lane`.
template <int DT>
__device__ __forceinline__ void acc_pos(int lane, int v, int& r, int& c) {
  if constexpr (DT == DT_F64) {
    r = 4 * v + (lane >> 4);
    c = lane & 15;
  } else {
    r = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
    c = lane & 31;
  }
}

template <class T>
__device__ __forceinline__ T to_op(double v) { return (T)v; }
template <>
__device__ __forceinline__ __bf16 to_op<__bf16>(double v) { return (__bf16)(float)v; }
template <>
__device__ __forceinline__ _Float16 to_op<_Float16>(double v) { return (_Float16)(float)v; }

template <class T>
__device__ __forceinline__ double from_op(T v) { return (double)v; }
template <>
__device__ __forceinline__ double from_op<__bf16>(__bf16 v) { return (double)(float)v; }
template <>
__device__ __forceinline__ double from_op<_Float16>(_Float16 v) { return (double)(float)v; }

// Global-memory access through address-space-1 pointers: the item pointers
// are generic, and flat instructions would also count against the LDS
// wait counter, coupling the LDS pipeline to outstanding global loads.
template <class T> using gptr = const __attribute__((address_space(1))) T*;
template <class T> using gptr_mut = __attribute__((address_space(1))) T*;
// LDS DMA of one 16-byte chunk per lane to LDS address lds (wave-uniform,
// through M0) + 16 * lane, written as assembly so that the compiler does not
// count it as an LDS write: it would otherwise wait for every DMA in flight
// (vmcnt(0)) before each transposing LDS read, because it cannot tell which
// LDS those reads touch.  The K loop waits for its DMAs itself (vmcnt +
// barrier).  The s_nop gives the M0 write the wait state an LDS DMA needs.
__device__ __forceinline__ void lds_dma16(__amdgpu_buffer_rsrc_t r, unsigned lds, int voff) {
  asm volatile("s_nop 0\n\tbuffer_load_dwordx4 %0, %1, 0 offen lds" ::"v"(voff), "s"(r),
               "{m0}"(__builtin_amdgcn_readfirstlane(lds))
               : "memory");
}
template <class T>
__device__ __forceinline__ T gld(const void* p, int64_t i) { return ((gptr<T>)p)[i]; }
template <class T>
__device__ __forceinline__ void gst(void* p, int64_t i, T v) { ((gptr_mut<T>)p)[i] = v; }

// Four consecutive elements per access (EV = 4): the epilogue moves 16-32
// byte vectors per lane instead of 2-8 byte scalars.  idx is a multiple of
// 4 (np is a multiple of 64), so every vector access is naturally aligned.
constexpr int EV = 4;
struct V4 {
  double v[EV];
};
template <class T>
using vec4 = T __attribute__((ext_vector_type(EV)));

template <class T>
__device__ __forceinline__ V4 gld4(const void* p, int64_t idx) {
  const vec4<T> w = *(gptr<vec4<T>>)((const T*)p + idx);
  V4 r;
#pragma unroll
  for (int e = 0; e < EV; ++e) r.v[e] = from_op<T>(w[e]);
  return r;
}
template <class T>
__device__ __forceinline__ void gst4(void* p, int64_t idx, const V4& x) {
  vec4<T> w;
#pragma unroll
  for (int e = 0; e < EV; ++e) w[e] = to_op<T>(x.v[e]);
  *(gptr_mut<vec4<T>>)((T*)p + idx) = w;
}

// Operand-type access; split BF16 stores hi = bf16(v) and lo = bf16(v - hi)
// in the second plane (at + np^2) and reads back hi + lo.
template <int DT>
__device__ __forceinline__ V4 ld_op4(const void* p, int64_t idx, int64_t np2) {
  using T = typename Tr<DT>::T;
  V4 r = gld4<T>(p, idx);
  if constexpr (DT == DT_BF16X3) {
    const V4 lo = gld4<T>(p, idx + np2);
#pragma unroll
    for (int e = 0; e < EV; ++e) r.v[e] += lo.v[e];
  }
  return r;
}
template <int DT>
__device__ __forceinline__ void st_op4(void* p, int64_t idx, int64_t np2, const V4& x) {
  using T = typename Tr<DT>::T;
  gst4<T>(p, idx, x);
  if constexpr (DT == DT_BF16X3) {
    V4 lo;
#pragma unroll
    for (int e = 0; e < EV; ++e) lo.v[e] = x.v[e] - from_op<T>(to_op<T>(x.v[e]));
    gst4<T>(p, idx + np2, lo);
  }
}

// Single-pass fused epilogue (the FP64/FP32 products) for the four elements
// (gr, gc .. gc+3) of item `it`
// (idx = gr*np + gc); element `dpos` (or none, -1) lies on the leading
// n x n diagonal.  Per element the arithmetic is that of the propagator
// step being fused: a = (A B)[gr, gc] in the accumulation precision.
template <int DT, int EPI>
__device__ __forceinline__ void epilogue4(const GItem& it, int64_t idx, int dpos, const V4& a) {
  using Acc = typename Tr<DT>::Acc;
  const double* s = it.s;
  const int64_t np2 = (int64_t)it.np * it.np;
  // E = the product's second input (same dtype as the operands, or FP64)
  auto load_e = [&]() -> V4 {
    return (it.flags & F_E_F64) ? gld4<double>(it.in0, idx) : ld_op4<DT>(it.in0, idx, np2);
  };
  if constexpr (EPI == EPI_AFFINE) {
    V4 v;
#pragma unroll
    for (int e = 0; e < EV; ++e) v.v[e] = s[0] * a.v[e];
    if (!(it.flags & F_E_NONE)) {
      const V4 E = load_e();
#pragma unroll
      for (int e = 0; e < EV; ++e) v.v[e] += s[1] * E.v[e];
    }
#pragma unroll
    for (int e = 0; e < EV; ++e)
      if (e == dpos) v.v[e] += s[2];
    if (it.flags & F_OUT0_F64) gst4<double>(it.out0, idx, v);
    else st_op4<DT>(it.out0, idx, np2, v);
  } else if constexpr (EPI == EPI_RK4 || EPI == EPI_EULER) {
    V4 k;
#pragma unroll
    for (int e = 0; e < EV; ++e) k.v[e] = s[0] * a.v[e];
    if (!(it.flags & F_E_NONE)) {
      const V4 E = load_e();
#pragma unroll
      for (int e = 0; e < EV; ++e) k.v[e] += s[1] * E.v[e];
    }
    if (s[3] != 0.0) {  // identity term of the field (dX/dt = I - A X)
#pragma unroll
      for (int e = 0; e < EV; ++e)
        if (e == dpos) k.v[e] += s[3];
    }
    const double h = s[2];
    const V4 x = gld4<double>(it.x, idx);
    V4 o;
    if constexpr (EPI == EPI_EULER) {
#pragma unroll
      for (int e = 0; e < EV; ++e) o.v[e] = x.v[e] + h * k.v[e];
      gst4<double>(it.out1, idx, o);
    } else {
      void* K = it.out1;
      if (it.stage == 1) {
        gst4<Acc>(K, idx, k);
#pragma unroll
        for (int e = 0; e < EV; ++e) o.v[e] = x.v[e] + 0.5 * h * k.v[e];
      } else if (it.stage == 2 || it.stage == 3) {
        V4 kk = gld4<Acc>(K, idx);
#pragma unroll
        for (int e = 0; e < EV; ++e) kk.v[e] = kk.v[e] + 2.0 * k.v[e];
        gst4<Acc>(K, idx, kk);
        const double c = it.stage == 2 ? 0.5 * h : h;
#pragma unroll
        for (int e = 0; e < EV; ++e) o.v[e] = x.v[e] + c * k.v[e];
      } else {
        const V4 kk = gld4<Acc>(K, idx);
#pragma unroll
        for (int e = 0; e < EV; ++e) o.v[e] = x.v[e] + (h / 6.0) * (kk.v[e] + k.v[e]);
        gst4<double>(it.x, idx, o);
      }
    }
    st_op4<DT>(it.out0, idx, np2, o);
  } else if constexpr (EPI == EPI_POLYP) {
    const V4 p0 = ld_op4<DT>(it.in0, idx, np2), p1 = ld_op4<DT>(it.in1, idx, np2);
    V4 v;
#pragma unroll
    for (int e = 0; e < EV; ++e) v.v[e] = s[1] * p0.v[e] + s[2] * p1.v[e] + s[3] * a.v[e];
#pragma unroll
    for (int e = 0; e < EV; ++e)
      if (e == dpos) v.v[e] += s[0];
    st_op4<DT>(it.out0, idx, np2, v);
    st_op4<DT>(it.out1, idx, np2, a);
  } else {  // EPI_POLYX
    const V4 p0 = ld_op4<DT>(it.in0, idx, np2), p1 = ld_op4<DT>(it.in1, idx, np2),
             p2 = ld_op4<DT>(it.in2, idx, np2);
    V4 v;
#pragma unroll
    for (int e = 0; e < EV; ++e) v.v[e] = a.v[e] + s[5] * p0.v[e] + s[6] * p1.v[e] + s[7] * p2.v[e];
#pragma unroll
    for (int e = 0; e < EV; ++e)
      if (e == dpos) v.v[e] += s[4];
    gst4<double>(it.out1, idx, v);
    st_op4<DT>(it.out0, idx, np2, v);
  }
}

// The epilogue of the 16-bit products, split in two phases: a thread issues
// the global loads of the element groups of the next round (epi_load)
// before it combines the current ones with the products and stores them
// (epi_apply).  Every access goes through a buffer resource over what the
// output tile touches of its matrix, rebased to the tile's first element;
// an operand that an item does not have (the accumulator of RK4 stage 1)
// gets an empty range, so its loads return zeros and no load sits behind a
// branch.  A branch around a load would make the compiler wait for that
// load where the paths merge, and since loads and stores share one
// in-order counter, every such wait would also wait for all stores issued
// before it.  The loaded values stay raw (operand type) until epi_apply.
// The affine product and the RK4 stage update run in FP32, on an FP32
// state (F_X_F32): the product is itself an FP32 accumulation of 16-bit
// operands, and FP32 keeps everything such a step produces.  The Euler
// update (FP64 state) and every FP64 output stay in FP64.  The identity
// term touches one element of the diagonal tiles only, so it sits behind a
// branch that other groups skip.
typedef float f4v __attribute__((ext_vector_type(EV)));
typedef unsigned u4v __attribute__((ext_vector_type(4)));
typedef unsigned u2v __attribute__((ext_vector_type(2)));
typedef __amdgpu_buffer_rsrc_t rsrc_t;

// Resource over `extent` elements of `esz` bytes from element `off` of p;
// an absent operand gets zero records.
__device__ __forceinline__ rsrc_t tile_rsrc(const void* p, int64_t off, int esz, int64_t extent, bool present) {
  char* base = present ? (char*)p + off * esz : (char*)p;
  return __builtin_amdgcn_make_buffer_rsrc(base, (short)0, present ? (int)(extent * esz) : 0, 0x00020000);
}
// four consecutive elements at element offset `off`
__device__ __forceinline__ f4v bld_f32(rsrc_t r, int off) {
  return __builtin_bit_cast(f4v, __builtin_amdgcn_raw_buffer_load_b128(r, off * 4, 0, 0));
}
__device__ __forceinline__ d4 bld_f64(rsrc_t r, int off) {
  const d2 lo = __builtin_bit_cast(d2, __builtin_amdgcn_raw_buffer_load_b128(r, off * 8, 0, 0));
  const d2 hi = __builtin_bit_cast(d2, __builtin_amdgcn_raw_buffer_load_b128(r, off * 8 + 16, 0, 0));
  return d4{lo.x, lo.y, hi.x, hi.y};
}
template <class T>
__device__ __forceinline__ vec4<T> bld_16(rsrc_t r, int off) {
  return __builtin_bit_cast(vec4<T>, __builtin_amdgcn_raw_buffer_load_b64(r, off * 2, 0, 0));
}
__device__ __forceinline__ void bst_f32(rsrc_t r, int off, f4v x) {
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4v, x), r, off * 4, 0, 0);
}
__device__ __forceinline__ void bst_f64(rsrc_t r, int off, const V4& x) {
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4v, d2{x.v[0], x.v[1]}), r, off * 8, 0, 0);
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4v, d2{x.v[2], x.v[3]}), r, off * 8 + 16, 0, 0);
}
template <class T>
__device__ __forceinline__ void bst_16(rsrc_t r, int off, vec4<T> w) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2v, w), r, off * 2, 0, 0);
}
template <class T>
__device__ __forceinline__ f4v widen16(vec4<T> w) {
  f4v r;
#pragma unroll
  for (int e = 0; e < EV; ++e) r[e] = (float)w[e];
  return r;
}
__device__ __forceinline__ V4 widen(f4v a) {
  V4 r;
#pragma unroll
  for (int e = 0; e < EV; ++e) r.v[e] = (double)a[e];
  return r;
}
__device__ __forceinline__ void add_diag(f4v& v, int dpos, float d) {
  if (dpos >= 0) {
#pragma unroll
    for (int e = 0; e < EV; ++e)
      if (e == dpos) v[e] += d;
  }
}
__device__ __forceinline__ void add_diag(V4& v, int dpos, double d) {
  if (dpos >= 0) {
#pragma unroll
    for (int e = 0; e < EV; ++e)
      if (e == dpos) v.v[e] += d;
  }
}

// Operand-type matrices as (hi, lo) planes: split BF16 stores hi = bf16(v)
// and lo = bf16(v - hi) in the second plane (pl = np^2 elements further) and
// reads back hi + lo; the other types have one plane.
template <int DT>
struct Op4 {
  vec4<typename Tr<DT>::T> w[DT == DT_BF16X3 ? 2 : 1];
};
template <int DT>
__device__ __forceinline__ Op4<DT> bld_op(rsrc_t r, int off, int pl) {
  using T = typename Tr<DT>::T;
  Op4<DT> o;
  o.w[0] = bld_16<T>(r, off);
  if constexpr (DT == DT_BF16X3) o.w[1] = bld_16<T>(r, off + pl);
  return o;
}
template <int DT>
__device__ __forceinline__ f4v op_f32(const Op4<DT>& o) {  // hi + lo in FP32
  f4v r = widen16(o.w[0]);
  if constexpr (DT == DT_BF16X3) r += widen16(o.w[1]);
  return r;
}
template <int DT>
__device__ __forceinline__ V4 op_f64(const Op4<DT>& o) {  // hi + lo in FP64
  V4 r;
#pragma unroll
  for (int e = 0; e < EV; ++e) r.v[e] = from_op(o.w[0][e]);
  if constexpr (DT == DT_BF16X3) {
#pragma unroll
    for (int e = 0; e < EV; ++e) r.v[e] += from_op(o.w[1][e]);
  }
  return r;
}
template <int DT>
__device__ __forceinline__ void bst_op(rsrc_t r, int off, int pl, f4v x) {  // from FP32
  using T = typename Tr<DT>::T;
  vec4<T> w;
#pragma unroll
  for (int e = 0; e < EV; ++e) w[e] = (T)x[e];
  bst_16<T>(r, off, w);
  if constexpr (DT == DT_BF16X3) {  // x - hi is exact in FP32
    vec4<T> lo;
#pragma unroll
    for (int e = 0; e < EV; ++e) lo[e] = (T)(x[e] - (float)w[e]);
    bst_16<T>(r, off + pl, lo);
  }
}
template <int DT>
__device__ __forceinline__ void bst_op(rsrc_t r, int off, int pl, const V4& x) {  // from FP64
  using T = typename Tr<DT>::T;
  vec4<T> w;
#pragma unroll
  for (int e = 0; e < EV; ++e) w[e] = to_op<T>(x.v[e]);
  bst_16<T>(r, off, w);
  if constexpr (DT == DT_BF16X3) {
    vec4<T> lo;
#pragma unroll
    for (int e = 0; e < EV; ++e) lo[e] = to_op<T>(x.v[e] - from_op<T>(w[e]));
    bst_16<T>(r, off + pl, lo);
  }
}

// Resources of one output tile's epilogue.  E (in0) is FP64 or of operand
// type; the kernel picks the epilogue body by the item's E mode EM
// (0 none, 1 FP64, 2 operand type), so only the loads of that mode exist.
struct EpiRs {
  rsrc_t e64, eop;       // E: FP64, operand type
  rsrc_t x, kq;          // RK4: FP32 state, FP32 stage accumulator (stage >= 2); Euler: FP64 state
  rsrc_t i1, i2;         // POLYP/POLYX inputs (operand type); POLY* take in0 from eop
  rsrc_t o0d, o0t;       // out0 as FP64 / operand type
  rsrc_t o1;             // out1 (RK4: FP32, Euler and POLYX: FP64, POLYP: operand type)
  int pl;                // plane offset (elements) of split BF16 operands
};
template <int DT, int EPI>
__device__ __forceinline__ EpiRs epi_rsrc(const GItem& it, int row0, int col0, int bm, int bn) {
  using T = typename Tr<DT>::T;
  constexpr int TS = (int)sizeof(T);
  const int64_t np = it.np, np2 = np * np;
  const int64_t off = (int64_t)row0 * np + col0;
  const int64_t ext = (int64_t)(bm - 1) * np + bn;              // one plane
  const int64_t ext_op = (DT == DT_BF16X3 ? np2 : 0) + ext;     // all planes of an operand-type matrix
  const bool has_e = !(it.flags & F_E_NONE), e_f64 = (it.flags & F_E_F64) != 0;
  const bool poly = EPI == EPI_POLYP || EPI == EPI_POLYX;
  EpiRs r;
  r.pl = DT == DT_BF16X3 ? (int)np2 : 0;
  r.e64 = tile_rsrc(it.in0, off, 8, ext, !poly && has_e && e_f64);
  r.eop = tile_rsrc(it.in0, off, TS, ext_op, poly || (has_e && !e_f64));
  r.x = EPI == EPI_EULER ? tile_rsrc(it.x, off, 8, ext, true) : tile_rsrc(it.x, off, 4, ext, EPI == EPI_RK4);
  r.kq = tile_rsrc(it.out1, off, 4, ext, EPI == EPI_RK4 && it.stage >= 2);
  r.i1 = tile_rsrc(it.in1, off, TS, ext_op, poly);
  r.i2 = tile_rsrc(it.in2, off, TS, ext_op, EPI == EPI_POLYX);
  const bool o0_f64 = EPI == EPI_AFFINE && (it.flags & F_OUT0_F64);
  r.o0d = tile_rsrc(it.out0, off, 8, ext, o0_f64);
  r.o0t = tile_rsrc(it.out0, off, TS, ext_op, !o0_f64);
  const int o1sz = EPI == EPI_RK4 ? 4 : EPI == EPI_POLYP ? TS : 8;
  r.o1 = tile_rsrc(it.out1, off, o1sz, EPI == EPI_POLYP ? ext_op : ext, EPI != EPI_AFFINE);
  return r;
}

template <int DT>
struct EpiIn {
  d4 e64;        // E (EM 1); Euler: FP64 state in xd
  Op4<DT> eop;   // E (EM 2); POLYP/POLYX: in0
  Op4<DT> i1, i2;
  f4v xf, kq;    // RK4 FP32 state and stage accumulator
  d4 xd;         // Euler FP64 state
};

template <int DT, int EPI, int EM>
__device__ __forceinline__ EpiIn<DT> epi_load(const EpiRs& rs, int off) {
  EpiIn<DT> in;
  if constexpr (EM == 1) in.e64 = bld_f64(rs.e64, off);
  if constexpr (EM == 2 || EPI == EPI_POLYP || EPI == EPI_POLYX) in.eop = bld_op<DT>(rs.eop, off, rs.pl);
  if constexpr (EPI == EPI_RK4) {
    in.xf = bld_f32(rs.x, off);
    in.kq = bld_f32(rs.kq, off);  // zeros at stage 1 (empty range)
  } else if constexpr (EPI == EPI_EULER) {
    in.xd = bld_f64(rs.x, off);
  } else if constexpr (EPI == EPI_POLYP || EPI == EPI_POLYX) {
    in.i1 = bld_op<DT>(rs.i1, off, rs.pl);
    if constexpr (EPI == EPI_POLYX) in.i2 = bld_op<DT>(rs.i2, off, rs.pl);
  }
  return in;
}

__device__ __forceinline__ V4 to_v4(d4 d) { return V4{{d.x, d.y, d.z, d.w}}; }

// af: the four FP32 accumulations of the product
template <int DT, int EPI, int EM>
__device__ __forceinline__ void epi_apply(const GItem& it, const EpiRs& rs, int off, int dpos, const f4v& af,
                                          const EpiIn<DT>& in) {
  static_assert(std::is_same<typename Tr<DT>::Acc, float>::value, "16-bit products accumulate in FP32");
  const double* s = it.s;
  // E in FP32 / FP64 (EM 0: no E term)
  auto e32 = [&]() -> f4v {
    if constexpr (EM == 1) return __builtin_convertvector(in.e64, f4v);
    else return op_f32<DT>(in.eop);
  };
  auto e64 = [&]() -> V4 {
    if constexpr (EM == 1) return to_v4(in.e64);
    else return op_f64<DT>(in.eop);
  };
  if constexpr (EPI == EPI_AFFINE) {
    if (it.flags & F_OUT0_F64) {
      const V4 a = widen(af);
      V4 v;
#pragma unroll
      for (int e = 0; e < EV; ++e) v.v[e] = s[0] * a.v[e];
      if constexpr (EM != 0) {
        const V4 ev = e64();
#pragma unroll
        for (int e = 0; e < EV; ++e) v.v[e] += s[1] * ev.v[e];
      }
      add_diag(v, dpos, s[2]);
      bst_f64(rs.o0d, off, v);
    } else {
      f4v v = (float)s[0] * af;
      if constexpr (EM != 0) v += (float)s[1] * e32();
      add_diag(v, dpos, (float)s[2]);
      bst_op<DT>(rs.o0t, off, rs.pl, v);
    }
  } else if constexpr (EPI == EPI_RK4) {
    f4v k = (float)s[0] * af;
    if constexpr (EM != 0) k += (float)s[1] * e32();
    if (s[3] != 0.0) add_diag(k, dpos, (float)s[3]);  // identity term of the field (dX/dt = I - A X)
    // the state of a fine solve with 16-bit products is FP32 (F_X_F32)
    const double h = s[2];
    if (it.stage == 4) {  // X <- X + h/6 (k1 + 2 k2 + 2 k3 + k4)
      const f4v o = in.xf + (float)(h / 6.0) * (in.kq + k);
      bst_f32(rs.x, off, o);
      bst_op<DT>(rs.o0t, off, rs.pl, o);
    } else {
      bst_f32(rs.o1, off, it.stage == 1 ? k : in.kq + 2.0f * k);
      bst_op<DT>(rs.o0t, off, rs.pl, in.xf + (float)(it.stage == 3 ? h : 0.5 * h) * k);
    }
  } else if constexpr (EPI == EPI_EULER) {
    const V4 a = widen(af);
    V4 k;
#pragma unroll
    for (int e = 0; e < EV; ++e) k.v[e] = s[0] * a.v[e];
    if constexpr (EM != 0) {
      const V4 ev = e64();
#pragma unroll
      for (int e = 0; e < EV; ++e) k.v[e] += s[1] * ev.v[e];
    }
    if (s[3] != 0.0) add_diag(k, dpos, s[3]);
    const V4 p = to_v4(in.xd);
    V4 o;
#pragma unroll
    for (int e = 0; e < EV; ++e) o.v[e] = p.v[e] + s[2] * k.v[e];
    bst_f64(rs.o1, off, o);
    bst_op<DT>(rs.o0t, off, rs.pl, o);
  } else if constexpr (EPI == EPI_POLYP) {
    const V4 a = widen(af), p = op_f64<DT>(in.eop), q = op_f64<DT>(in.i1);
    V4 v;
#pragma unroll
    for (int e = 0; e < EV; ++e) v.v[e] = s[1] * p.v[e] + s[2] * q.v[e] + s[3] * a.v[e];
    add_diag(v, dpos, s[0]);
    bst_op<DT>(rs.o0t, off, rs.pl, v);
    bst_op<DT>(rs.o1, off, rs.pl, a);
  } else {  // EPI_POLYX
    const V4 a = widen(af), p = op_f64<DT>(in.eop), q = op_f64<DT>(in.i1), r = op_f64<DT>(in.i2);
    V4 v;
#pragma unroll
    for (int e = 0; e < EV; ++e) v.v[e] = a.v[e] + s[5] * p.v[e] + s[6] * q.v[e] + s[7] * r.v[e];
    add_diag(v, dpos, s[4]);
    bst_f64(rs.o1, off, v);
    bst_op<DT>(rs.o0t, off, rs.pl, v);
  }
}

// Threads per workgroup: the 256-wide 16-bit tiles use 8 waves (2 x 4, each
// 128 x 64) so that two waves share every SIMD; the others 4 waves (2 x 2).
template <int DT, int BM>
constexpr int gemm_nt() {
  return (BM == 256 && DT != DT_F64 && DT != DT_F32) ? 512 : 256;
}

// ILV (FP64 only): the interleaved schedule of a K tile's last step, for
// launches of large products (see ktile)
template <int DT, int BM, int BK, int EPI, bool ILV = false>
__global__ __launch_bounds__((gemm_nt<DT, BM>()), (BM == 128 && (DT != DT_F64 || BK == 16)) ? 2 : 1) void gemm_kernel(const GItem* __restrict__ items,
                                                   const int* __restrict__ tile_start, int nitems,
                                                   int total_tiles, const int* __restrict__ live) {
  using TR = Tr<DT>;
  using T = typename TR::T;
  using G16 = typename TR::G16;
  using AccV = typename TR::AccV;
  using FV = typename TR::FV;
  constexpr int MI = TR::MI, V = TR::V, NACC = TR::NACC;
  constexpr int BN = BM;
  constexpr int NT = gemm_nt<DT, BM>();  // threads
  constexpr int NWC = NT / 128;          // waves along N (2 along M)
  constexpr int WM = BM / 2, WN = BN / NWC;
  constexpr int RM = WM / MI, RN = WN / MI;
  constexpr int NQ = 64 / MI;            // lane groups along k
  constexpr int KC = NQ * V;             // k per chunk
  constexpr int W = 16 / sizeof(T);      // elements per 16-byte chunk
  // global prefetch depth in K tiles: the 16-bit K tiles of the 128-wide
  // tiles are short next to the memory latency, so their loads are issued
  // two tiles ahead (the 256-wide tiles have no registers for a second set)
  constexpr int PF = (DT == DT_F64 || DT == DT_F32 || BM > 128) ? 1 : 2;
  // 16-bit A tiles fetched one K tile ahead go from global memory straight
  // into LDS (buffer loads with the LDS flag): no staging registers and no
  // LDS store instructions.  Such a load writes the 16-byte chunks of a wave
  // to 1 KB of consecutive LDS, so the tile is stored unpadded, 16-byte chunk
  // j of row r at chunk position j ^ aswz(r) of that row: the lane that fills
  // a position loads the chunk that belongs there, and the fragment reads
  // (32 rows at one chunk) fall on distinct banks.
  // (the ring below implies it for the 128-wide tiles as well)
  constexpr bool RING = DT != DT_F64 && DT != DT_F32 && BK == 32 && (BM == 256 || BM == 128);
  constexpr bool ADMA = DT != DT_F64 && DT != DT_F32 && (PF == 1 || RING);
  constexpr int CPR = BK / (16 / (int)sizeof(T));  // 16-byte chunks per A row
  constexpr int CPR_SH = CPR == 8 ? 3 : CPR == 4 ? 2 : CPR == 2 ? 1 : 0;
  static_assert(!ADMA || CPR == 4 || CPR == 8, "A swizzle assumes 4 or 8 chunks per row");
  static_assert(!ADMA || TR::V == 16 / (int)sizeof(T), "A fragment reads assume one chunk per k-vector");
  auto aswz = [](int r) { return (r ^ (r >> CPR_SH)) & (CPR - 1); };
  // The 256 x 32 and 128 x 32 16-bit tiles go further: B comes by LDS DMA
  // as well, into a ring of NS stages, so NS - 1 K tiles of loads are in
  // flight while one is computed.  B keeps its row-major global layout in
  // LDS (16-byte chunk j of k-row r at position j ^ bsw(r)); each lane's
  // eight k-values of one column are gathered by two transposing LDS reads
  // (ds_read_b64_tr_b16: within 16 lanes, lane i receives element i % 4 of
  // the 8-byte reads of lanes 4j + i / 4, j = 0..3).  bsw(r) = 5 (r mod 4)
  // puts the 16 lanes of such a read (4 rows x 32 bytes) on distinct banks
  // for rows of 32 and of 16 chunks (checked by enumeration in a 32-bank and
  // in a 64-bank model).
  constexpr int NS = RING ? 4 : 2;  // LDS stages
  auto bsw = [](int r) { return 5 * (r & 3); };
  constexpr int PADA = ADMA ? 0 : 16 / (int)sizeof(T);
  constexpr int LDA_S = BK + PADA;       // LDS row stride of A (elements)
  constexpr int A_CHUNKS = BM * BK / W;  // 16-byte chunks of an A tile
  constexpr int B_BLOCKS = (BK / V) * (BN / W);
  static_assert(BK % KC == 0, "BK must be a multiple of the MFMA k chunk");
  static_assert(A_CHUNKS % NT == 0, "A tile must split evenly over the threads");
  static_assert(B_BLOCKS <= NT || B_BLOCKS % NT == 0, "B tile split");
  constexpr int A_PER_T = A_CHUNKS / NT;
  constexpr int BR_PER_T = BK * BN / W / NT;  // B chunks per thread (ring)
  static_assert(!RING || (BK * BN / W) % NT == 0, "B tile split (ring)");
  static_assert(!RING || (BN / W) == 32 || (BN / W) == 16, "the B swizzle assumes 16 or 32 chunks per k-row");
  constexpr int B_PER_T = B_BLOCKS >= NT ? B_BLOCKS / NT : 1;
  // When the tile has fewer B blocks (V rows x 16 bytes) than threads, the
  // RSPLIT threads of a block share its rows (VR each) so that every thread
  // loads and stores the same amount; their LDS stores are VR-element parts
  // of the k-vectors.
  constexpr int RSPLIT = B_BLOCKS < NT ? NT / B_BLOCKS : 1;
  constexpr int VR = V / RSPLIT;
  static_assert(V % RSPLIT == 0 && B_BLOCKS * RSPLIT >= NT, "B row split");
  typedef T PV __attribute__((ext_vector_type(VR)));
  // pipeline step: SUBV k-values per lane (FP64/FP32: half of the lane's
  // 4-vector, 2 MFMAs deep; 16-bit: one MFMA), SUB steps per KC chunk
  constexpr int SUBV = (DT == DT_F64 || DT == DT_F32) ? 2 : V;
  constexpr int SUB = V / SUBV;
  constexpr int NSTEP = (BK / KC) * SUB;
  static_assert(NSTEP % 2 == 0, "pipeline steps per K tile must be even");
  // B column swizzle inside aligned groups of G columns (G columns = 128 bytes
  // of k-vectors): a thread stores W adjacent columns, so without it the lanes
  // of one store sit W columns apart and hit the same banks; the XOR with the
  // W-block index spreads them, and the fragment reads (consecutive columns)
  // stay a permutation of one aligned group.
  constexpr int GS = 128 / (V * (int)sizeof(T));
  auto bswz = [](int c) { return c ^ ((c / W) & (GS - 1)); };

  // one LDS block: two stages of A and B tiles during the K loop, reused
  // by the epilogue to stage accumulators
  constexpr int A_STAGE = BM * LDA_S, B_STAGE = BK * BN;
  constexpr int SMEM_K = NS * (A_STAGE + B_STAGE) * (int)sizeof(T);
  constexpr int SMEM_E = 2 * TR::MI * (BN + 16 / (int)sizeof(typename TR::Acc)) * (int)sizeof(typename TR::Acc);
  constexpr int SMEM = SMEM_K > SMEM_E ? SMEM_K : SMEM_E;
  __shared__ __attribute__((aligned(16))) char smem[SMEM];
  T (*As)[A_STAGE] = reinterpret_cast<T (*)[A_STAGE]>(smem);
  T (*Bs)[B_STAGE] = reinterpret_cast<T (*)[B_STAGE]>(smem + NS * A_STAGE * sizeof(T));

  // Workgroup barrier for LDS reuse.  The 16-bit epilogue's stores need not
  // complete at it (no workgroup reads another's global writes within a
  // launch): waiting only for LDS lets them drain behind later work, where
  // __syncthreads would wait for every one of them.
  auto epi_sync = [](auto lds_only_c) {
    if constexpr (decltype(lds_only_c)::value)
      asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
    else
      __syncthreads();
  };
  const int wave = threadIdx.x >> 6;  // wave-uniform
  const int wr = wave / NWC, wc = wave % NWC;

  // tile range of this workgroup
  int t_begin, t_end, t_step;
  const int G = gridDim.x;
  if ((G & 7) == 0 && total_tiles >= G) {
    const int xcd = blockIdx.x & 7;
    const int per = G >> 3;
    const int lo = (int)(((int64_t)total_tiles * xcd) >> 3);
    const int hi = (int)(((int64_t)total_tiles * (xcd + 1)) >> 3);
    t_begin = lo + (blockIdx.x >> 3);
    t_end = hi;
    t_step = per;
  } else {
    t_begin = blockIdx.x;
    t_end = total_tiles;
    t_step = G;
  }

  const int tbase = tile_start[0];
  for (int t = t_begin; t < t_end; t += t_step) {
    // The per-thread indices are re-derived for every tile from an opaque
    // copy of the thread index: the addresses built from them are then
    // computed per tile and dead during the epilogue, instead of being
    // hoisted to the kernel's start and spilled.
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int lane = tid & 63;
    const int lr = lane % MI, lq = lane / MI;
    // locate the item (binary search over prefix sums)
    const int tv = t + tbase;
    int lo = 0, hi = nitems - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (tile_start[mid] <= tv) lo = mid; else hi = mid - 1;
    }
    const GItem& it = items[lo];
    if (live != nullptr && live[it.inst] == 0) continue;  // uniform across the workgroup
    const int np = it.np;
    const int tiles = np / BM;
    const int local = tv - tile_start[lo];
    constexpr int GROUP = 8;
    const int per_group = GROUP * tiles;
    const int grp = local / per_group;
    const int first_m = grp * GROUP;
    const int gsz = min(tiles - first_m, GROUP);
    const int in_grp = local - grp * per_group;
    const int tm = first_m + in_grp % gsz;
    const int tn = in_grp / gsz;
    const int row0 = tm * BM, col0 = tn * BN;

    const T* __restrict__ Ag = (const T*)it.a + (int64_t)row0 * np;
    const T* __restrict__ Bg = (const T*)it.b + col0;

    AccV acc[RM][RN];
#pragma unroll
    for (int i = 0; i < RM; ++i)
#pragma unroll
      for (int j = 0; j < RN; ++j)
#pragma unroll
        for (int v = 0; v < NACC; ++v) acc[i][j][v] = 0;

    // PF register staging sets: tile kt's global loads land in set kt % PF
    G16 ra[PF][ADMA ? 1 : A_PER_T];
    G16 rb[PF][B_PER_T][VR];

    const int64_t np2 = (int64_t)np * np;
    const int nkps = np / BK;  // K tiles per segment
    // F_SPLIT_A (16-bit types): the left operand is two planes, hi then lo at
    // + np^2, and the product is A_hi B + A_lo B, one K segment each,
    // accumulated in FP32 in that order
    const bool split_a = (DT == DT_BF16 || DT == DT_F16) && (it.flags & F_SPLIT_A);
    // Global loads through buffer resources rebased at every K tile: the
    // per-lane byte offsets are loop-invariant and small, and a resource's
    // record count is the exact extent of the tile's panel, so a load can
    // never leave it (out-of-range buffer loads return zero).
    auto gload = [&](int kt, int set, int dbuf) {
      // segment 0: (A_hi, B_hi); 1: (A_hi, B_lo); 2: (A_lo, B_hi)
      const int seg = kt / nkps;
      const int k0 = (kt - seg * nkps) * BK;
      const T* As_g = Ag + (split_a ? seg * np2 : (seg == 2 ? np2 : 0)) + k0;
      const T* Bs_g = Bg + (!split_a && seg == 1 ? np2 : 0) + (int64_t)k0 * np;
      const __amdgpu_buffer_rsrc_t ra_rs = __builtin_amdgcn_make_buffer_rsrc(
          const_cast<T*>(As_g), (short)0, ((BM - 1) * np + BK) * (int)sizeof(T), 0x00020000);
      const __amdgpu_buffer_rsrc_t rb_rs = __builtin_amdgcn_make_buffer_rsrc(
          const_cast<T*>(Bs_g), (short)0, ((BK - 1) * np + BN) * (int)sizeof(T), 0x00020000);
      if constexpr (ADMA) {
        // position p = NT*u + tid of LDS buffer dbuf (wave-uniform base, lane
        // offset 16 bytes per lane) receives chunk (p % CPR) ^ aswz(row).
        // The ring issues its DMAs as assembly (it waits for them itself);
        // the other tiles rely on the compiler's wait at __syncthreads.
#pragma unroll
        for (int u = 0; u < A_PER_T; ++u) {
          const int p = tid + NT * u;
          const int r = p / CPR, cc = (p % CPR) ^ aswz(r);
          if constexpr (RING) {
            lds_dma16(ra_rs, (unsigned)(size_t)(__attribute__((address_space(3))) void*)(&As[dbuf][(NT * u + wave * 64) * W]),
                      (r * np + cc * W) * (int)sizeof(T));
          } else {
            __attribute__((address_space(3))) void* dst =
                (__attribute__((address_space(3))) void*)(&As[dbuf][(NT * u + wave * 64) * W]);
            __builtin_amdgcn_raw_ptr_buffer_load_lds(ra_rs, dst, 16, (r * np + cc * W) * (int)sizeof(T), 0, 0, 0);
          }
        }
      } else {
#pragma unroll
        for (int u = 0; u < A_PER_T; ++u) {
          const int c = tid + NT * u;
          const int r = c / (BK / W), cc = c % (BK / W);
          ra[set][u] = __builtin_bit_cast(G16, __builtin_amdgcn_raw_buffer_load_b128(
                                              ra_rs, (r * np + cc * W) * (int)sizeof(T), 0, 0));
        }
      }
      if constexpr (RING) {
#pragma unroll
        for (int u = 0; u < BR_PER_T; ++u) {
          const int p = tid + NT * u;
          const int r = p / (BN / W), cc = (p % (BN / W)) ^ bsw(r);
          lds_dma16(rb_rs, (unsigned)(size_t)(__attribute__((address_space(3))) void*)(&Bs[dbuf][(NT * u + wave * 64) * W]),
                    (r * np + cc * W) * (int)sizeof(T));
        }
      } else {
#pragma unroll
        for (int u = 0; u < B_PER_T; ++u) {
          const int blk = RSPLIT > 1 ? tid % B_BLOCKS : tid + NT * u;
          const int r0 = RSPLIT > 1 ? (tid / B_BLOCKS) * VR : 0;
          const int kb = blk / (BN / W), cb = blk % (BN / W);
#pragma unroll
          for (int r = 0; r < VR; ++r)
            rb[set][u][r] = __builtin_bit_cast(G16, __builtin_amdgcn_raw_buffer_load_b128(
                                                   rb_rs, ((kb * V + r0 + r) * np + cb * W) * (int)sizeof(T), 0, 0));
        }
      }
    };
    auto lstore = [&](int buf, int set) {
      if constexpr (!ADMA) {
#pragma unroll
        for (int u = 0; u < A_PER_T; ++u) {
          const int c = tid + NT * u;
          const int r = c / (BK / W), cc = c % (BK / W);
          *(G16*)(&As[buf][r * LDA_S + cc * W]) = ra[set][u];
        }
      }
      // The B store addresses are recomputed at every store from an opaque
      // copy of the thread index: hoisted out of the K loop they would hold
      // W registers per thread for the whole loop.
      int tid_o = tid;
      asm volatile("" : "+v"(tid_o));
#pragma unroll
      for (int u = 0; u < B_PER_T; ++u) {
        const int blk = RSPLIT > 1 ? tid_o % B_BLOCKS : tid_o + NT * u;
        const int r0 = RSPLIT > 1 ? (tid_o / B_BLOCKS) * VR : 0;
        const int kb = blk / (BN / W), cb = blk % (BN / W);
        T* bcol = &Bs[buf][(kb * BN + cb * W) * V + r0];
        const int sw = cb & (GS - 1);
#pragma unroll
        for (int w = 0; w < W; ++w) {
          PV col;
#pragma unroll
          for (int r = 0; r < VR; ++r) col[r] = rb[set][u][r][w];
          // bswz(cb * W + w) = cb * W + (w ^ (cb & (GS - 1))) for W == GS
          *(PV*)(bcol + ((W == GS ? (w ^ sw) : (bswz(cb * W + w) - cb * W)) * V)) = col;
        }
      }
    };

    // K tiles of all segments in sequence (one segment unless split BF16).
    // Software pipeline at the granularity of one "step" (SUBV k-values per
    // lane group of a KC chunk): the fragments of step s+1 are read from LDS
    // while the MFMAs of step s run.  At the last step of a K tile the next
    // tile (already in registers) is stored to the other LDS buffer, one
    // barrier publishes it, its first fragments are requested and only then
    // are the last MFMAs of the current tile issued, so they cover the LDS
    // latency; the global loads of tile kt+2 go out right after the barrier.
    const int nk = nkps * (split_a ? 2 : nseg<DT>());
    FV fa0[RM], fb0[RN], fa1[RM], fb1[RN];
    auto read_frag = [&](FV (&fa)[RM], FV (&fb)[RN], int buf, int sidx) {
      const int ch = sidx / SUB, sub = sidx % SUB;
#pragma unroll
      for (int i = 0; i < RM; ++i) {
        const int r = wr * WM + i * MI + lr;
        if constexpr (ADMA)  // 16-bit: one lane's k-vector is one chunk (V == W)
          fa[i] = *(const FV*)(&As[buf][r * LDA_S + ((ch * NQ + lq) ^ aswz(r)) * W]);
        else
          fa[i] = *(const FV*)(&As[buf][r * LDA_S + ch * KC + lq * V + sub * SUBV]);
      }
      if constexpr (RING) {
        // lane (g, jj, a) = (lane / 16, lane / 4 % 4, lane % 4) supplies row
        // r (then r + 4), columns c .. c+3; lane l receives k-rows
        // ch*KC + 8 (l / 32) + 0..7 of column wc*WN + j*MI + l % 32.  The
        // ring's DMAs are assembly (lds_dma16), so the compiler adds no wait
        // for them before these reads, and waits for the reads themselves
        // only where the MFMAs use them.
        typedef short s4v __attribute__((ext_vector_type(4)));
        typedef short s8v __attribute__((ext_vector_type(8)));
        typedef __attribute__((address_space(3))) s4v* lp;
        const int g = lane >> 4, jj = (lane >> 2) & 3, a = lane & 3;
        const int r = ch * KC + 8 * (g >> 1) + jj;
#pragma unroll
        for (int j = 0; j < RN; ++j) {
          const int c = wc * WN + j * MI + 16 * (g & 1) + 4 * a;
          const lp p = (lp)(__attribute__((address_space(3))) T*)(&Bs[buf][r * BN + ((c / W) ^ bsw(r)) * W + (c % W)]);
          const s4v lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16(p);
          const s4v hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16(p + BN);
          fb[j] = __builtin_bit_cast(FV, (s8v)__builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7));
        }
      } else {
#pragma unroll
        for (int j = 0; j < RN; ++j)
          fb[j] = *(const FV*)(&Bs[buf][((ch * NQ + lq) * BN + bswz(wc * WN + j * MI + lr)) * V + sub * SUBV]);
      }
    };
    // FP64: the MFMAs of k-value t of a step (t < SUBV)
    auto mfma_k = [&](const FV (&fa)[RM], const FV (&fb)[RN], int t) {
#pragma unroll
      for (int i = 0; i < RM; ++i)
#pragma unroll
        for (int j = 0; j < RN; ++j) mma1<DT>(acc[i][j], fa[i][t], fb[j][t]);
    };
    auto mfma_step = [&](const FV (&fa)[RM], const FV (&fb)[RN]) {
      if constexpr (DT == DT_F64 || DT == DT_F32) {
        // k-value outermost: consecutive MFMAs update different accumulators
#pragma unroll
        for (int t = 0; t < SUBV; ++t)
#pragma unroll
          for (int i = 0; i < RM; ++i)
#pragma unroll
            for (int j = 0; j < RN; ++j) mma1<DT>(acc[i][j], fa[i][t], fb[j][t]);
      } else {
#pragma unroll
        for (int i = 0; i < RM; ++i)
#pragma unroll
          for (int j = 0; j < RN; ++j) mma<DT>(acc[i][j], fa[i], fb[j]);
      }
    };
    // One K tile.  Step s (compile-time) computes with fragment set s & 1
    // and fills the other set.  At the last step the successor tile kt+1
    // goes from its staging set to the other LDS buffer, one barrier
    // publishes it, its first fragments are requested, the same staging set
    // is refilled with tile kt+1+PF (global loads stay in flight for PF K
    // tiles of MFMA work) and only then are the tile's last MFMAs issued,
    // covering the LDS latency.  Every K tile runs the same code: after the
    // last one the boundary work repeats tile nk-1 (clamped indices, never
    // used), which keeps the loop free of branches that would make the
    // compiler's LDS wait counts conservative.
    auto ktile = [&](auto par_c, int kt) {
      constexpr int set = PF == 2 ? (decltype(par_c)::value ^ 1) : 0;
      const int cur = kt & 1;
      static_for(std::make_integer_sequence<int, NSTEP>(), [&](auto s_c) {
        constexpr int sidx = decltype(s_c)::value;
        FV(&fa_c)[RM] = (sidx & 1) ? fa1 : fa0;
        FV(&fb_c)[RN] = (sidx & 1) ? fb1 : fb0;
        FV(&fa_n)[RM] = (sidx & 1) ? fa0 : fa1;
        FV(&fb_n)[RN] = (sidx & 1) ? fb0 : fb1;
        if constexpr (DT == DT_F64 && ILV && sidx + 1 == NSTEP) {
          // FP64, launches of large products (ILV; on launches of many small
          // products this schedule more than doubled the time of their
          // latency-bound launches, which keep the block order): the
          // per-tile work runs in the MFMAs' shadow.  The MFMAs
          // of the step's first k-value carry the LDS stores of the next
          // tile (one store and two VALU instructions after each), those
          // of the second k-value the fragment reads and global loads
          // issued after the barrier; the per-accumulator order of the
          // MFMAs is that of mfma_step.  FP64 fine step at n = 4096:
          // 65.9 -> 69.5 TFLOP/s (the same for FP32 lost 1.6 %).
          static_assert(SUBV == 2, "the FP64 step is split by k-value");
          __builtin_amdgcn_sched_barrier(0);
          mfma_k(fa_c, fb_c, 0);
          lstore(cur ^ 1, set);
          static_for(std::make_integer_sequence<int, RM * RN>(), [&](auto) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // MFMA
            __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);  // LDS write
            __builtin_amdgcn_sched_group_barrier(0x002, 2, 0);  // VALU
          });
          __builtin_amdgcn_sched_barrier(0);
          __syncthreads();
          read_frag(fa_n, fb_n, cur ^ 1, 0);
          gload(min(kt + 1 + PF, nk - 1), set, cur);
          mfma_k(fa_c, fb_c, 1);
          static_for(std::make_integer_sequence<int, RM * RN>(), [&](auto) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // MFMA
            __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // LDS read
            __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);  // global load
          });
          __builtin_amdgcn_sched_barrier(0);
        } else {
          if constexpr (sidx + 1 < NSTEP) {
            read_frag(fa_n, fb_n, cur, sidx + 1);
          } else {
            lstore(cur ^ 1, set);
            __syncthreads();
            read_frag(fa_n, fb_n, cur ^ 1, 0);
            gload(min(kt + 1 + PF, nk - 1), set, cur);  // A (ADMA): into the buffer just released
          }
          __builtin_amdgcn_sched_barrier(0);
          mfma_step(fa_c, fb_c);
          __builtin_amdgcn_sched_barrier(0);
        }
      });
    };

    // Ring K loop: tile kt sits in stage kt % NS.  At its last step a wave
    // waits until only the loads of tiles kt+2 .. kt+NS-1 are outstanding
    // (its own loads of tile kt+1 have landed) and its LDS reads are done;
    // the barrier then publishes tile kt+1 to all waves and frees stage
    // kt % NS, which is refilled with tile kt+NS at once.  Every thread
    // issues LPT loads per tile in every K tile (clamped tile index after
    // the last), so the outstanding count is the same everywhere.  Every
    // step interleaves its MFMAs with the next step's fragment reads (one
    // LDS read after each MFMA), so the reads of all waves are spread over
    // the step instead of arriving in bursts; at the barrier step they
    // start right after the barrier.  FP16 fine step at n = 4096: 668 TFLOP/s
    // with the reads issued as a block after the MFMAs (the transposing
    // ones waited for inside their own assembly block), 700 interleaved.
    constexpr int LPT = A_PER_T + BR_PER_T;
    auto ring_sync = [](auto n_c) {
      asm volatile("s_waitcnt vmcnt(%0) lgkmcnt(0)\n\ts_barrier" ::"n"(decltype(n_c)::value) : "memory");
    };
    // scheduling pattern of a step: MFMA, LDS read, MFMA, ... (RM + 2 RN
    // reads, RM RN MFMAs)
    auto interleave = [&]() {
      static_for(std::make_integer_sequence<int, RM * RN>(), [&](auto) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
      });
    };
    auto ktile_ring = [&](int kt) {
      const int cur = kt & (NS - 1), nxt = (kt + 1) & (NS - 1);
      static_for(std::make_integer_sequence<int, NSTEP>(), [&](auto s_c) {
        constexpr int sidx = decltype(s_c)::value;
        FV(&fa_c)[RM] = (sidx & 1) ? fa1 : fa0;
        FV(&fb_c)[RN] = (sidx & 1) ? fb1 : fb0;
        FV(&fa_n)[RM] = (sidx & 1) ? fa0 : fa1;
        FV(&fb_n)[RN] = (sidx & 1) ? fb0 : fb1;
        if constexpr (sidx + 1 < NSTEP) {
          read_frag(fa_n, fb_n, cur, sidx + 1);
          mfma_step(fa_c, fb_c);
          interleave();
        } else {
          ring_sync(std::integral_constant<int, (NS - 2) * LPT>());
          __builtin_amdgcn_sched_barrier(0);
          read_frag(fa_n, fb_n, nxt, 0);
          mfma_step(fa_c, fb_c);
          interleave();
          __builtin_amdgcn_sched_barrier(0);
          gload(min(kt + NS, nk - 1), 0, cur);
        }
        __builtin_amdgcn_sched_barrier(0);
      });
    };

    // the previous output tile's epilogue may still read LDS
    epi_sync(std::integral_constant<bool, (DT != DT_F64 && DT != DT_F32)>());
    if constexpr (RING) {
      static_for(std::make_integer_sequence<int, NS>(), [&](auto s_c) {
        constexpr int st = decltype(s_c)::value;
        gload(min(st, nk - 1), 0, st);
      });
      ring_sync(std::integral_constant<int, (NS - 1) * LPT>());
      read_frag(fa0, fb0, 0, 0);
      for (int kt = 0; kt < nk; ++kt) ktile_ring(kt);
    } else {
    gload(0, 0, 0);
    lstore(0, 0);
    gload(min(1, nk - 1), PF - 1, 1);
    if (PF == 2) gload(min(2, nk - 1), 0, 0);
    __syncthreads();
    read_frag(fa0, fb0, 0, 0);
    if constexpr (PF == 1) {
      for (int kt = 0; kt < nk; ++kt) ktile(std::integral_constant<int, 0>(), kt);
    } else {
      for (int kt = 0; kt < nk; kt += 2) {
        ktile(std::integral_constant<int, 0>(), kt);
        if (kt + 1 < nk) ktile(std::integral_constant<int, 1>(), kt + 1);  // nk is odd only for 64-wide tiles
      }
    }
    }

    // Fused epilogue, staged through LDS in RM passes: in pass i every wave
    // writes its accumulator row block i (MI rows), then all threads
    // walk the 2*MI x BN staged rows in row-major order, so the epilogue's
    // global traffic is coalesced and the accumulators are only ever
    // indexed statically.
    {
      // the clamped A reload of the last K tile may still be landing in LDS
      if constexpr (ADMA) __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
      using Acc = typename TR::Acc;
      constexpr int CROWS = 2 * MI;
      constexpr int CLD = BN + 16 / (int)sizeof(Acc);
      static_assert(CROWS * CLD * (int)sizeof(Acc) <= SMEM, "epilogue staging must fit in LDS");
      Acc* Cs = reinterpret_cast<Acc*>(smem);
      const int n_valid = it.n;
      // ITER element groups per thread and pass
      constexpr int ITER = CROWS * BN / EV / NT;
      static_assert(CROWS * BN / EV % NT == 0, "epilogue split");
      auto stage_acc = [&](auto i_c) {
        constexpr int i = decltype(i_c)::value;
#pragma unroll
        for (int j = 0; j < RN; ++j)
#pragma unroll
          for (int v = 0; v < NACC; ++v) {
            int r, c;
            acc_pos<DT>(lane, v, r, c);
            Cs[(wr * MI + r) * CLD + wc * WN + j * MI + c] = (Acc)acc[i][j][v];
          }
      };
      if constexpr (DT == DT_F64 || DT == DT_F32) {
        static_for(std::make_integer_sequence<int, RM>(), [&](auto i_c) {
          constexpr int i = decltype(i_c)::value;
          __syncthreads();  // K loop / previous pass readers are done with LDS
          stage_acc(i_c);
          __syncthreads();
          for (int e = tid; e < CROWS * BN / EV; e += NT) {
            const int rr = (e * EV) / BN, cc = (e * EV) % BN;
            const int gr = row0 + (rr / MI) * WM + i * MI + (rr % MI);
            const int gc = col0 + cc;
            V4 a;
#pragma unroll
            for (int q = 0; q < EV; ++q) a.v[q] = (double)Cs[rr * CLD + cc + q];
            const int dpos = (gr >= gc && gr < gc + EV && gr < n_valid) ? gr - gc : -1;
            epilogue4<DT, EPI>(it, (int64_t)gr * np + gc, dpos, a);
          }
        });
      } else {
        // 16-bit products: EG element groups per round, ROUNDS rounds per
        // pass; the loads of round R+1 (of the next pass, at a pass's last
        // round) are issued before the stores of round R.
        constexpr int EG = ITER < 2 ? ITER : 2;
        static_assert(ITER % EG == 0, "epilogue split");
        constexpr int ROUNDS = ITER / EG;
        constexpr int NR = RM * ROUNDS;
        const EpiRs rs = epi_rsrc<DT, EPI>(it, row0, col0, BM, BN);
        // Group m = round * EG + g of a pass covers staged row rr0 + m * RS,
        // columns cc .. cc+3 (the same for every group of a thread), so all
        // offsets are one per-thread base plus compile-time multiples:
        // staged row rr0 + m RS is tile row rr0 + trow(pass, m), as RS
        // divides MI.
        constexpr int GPR = BN / EV;  // element groups per staged row
        constexpr int RS = NT / GPR;  // staged rows per sweep of the threads
        static_assert(NT % GPR == 0 && MI % RS == 0, "epilogue group layout");
        const int cc = (tid % GPR) * EV, rr0 = tid / GPR;
        const int gbase = rr0 * np + cc;             // tile-relative element offset
        const int lbase = rr0 * CLD + cc;            // staged element
        const int dbase = row0 + rr0 - (col0 + cc);  // row minus column, before trow
        const int rmax = n_valid - (row0 + rr0);     // diagonal terms only for trow < rmax
        auto body = [&](auto em_c) {
          constexpr int EM = decltype(em_c)::value;
          EpiIn<DT> in[2][EG];
          auto load_round = [&](auto r_c) {
            constexpr int R = decltype(r_c)::value;
            constexpr int i = R / ROUNDS;
#pragma unroll
            for (int g = 0; g < EG; ++g) {
              const int m = (R % ROUNDS) * EG + g;
              const int trow = (m * RS / MI) * WM + i * MI + (m * RS) % MI;
              in[R & 1][g] = epi_load<DT, EPI, EM>(rs, gbase + trow * np);
            }
          };
          load_round(std::integral_constant<int, 0>());
          static_for(std::make_integer_sequence<int, RM>(), [&](auto i_c) {
            constexpr int i = decltype(i_c)::value;
            epi_sync(std::true_type());  // K loop / previous pass readers are done with LDS
            stage_acc(i_c);
            epi_sync(std::true_type());
            static_for(std::make_integer_sequence<int, ROUNDS>(), [&](auto r_c) {
              constexpr int R = i * ROUNDS + decltype(r_c)::value;
              if constexpr (R + 1 < NR) load_round(std::integral_constant<int, R + 1>());
#pragma unroll
              for (int g = 0; g < EG; ++g) {
                const int m = decltype(r_c)::value * EG + g;
                const int trow = (m * RS / MI) * WM + i * MI + (m * RS) % MI;
                const f4v af = *(const f4v*)&Cs[lbase + m * RS * CLD];
                const int d = dbase + trow;
                const int dpos = (d >= 0 && d < EV && trow < rmax) ? d : -1;
                epi_apply<DT, EPI, EM>(it, rs, gbase + trow * np, dpos, af, in[R & 1][g]);
              }
            });
          });
        };
        if constexpr (EPI == EPI_POLYP || EPI == EPI_POLYX) {
          body(std::integral_constant<int, 0>());
        } else {
          if (it.flags & F_E_NONE) body(std::integral_constant<int, 0>());
          else if (it.flags & F_E_F64) body(std::integral_constant<int, 1>());
          else body(std::integral_constant<int, 2>());
        }
      }
    }
  }
}

template <int DT, int BM, int BK>
hipError_t launch_cfg(int epi, const GItem* items, const int* ts, int nitems, int total, int grid,
                      const int* live, hipStream_t st) {
  dim3 g(grid), b(gemm_nt<DT, BM>());
  // FP64: the interleaved schedule when the items average at least 64 tiles
  // of 128 (orders of 1024 and more)
  const bool ilv = DT == DT_F64 && BM == 128 && total >= 64 * nitems;
  auto go = [&](auto ilv_c) -> hipError_t {
    constexpr bool I = decltype(ilv_c)::value;
    switch (epi) {
      case EPI_AFFINE: hipLaunchKernelGGL((gemm_kernel<DT, BM, BK, EPI_AFFINE, I>), g, b, 0, st, items, ts, nitems, total, live); break;
      case EPI_RK4: hipLaunchKernelGGL((gemm_kernel<DT, BM, BK, EPI_RK4, I>), g, b, 0, st, items, ts, nitems, total, live); break;
      case EPI_EULER: hipLaunchKernelGGL((gemm_kernel<DT, BM, BK, EPI_EULER, I>), g, b, 0, st, items, ts, nitems, total, live); break;
      case EPI_POLYP: hipLaunchKernelGGL((gemm_kernel<DT, BM, BK, EPI_POLYP, I>), g, b, 0, st, items, ts, nitems, total, live); break;
      case EPI_POLYX: hipLaunchKernelGGL((gemm_kernel<DT, BM, BK, EPI_POLYX, I>), g, b, 0, st, items, ts, nitems, total, live); break;
      default: return hipErrorInvalidValue;
    }
    return hipSuccess;
  };
  hipError_t e;
  if constexpr (DT == DT_F64 && BM == 128) e = ilv ? go(std::true_type()) : go(std::false_type());
  else e = go(std::false_type());
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

template <int DT, int BM, int BK>
int occupancy_cfg() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, gemm_kernel<DT, BM, BK, EPI_RK4>, gemm_nt<DT, BM>(), 0) !=
          hipSuccess ||
      nb < 1)
    nb = 1;
  return nb;
}

}  // namespace

// Supported configurations: bm in {64, 128}; bk per dtype.
#define FM_CFG_LIST(X) \
  X(DT_F64, 128, 16)   \
  X(DT_F64, 128, 32)   \
  X(DT_F64, 64, 16)    \
  X(DT_F64, 64, 32)    \
  X(DT_F32, 128, 32)   \
  X(DT_F32, 128, 16)   \
  X(DT_F32, 64, 32)    \
  X(DT_BF16, 128, 64)  \
  X(DT_BF16, 128, 32)  \
  X(DT_BF16, 256, 32)  \
  X(DT_BF16, 256, 64)  \
  X(DT_BF16, 64, 64)   \
  X(DT_F16, 128, 64)   \
  X(DT_F16, 128, 32)   \
  X(DT_F16, 256, 32)   \
  X(DT_F16, 256, 64)   \
  X(DT_F16, 64, 64)    \
  X(DT_BF16X3, 128, 64) \
  X(DT_BF16X3, 256, 32) \
  X(DT_BF16X3, 64, 64)

hipError_t launch_gemm(const GemmCfg& cfg, int epi, const GItem* items, const int* tile_start, int nitems,
                       int total_tiles, int grid, const int* live, hipStream_t st) {
  if (total_tiles <= 0 || nitems <= 0) return hipSuccess;
  if (grid > total_tiles) grid = total_tiles;
  if (grid >= 8) grid &= ~7;  // whole XCD rounds (see the tile split in the kernel)
  if (grid < 1) grid = 1;
#define FM_DISPATCH(D, M, K) \
  if (cfg.dt == D && cfg.bm == M && cfg.bk == K) return launch_cfg<D, M, K>(epi, items, tile_start, nitems, total_tiles, grid, live, st);
  FM_CFG_LIST(FM_DISPATCH)
#undef FM_DISPATCH
  return hipErrorInvalidValue;
}

std::vector<GemmCfg> gemm_configs(int dt) {
  std::vector<GemmCfg> v;
#define FM_LIST(D, M, K) \
  if (dt == D) v.push_back(GemmCfg{D, M, K});
  FM_CFG_LIST(FM_LIST)
#undef FM_LIST
  return v;
}

int gemm_max_grid(const GemmCfg& cfg) {
  // queried once per (device, configuration), then served from a table
  static std::mutex mu;
  static std::map<std::tuple<int, int, int, int>, int> cache;
  int dev = 0;
  (void)hipGetDevice(&dev);
  const auto key = std::make_tuple(dev, cfg.dt, cfg.bm, cfg.bk);
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 256;
  int occ = 1;
#define FM_OCC(D, M, K) \
  if (cfg.dt == D && cfg.bm == M && cfg.bk == K) occ = occupancy_cfg<D, M, K>();
  FM_CFG_LIST(FM_OCC)
#undef FM_OCC
  cache[key] = cus * occ;
  return cus * occ;
}

}  // namespace fm
