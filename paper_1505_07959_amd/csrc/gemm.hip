// Grouped, persistent MFMA GEMM for gfx950 with the propagators' epilogues
// fused in.  C = A * B for square np x np row-major operands, one launch over
// a list of independent products (all time slices of all problems of one
// parareal stage).
//
// Design (CDNA4):
//  * 256 threads = 4 wavefronts in a 2 x 2 grid; each wave owns a
//    (BM/2) x (BM/2) block of C built from MFMA tiles (BM = 256 for the
//    16-bit types: 128 x 128 per wave halves LDS and L2 traffic per flop):
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

namespace fm {
namespace {

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
  static constexpr int MI = 16, V = 4, NACC = 4;
};
template <> struct Tr<DT_F32> {
  using T = float; using Acc = float; using AccV = f16v;
  using G16 = f4; using LV = f4;
  static constexpr int MI = 32, V = 4, NACC = 16;
};
template <> struct Tr<DT_BF16> {
  using T = __bf16; using Acc = float; using AccV = f16v;
  using G16 = bf8; using LV = bf8;
  static constexpr int MI = 32, V = 8, NACC = 16;
};
template <> struct Tr<DT_F16> {
  using T = _Float16; using Acc = float; using AccV = f16v;
  using G16 = h8; using LV = h8;
  static constexpr int MI = 32, V = 8, NACC = 16;
};
// split BF16: every operand matrix is two BF16 planes (hi, then lo at +np^2)
template <> struct Tr<DT_BF16X3> {
  using T = __bf16; using Acc = float; using AccV = f16v;
  using G16 = bf8; using LV = bf8;
  static constexpr int MI = 32, V = 8, NACC = 16;
};

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

// Operand-type element access; split BF16 stores hi = bf16(v) and
// lo = bf16(v - hi) in the second plane.
template <int DT>
__device__ __forceinline__ double ld_op(const void* p, int64_t idx, int64_t np2) {
  using T = typename Tr<DT>::T;
  if constexpr (DT == DT_BF16X3) return from_op(((const T*)p)[idx]) + from_op(((const T*)p)[idx + np2]);
  else return from_op(((const T*)p)[idx]);
}
template <int DT>
__device__ __forceinline__ void st_op(void* p, int64_t idx, int64_t np2, double v) {
  using T = typename Tr<DT>::T;
  const T hi = to_op<T>(v);
  ((T*)p)[idx] = hi;
  if constexpr (DT == DT_BF16X3) ((T*)p)[idx + np2] = to_op<T>(v - from_op(hi));
}

// Fused epilogue for one element (gr, gc) of item `it` (idx = gr*np + gc).
template <int DT, int EPI>
__device__ __forceinline__ void epilogue(const GItem& it, int n, int64_t idx, bool diag, double a) {
  using Acc = typename Tr<DT>::Acc;
  const double* s = it.s;
  const int64_t np2 = (int64_t)it.np * it.np;
  if constexpr (EPI == EPI_AFFINE) {
    double v = s[0] * a;
    if (!(it.flags & F_E_NONE))
      v += s[1] * ((it.flags & F_E_F64) ? ((const double*)it.in0)[idx] : ld_op<DT>(it.in0, idx, np2));
    if (diag) v += s[2];
    if (it.flags & F_OUT0_F64) ((double*)it.out0)[idx] = v;
    else st_op<DT>(it.out0, idx, np2, v);
  } else if constexpr (EPI == EPI_RK4 || EPI == EPI_EULER) {
    double k = s[0] * a;
    if (!(it.flags & F_E_NONE))
      k += s[1] * ((it.flags & F_E_F64) ? ((const double*)it.in0)[idx] : ld_op<DT>(it.in0, idx, np2));
    const double h = s[2];
    const double x = it.x[idx];
    if constexpr (EPI == EPI_EULER) {
      const double xn = x + h * k;
      ((double*)it.out1)[idx] = xn;
      st_op<DT>(it.out0, idx, np2, xn);
    } else {
      Acc* K = (Acc*)it.out1;
      switch (it.stage) {
        case 1: K[idx] = (Acc)k; st_op<DT>(it.out0, idx, np2, x + 0.5 * h * k); break;
        case 2: K[idx] = (Acc)((double)K[idx] + 2.0 * k); st_op<DT>(it.out0, idx, np2, x + 0.5 * h * k); break;
        case 3: K[idx] = (Acc)((double)K[idx] + 2.0 * k); st_op<DT>(it.out0, idx, np2, x + h * k); break;
        default: {
          const double xn = x + (h / 6.0) * ((double)K[idx] + k);
          it.x[idx] = xn;
          st_op<DT>(it.out0, idx, np2, xn);
        }
      }
    }
  } else if constexpr (EPI == EPI_POLYP) {
    double v = s[1] * ld_op<DT>(it.in0, idx, np2) + s[2] * ld_op<DT>(it.in1, idx, np2) + s[3] * a;
    if (diag) v += s[0];
    st_op<DT>(it.out0, idx, np2, v);
    st_op<DT>(it.out1, idx, np2, a);
  } else {  // EPI_POLYX
    double v = a + s[5] * ld_op<DT>(it.in0, idx, np2) + s[6] * ld_op<DT>(it.in1, idx, np2) +
               s[7] * ld_op<DT>(it.in2, idx, np2);
    if (diag) v += s[4];
    ((double*)it.out1)[idx] = v;
    st_op<DT>(it.out0, idx, np2, v);
  }
  (void)n;
}

template <int DT, int BM, int BK, int EPI>
__global__ __launch_bounds__(256, (BM == 128 && (DT != DT_F64 || BK == 16)) ? 2 : 1) void gemm_kernel(const GItem* __restrict__ items,
                                                   const int* __restrict__ tile_start, int nitems,
                                                   int total_tiles, const int* __restrict__ live) {
  using TR = Tr<DT>;
  using T = typename TR::T;
  using G16 = typename TR::G16;
  using LV = typename TR::LV;
  using AccV = typename TR::AccV;
  constexpr int MI = TR::MI, V = TR::V, NACC = TR::NACC;
  constexpr int BN = BM;
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int RM = WM / MI, RN = WN / MI;
  constexpr int NQ = 64 / MI;            // lane groups along k
  constexpr int KC = NQ * V;             // k per chunk
  constexpr int W = 16 / sizeof(T);      // elements per 16-byte chunk
  constexpr int PADA = 16 / sizeof(T);
  constexpr int LDA_S = BK + PADA;       // LDS row stride of A (elements)
  constexpr int A_CHUNKS = BM * BK / W;  // 16-byte chunks of an A tile
  constexpr int B_BLOCKS = (BK / V) * (BN / W);
  static_assert(BK % KC == 0, "BK must be a multiple of the MFMA k chunk");
  static_assert(A_CHUNKS % 256 == 0, "A tile must split evenly over 256 threads");
  static_assert(B_BLOCKS <= 256 || B_BLOCKS % 256 == 0, "B tile split");
  constexpr int A_PER_T = A_CHUNKS / 256;
  constexpr int B_PER_T = B_BLOCKS >= 256 ? B_BLOCKS / 256 : 1;
  // B column swizzle inside aligned groups of G columns (G columns = 128 bytes
  // of k-vectors): a thread stores W adjacent columns, so without it the lanes
  // of one store sit W columns apart and hit the same banks; the XOR with the
  // W-block index spreads them, and the fragment reads (consecutive columns)
  // stay a permutation of one aligned group.
  constexpr int GS = 128 / (V * (int)sizeof(T));
  auto bswz = [](int c) { return c ^ ((c / W) & (GS - 1)); };

  __shared__ __attribute__((aligned(16))) T As[2][BM * LDA_S];
  __shared__ __attribute__((aligned(16))) T Bs[2][BK * BN];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int lr = lane % MI, lq = lane / MI;

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

    G16 ra[A_PER_T];
    G16 rb[B_PER_T][V];
    bool b_active[B_PER_T];

    const int64_t np2 = (int64_t)np * np;
    const int nkps = np / BK;  // K tiles per segment
    auto gload = [&](int kt) {
      // segment 0: (A_hi, B_hi); 1: (A_hi, B_lo); 2: (A_lo, B_hi)
      const int seg = kt / nkps;
      const int k0 = (kt - seg * nkps) * BK;
      const T* __restrict__ As_g = Ag + (seg == 2 ? np2 : 0);
      const T* __restrict__ Bs_g = Bg + (seg == 1 ? np2 : 0);
#pragma unroll
      for (int u = 0; u < A_PER_T; ++u) {
        const int c = tid + 256 * u;
        const int r = c / (BK / W), cc = c % (BK / W);
        ra[u] = *(const G16*)(As_g + (int64_t)r * np + k0 + cc * W);
      }
#pragma unroll
      for (int u = 0; u < B_PER_T; ++u) {
        const int blk = tid + 256 * u;
        b_active[u] = blk < B_BLOCKS;
        if (b_active[u]) {
          const int kb = blk / (BN / W), cb = blk % (BN / W);
#pragma unroll
          for (int r = 0; r < V; ++r) rb[u][r] = *(const G16*)(Bs_g + (int64_t)(k0 + kb * V + r) * np + cb * W);
        }
      }
    };
    auto lstore = [&](int buf) {
#pragma unroll
      for (int u = 0; u < A_PER_T; ++u) {
        const int c = tid + 256 * u;
        const int r = c / (BK / W), cc = c % (BK / W);
        *(G16*)(&As[buf][r * LDA_S + cc * W]) = ra[u];
      }
#pragma unroll
      for (int u = 0; u < B_PER_T; ++u) {
        if (b_active[u]) {
          const int blk = tid + 256 * u;
          const int kb = blk / (BN / W), cb = blk % (BN / W);
#pragma unroll
          for (int w = 0; w < W; ++w) {
            LV col;
#pragma unroll
            for (int r = 0; r < V; ++r) col[r] = rb[u][r][w];
            *(LV*)(&Bs[buf][(kb * BN + bswz(cb * W + w)) * V]) = col;
          }
        }
      }
    };

    // K tiles of all segments in sequence (one segment unless split BF16)
    const int nk = nkps * nseg<DT>();
    gload(0);
    lstore(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
      const int cur = kt & 1;
      if (kt + 1 < nk) gload(kt + 1);
#pragma unroll
      for (int ch = 0; ch < BK / KC; ++ch) {
        LV a[RM], b[RN];
#pragma unroll
        for (int i = 0; i < RM; ++i)
          a[i] = *(const LV*)(&As[cur][(wr * WM + i * MI + lr) * LDA_S + ch * KC + lq * V]);
#pragma unroll
        for (int j = 0; j < RN; ++j)
          b[j] = *(const LV*)(&Bs[cur][((ch * NQ + lq) * BN + bswz(wc * WN + j * MI + lr)) * V]);
        // k-step outermost: consecutive MFMAs update different accumulators,
        // so none waits on the previous one's result
        if constexpr (DT == DT_F64 || DT == DT_F32) {
#pragma unroll
          for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int i = 0; i < RM; ++i)
#pragma unroll
              for (int j = 0; j < RN; ++j) mma1<DT>(acc[i][j], a[i][t], b[j][t]);
        } else {
#pragma unroll
          for (int i = 0; i < RM; ++i)
#pragma unroll
            for (int j = 0; j < RN; ++j) mma<DT>(acc[i][j], a[i], b[j]);
        }
      }
      if (kt + 1 < nk) lstore(cur ^ 1);
      __syncthreads();
    }

    // fused epilogue
    const int n_valid = it.n;
#pragma unroll
    for (int i = 0; i < RM; ++i)
#pragma unroll
      for (int j = 0; j < RN; ++j) {
        // one MFMA block at a time: keeps the epilogue's loads from being
        // hoisted all together (register pressure of the 256-wide tiles)
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int v = 0; v < NACC; ++v) {
          int r, c;
          acc_pos<DT>(lane, v, r, c);
          const int gr = row0 + wr * WM + i * MI + r;
          const int gc = col0 + wc * WN + j * MI + c;
          const int64_t idx = (int64_t)gr * np + gc;
          epilogue<DT, EPI>(it, n_valid, idx, gr == gc && gr < n_valid, (double)acc[i][j][v]);
        }
      }
  }
}

template <int DT, int BM, int BK>
hipError_t launch_cfg(int epi, const GItem* items, const int* ts, int nitems, int total, int grid,
                      const int* live, hipStream_t st) {
  dim3 g(grid), b(256);
  switch (epi) {
    case EPI_AFFINE: hipLaunchKernelGGL((gemm_kernel<DT, BM, BK, EPI_AFFINE>), g, b, 0, st, items, ts, nitems, total, live); break;
    case EPI_RK4: hipLaunchKernelGGL((gemm_kernel<DT, BM, BK, EPI_RK4>), g, b, 0, st, items, ts, nitems, total, live); break;
    case EPI_EULER: hipLaunchKernelGGL((gemm_kernel<DT, BM, BK, EPI_EULER>), g, b, 0, st, items, ts, nitems, total, live); break;
    case EPI_POLYP: hipLaunchKernelGGL((gemm_kernel<DT, BM, BK, EPI_POLYP>), g, b, 0, st, items, ts, nitems, total, live); break;
    case EPI_POLYX: hipLaunchKernelGGL((gemm_kernel<DT, BM, BK, EPI_POLYX>), g, b, 0, st, items, ts, nitems, total, live); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int DT, int BM, int BK>
int occupancy_cfg() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, gemm_kernel<DT, BM, BK, EPI_RK4>, 256, 0) != hipSuccess ||
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
