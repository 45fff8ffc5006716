// Internal declarations shared by the HIP sources of libfm (not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace fm {

// Product arithmetic (same numbering as fm_dtype in include/fm.h).
// DT_BF16X3: split BF16, a matrix is two BF16 planes (hi, lo = bf16(x - hi))
// stored back to back; products are A_hi B_hi + A_hi B_lo + A_lo B_hi.
enum Dt : int { DT_F64 = 0, DT_F32 = 1, DT_BF16 = 2, DT_F16 = 3, DT_BF16X3 = 4 };

// bytes per matrix element in the operand type (both planes for DT_BF16X3)
inline int dt_size(int dt) { return dt == DT_F64 ? 8 : (dt == DT_F32 || dt == DT_BF16X3 ? 4 : 2); }
// accumulator element size (FP64 for the FP64 path, FP32 otherwise)
inline int acc_size(int dt) { return dt == DT_F64 ? 8 : 4; }

// Epilogues fused into the GEMM C = A_op * B_op (n x n, padded order np).
enum Epi : int {
  // out0 = s0*acc + s1*E + s2*delta_ij.  E = in0 (may be null).
  EPI_AFFINE = 0,
  // RK4 stage `stage` (1..4) of X' = F(X) with k = s0*acc + s1*E, h = s2;
  // x = FP64 state, out1 = stage accumulator, out0 = next stage operand.
  EPI_RK4 = 1,
  // forward Euler: out1(FP64) = x + s2*(s0*acc + s1*E); out0 = op(out1).
  EPI_EULER = 2,
  // learned step, third product: out0 = c0 I + c1 K + c2 K2 + c3 acc (= p(K)),
  // out1 = acc (= K^3);  K = in0, K2 = in1 (op type); c = s[0..7].
  EPI_POLYP = 3,
  // learned step, last product: out1(FP64) = acc + c4 I + c5 K + c6 K2 + c7 K3,
  // out0 = op(out1);  K = in0, K2 = in1, K3 = in2.
  EPI_POLYX = 4,
};

// flags of a GEMM item
enum : int {
  F_OUT0_F64 = 1,   // out0 is FP64 (else operand type)
  F_E_F64 = 2,      // in0 is FP64 (else operand type) -- EPI_AFFINE/RK4/EULER
  F_E_NONE = 4,     // no E term
  F_X_F32 = 8,      // the RK4 state x is FP32 (16-bit products only)
  F_SPLIT_A = 16,   // BF16/FP16: a is two planes (hi, lo at + np^2); product = a_hi b + a_lo b
};

// One matrix product of a grouped launch.  All matrices are np x np,
// row-major with leading dimension np, zero outside the leading n x n block.
struct GItem {
  const void* a;    // left operand (operand type)
  const void* b;    // right operand (operand type)
  void* out0;
  void* out1;
  const void* in0;
  const void* in1;
  const void* in2;
  double* x;        // state for EPI_RK4 / EPI_EULER: FP64, or FP32 with F_X_F32
  double s[8];
  int np;
  int stage;
  int flags;
  int n;            // order of the unpadded problem (diagonal terms only for i < n)
  int inst;         // problem index (tiles of problems with live[inst] == 0 are skipped)
  int pad_;
};

// Tile configurations (one compiled kernel each).
struct GemmCfg {
  int dt;   // Dt
  int bm;   // workgroup tile (square)
  int bk;   // K tile
};

// Launch a grouped product over `nitems` items (device array `items`,
// device array `tile_start` of nitems+1 prefix sums of (np/bm)^2).
// All items must have np % cfg.bm == 0.  Returns hipSuccess or the launch error.
// tile_start[0] may be non-zero (a sub-range of a longer list): tiles are
// counted relative to it.  live: per-problem flags, or null for all live.
hipError_t launch_gemm(const GemmCfg& cfg, int epi, const GItem* items, const int* tile_start,
                       int nitems, int total_tiles, int grid, const int* live, hipStream_t st);

// All compiled tile configurations for a dtype (first = default).
std::vector<GemmCfg> gemm_configs(int dt);

// Number of workgroups a persistent launch of `cfg` should use (all tiles
// resident at most once): CUs * resident WGs per CU.
int gemm_max_grid(const GemmCfg& cfg);

// ---- elementwise / reduction kernels (ew.hip) ----
// dst(np x np, FP64) <- src (n x n, ld) zero padded
hipError_t stage_pad_f64(double* dst, int np, const double* src, int64_t n, int64_t ld, hipStream_t st);
// dst(op dtype, np x np) <- src(FP64) + shift*I (shift only on the leading n x n diagonal)
hipError_t convert_f64(void* dst, int dt, const double* src, double shift, int n, int np, hipStream_t st);
// The same as two planes of a 16-bit type (DT_BF16 or DT_F16): hi = op(v) at
// dst, lo = op(v - hi) at dst + np*np elements.
hipError_t convert_split_f64(void* dst, int dt, const double* src, double shift, int n, int np, hipStream_t st);
// dst (count elements of dtype dt) <- a fixed non-trivial pattern (for timing)
hipError_t fill_pattern(void* dst, int dt, int64_t count, hipStream_t st);
// dst(FP64 np x np) <- identity on the leading n x n block
hipError_t set_identity(double* dst, int n, int np, hipStream_t st);
// dst(FP64, np x np) <- src (n x n, ld n) padded ; or unpad dst(n x n) <- src(np)
hipError_t copy_in(double* dst, int np, const double* src, int n, hipStream_t st);
hipError_t copy_out(double* dst, int n, const double* src, int np, hipStream_t st);
hipError_t copy_f64(double* dst, const double* src, int64_t count, hipStream_t st);
// Batched copies between n x n (leading dimension n) and padded np x np FP64
// matrices: pad = 1: dst(np) <- src(n) zero padded; pad = 0: dst(n) <- src(np).
struct PadItem {
  double* dst;
  const double* src;
  int n;
  int np;
};
hipError_t launch_pad_copy(const PadItem* items, int nitems, int pad, hipStream_t st);

// Batched parareal correction: for each item j: U1 <- F + (Gnew - Gold); Gold <- Gnew;
// partial sums of ||U1 - Uold||^2 and ||U1||^2 (Uold read from U1 before the write)
// and a non-finite flag into part[j*nblk*2 ...].
struct CorrItem {
  double* u;          // U_{n+1} (in: U^k, out: U^{k+1})
  const double* f;    // F(U^k_n)
  const double* gnew; // G(U^{k+1}_n)
  double* gold;       // G(U^k_n) (updated to gnew)
  int64_t count;      // np*np
  int inst;           // problem index (skipped when live[inst] == 0)
  int slot;           // partial sums go to part[(slot * nblk + block) * 3 ...]
};
hipError_t launch_correction(const CorrItem* items, int nitems, double* part, int nblk, const int* live,
                             hipStream_t st);

// Batched fine-solve preparation: for each item, fo <- u (FP64 copy) and
// y <- op(u).  Items of non-live problems are skipped.
struct PrepItem {
  const double* u;
  double* fo;   // may be null (no copy)
  void* y;
  int64_t count;
  int inst;
  int pad_;
};
hipError_t launch_prep(const PrepItem* items, int nitems, int dt, const int* live, hipStream_t st);
// Batched precision change of whole matrices: FP64 -> FP32 (narrow = 1,
// round to nearest) or FP32 -> FP64 (narrow = 0, exact).
struct CastItem {
  const void* src;
  void* dst;
  int64_t count;
  int narrow;
  int pad_;
};
hipError_t launch_cast(const CastItem* items, int nitems, hipStream_t st);
// Deterministic reduction of `nitems` x nblk partial pairs into per-item
// (||d||^2, ||u||^2, nonfinite) triples in out[3*j].
hipError_t launch_reduce_pairs(const double* part, int nitems, int nblk, double* out, hipStream_t st);

// sum of squares / dot products (FP64, deterministic two-level)
hipError_t launch_dot(const double* a, const double* b, int64_t count, double* part, int nblk,
                      double* out, hipStream_t st);
// y <- y + alpha * x  (alpha read from device scalar *alpha_d times sign)
hipError_t launch_axpy_dev(double* y, const double* x, const double* alpha_d, double sign,
                           int64_t count, hipStream_t st);

// Batched FP64 dot products: out[item.slot] = <a, b> for every item
// (two-level, fixed order).  part needs nitems * nblk doubles.
struct DotItem {
  const double* a;
  const double* b;
  int64_t count;
  int slot;
  int mode;           // 0: dot product; 1: number of non-finite entries of a
  const double* sub;  // when non-null: <a - sub, b - sub>
};
hipError_t launch_dots(const DotItem* items, int nitems, double* part, int nblk, double* out, hipStream_t st);

// Linear combinations over a basis of FP64 matrices (the projection and
// the fine images of the modified parareal, Sec. 3):
//   LIN_ORTH:  out1 = z - sum_j alpha_j q_j
//   LIN_SWEEP: out1 = z - sum_j alpha_j q_j,  out2 = sum_j alpha_j fq_j (+ c)
//   LIN_SCALE: out1 = scale * z
//   LIN_AXPY:  out1 = z + scale * c
// q, fq: device arrays of s device pointers; alpha: device, s values; the
// sum runs over j in order (deterministic).  out1 may alias z.
enum LinMode { LIN_ORTH = 0, LIN_SWEEP = 1, LIN_SCALE = 2, LIN_AXPY = 3 };
struct LinItem {
  const double* const* q;
  const double* const* fq;
  const double* alpha;
  const double* z;
  const double* c;
  double* out1;
  double* out2;
  double scale;
  int64_t count;
  int s;
  int mode;
};
hipError_t launch_lincomb(const LinItem& it, hipStream_t st);

// ||A||_inf of an n x n device matrix into out[0] (device).
hipError_t launch_norm_inf(const double* a, int64_t n, int64_t ld, double* out, hipStream_t st);
// out (2n x 2n) = [[0, -c A], [c A, 0]].
hipError_t launch_rotation_generator(double* out, const double* a, int64_t n, int64_t ld, double c, hipStream_t st);

// Conjugate-gradient vector updates for a batch of problems (slot = problem):
//   step1: alpha = rr[slot] / pap[slot]; h += alpha p; r -= alpha ap
//   step2: beta = rr_new[slot] / rr[slot]; p = r + beta p
struct CgItem {
  double* h;
  double* r;
  double* p;
  const double* ap;
  int64_t count;
  int slot;
  int pad_;
};
// CG start: h = 0, r = src (passed in ap), p = src
hipError_t launch_cg_init(const CgItem* items, int nitems, hipStream_t st);
// y += x for every item (h = y, ap = x)
hipError_t launch_add(const CgItem* items, int nitems, hipStream_t st);
hipError_t launch_cg_step1(const CgItem* items, int nitems, const double* rr, const double* pap, hipStream_t st);
hipError_t launch_cg_step2(const CgItem* items, int nitems, const double* rr_new, const double* rr,
                           hipStream_t st);

}  // namespace fm
