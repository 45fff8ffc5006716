/*
 * fm.h -- C interface of the MI355X (gfx950) parareal matrix-function library.
 *
 * The library evaluates f(A) for a dense real n x n matrix A as the value at
 * time T of a matrix ODE (the homotopy model of Sec. 1 of Chehab & Petcu,
 * "Parallel Matrix Function Evaluation via Initial value ODE modelling") or as
 * the stable steady state of one (the steady-state model of Sec. 1 / Sec. 4),
 * integrating the ODE with the classical parareal algorithm (Sec. 2, Alg. 1):
 * a cheap coarse propagator G swept serially over N time slices, corrected by
 * an accurate fine propagator F whose N slice solves are independent.
 *
 * Conventions shared by every entry point:
 *  - Matrices are FP64, row-major.  Pointers marked "device" are HIP device
 *    pointers of the device that was current at fm_flow_create; pointers
 *    marked "host" are ordinary host memory.  Pointer arrays (const double*
 *    const*) are host arrays of `batch` device pointers.
 *  - Every call returns an fm_status; nothing throws across the interface.
 *    On an error the thread-local message of fm_last_error() says why; no
 *    output is written unless the status is FM_OK or FM_WARN_NOT_CONVERGED.
 *  - hip_stream is a hipStream_t (NULL = the default stream).  Calls order
 *    their device work on it.  fm_parareal_solve synchronises with it (it reads
 *    one scalar per iteration); the propagators are asynchronous.
 *  - A flow object is not thread-safe: calls on one flow must not overlap.
 */
#ifndef FM_H
#define FM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fm_flow_s* fm_flow;  /* opaque; owned by the library */

typedef enum {
  FM_OK = 0,
  FM_WARN_NOT_CONVERGED = 1,  /* result written: the iterate after max_iter */
  FM_ERR_INVALID = -1,        /* bad argument; nothing done */
  FM_ERR_NOMEM = -2,          /* device allocation failed */
  FM_ERR_DEVICE = -3,         /* HIP runtime error */
  FM_ERR_NONFINITE = -4,      /* an iterate became Inf/NaN (e.g. A(t) singular) */
  FM_ERR_UNSUPPORTED = -5     /* valid request the library does not implement */
} fm_status;

/* The matrix flows dX/dt = F(X). */
typedef enum {
  /* Sec. 2, Example 1: with A(t) = I + t (A - I), Q(t) = A(t)^{-1} solves
   * dQ/dt = -Q (A - I) Q = Q (I - A) Q, Q(0) = I, Q(1) = A^{-1}.  Requires
   * A(t) invertible on [0, 1] (e.g. A with positive eigenvalues); T = 1.     */
  FM_FLOW_INV_HOMOTOPY = 1,
  /* dX/dt = X - X A X: stable steady state A^{-1} (differential -Id there). */
  FM_FLOW_INV_STEADY = 2,
  /* dX/dt = A - X^2, A symmetric positive definite: stable steady state the
   * principal square root A^{1/2}.                                           */
  FM_FLOW_SQRT_STEADY = 3,
  /* Sec. 2, Example 2: with A(t) = t A, Q(t) = exp(t A) solves dQ/dt = A Q,
   * Q(0) = I; Q(T) = exp(T A).  One product per RK4 stage; no refinement
   * (max_refine must be 0).                                                 */
  FM_FLOW_EXP = 4,
  /* Sec. 4, Example 5: dX/dt = I - A X, linear, stable steady state A^{-1}
   * when the eigenvalues of A have positive real part.  One product per RK4
   * stage; Newton-Schulz refinement as for the other inverse flows.       */
  FM_FLOW_INV_LINEAR = 5
} fm_flow_kind;

/* Arithmetic of the dense products of the propagators (MFMA input type).  The
 * parareal iterates, the correction sum, the residual and the refinement are
 * always FP64; with FM_F32/BF16/F16/BF16X3 products accumulate in FP32.  The
 * fine propagator's state is FP64 between products for FM_F64/F32 and FP32
 * inside one fine propagation for the 16-bit types (narrowed from and widened
 * back to the FP64 slice state around it).  FM_BF16X3 splits each
 * operand into BF16 hi + lo parts and forms A_hi B_hi + A_hi B_lo + A_lo B_hi
 * (three BF16 MFMA products, ~16 significant bits).  With FM_BF16/FM_F16 the
 * fixed operand B of the two quadratic flows (A - I for the homotopy, A for
 * X - X A X) is held as hi + lo planes by default (option split_b): the first
 * product of each stage field is B_hi Y + B_lo Y, both planes in one launch
 * with one FP32 accumulation (the MFMA work of three 16-bit products per
 * stage instead of two).  The rounding of B is what the condition of A(t)
 * amplifies; that of Y and of the products is damped. */
typedef enum { FM_F64 = 0, FM_F32 = 1, FM_BF16 = 2, FM_F16 = 3, FM_BF16X3 = 4 } fm_dtype;

/* Coarse propagator G. */
typedef enum {
  FM_COARSE_EULER = 0,    /* forward Euler steps */
  FM_COARSE_LEARNED = 1,  /* degree-3 polynomial step X p(K) + q(K), K =
                             h (A - I) X (homotopy) or h (A X - I) (X - X A X),
                             coefficients from the loaded network, with a
                             per-slice fallback to Euler (see fm_params)    */
  FM_COARSE_CN = 2        /* Crank-Nicolson steps (linear flows only; see
                             FM_FINE_CN)                                    */
} fm_coarse;

/* Parareal variant.  FM_PARAREAL_MODIFIED is Alg. 3 (linear homogeneous,
 * FM_FLOW_EXP) or Alg. 4 (linear affine, FM_FLOW_INV_LINEAR) of Sec. 3: the
 * iterates U^k_0..U^k_N enlarge an F-orthonormal basis (globalQR, Alg. 2;
 * Frobenius inner products, a block whose remaining norm is <= 1e-7 of its
 * own is dropped: below that its direction is dominated by rounding), the fine propagator runs on the new basis blocks only (in
 * parallel; the flows are autonomous and the slices uniform, so one fine
 * propagation per block serves every slice), and the sweep is
 *   U^{k+1}_{n+1} = F(P U^{k+1}_n) + G((I - P) U^{k+1}_n) [- G(0)],
 * F(P U) from the stored fine images by linearity.  Stopping rule, stats and
 * refinement as for Alg. 1.  The basis holds at most (max_iter + 1)(N + 1)
 * and n^2 blocks (two FP64 n x n matrices each); every problem of a batch
 * must use the same variant; coarse must be FM_COARSE_EULER. */
typedef enum { FM_PARAREAL_CLASSICAL = 0, FM_PARAREAL_MODIFIED = 1 } fm_variant;

/* Fine propagator F. */
typedef enum {
  FM_FINE_RK4 = 0,    /* classical four-stage Runge-Kutta steps */
  FM_FINE_EULER = 1,  /* forward Euler steps (the fine scheme of the paper's
                         Example 1, Sec. 2) */
  FM_FINE_CN = 2      /* Crank-Nicolson steps, the scheme of both propagators
                         in the paper's Example 2 (Sec. 2), for the linear
                         flows dX/dt = s A X + b I (FM_FLOW_EXP: s = 1, b = 0;
                         FM_FLOW_INV_LINEAR: s = -1, b = 1):
                           (I - s h/2 A) X+ = (I + s h/2 A) X + h b I.
                         Per step size h the library forms
                         Y = (I - s h/2 A)^{-1} once by an FP64 Newton-Schulz
                         iteration from Y = I (requires (h/2) ||A||_inf < 0.75,
                         else FM_ERR_UNSUPPORTED) and D = s Y A, and takes
                         each step as X+ = X + h (D X + b Y): one product per
                         step, FP64 state */
} fm_fine;

typedef struct {
  int32_t kind;      /* fm_flow_kind */
  int32_t reserved;  /* must be 0 */
  int64_t n;         /* order, 1 <= n <= 16384 */
  const double* A;   /* device, n x n, row-major, leading dimension lda; copied
                        at fm_flow_create, may be freed afterwards        */
  int64_t lda;       /* >= n */
} fm_problem;

/* Problem statement of Alg. 1 (Sec. 2): time interval [0, T] in N uniform
 * slices T_n = n T / N; G = coarse_steps coarse steps per slice; F =
 * fine_steps steps of the fine scheme (fine_method) per slice.  Iteration k computes U^{k+1}
 * from U^k; it stops after the first k with
 *     max_n ||U^{k+1}_n - U^k_n||_F / ||U^{k+1}_n||_F <= tol,
 * or after max_iter iterations, or at k + 1 = N (then U equals the serial fine
 * solution).  After that, if max_refine > 0, FP64 refinement (Newton-Schulz
 * for the inverse flows, Newton with a conjugate-gradient Sylvester solve for
 * the square root) runs until the relative residual is <= refine_tol or
 * max_refine steps were made. */
typedef struct {
  double T;              /* final time; FM_FLOW_INV_HOMOTOPY requires 1.0 */
  int32_t N;             /* slices, 1..4096 */
  int32_t coarse_steps;  /* >= 1 */
  int32_t fine_steps;    /* >= 1 */
  int32_t max_iter;      /* >= 0 (0: the coarse sweep only, status FM_OK) */
  int32_t coarse;        /* fm_coarse */
  int32_t max_refine;    /* >= 0 */
  double tol;            /* >= 0 */
  double refine_tol;     /* >= 0 */
  int32_t fine_method;   /* fm_fine */
  int32_t variant;       /* fm_variant */
} fm_params;

typedef struct {
  int32_t iters;           /* parareal iterations performed, those before a
                              learned-step restart included (<= max_iter) */
  int32_t refine_steps;    /* refinement updates performed */
  int32_t learned_slices;  /* slice solves that used the learned step in the
                              last iteration (0 for Euler)                  */
  int32_t status;          /* fm_status of this instance */
  double increment;        /* last increment (see fm_params) */
  double residual_before;  /* FP64 relative residual before refinement:
                              ||I - A X||_F / sqrt(n) or ||A - X^2||_F / ||A||_F */
  double residual;         /* the same after refinement */
  double hist[64];         /* increment of iterations 1..64, in the order
                              run (across a restart)                        */
  /* Filled when the flow was created with option "timing=1" (else 0): HIP
   * event timing, on the solve's stream, of the fine propagator's GEMM
   * launches (both products of every RK4 stage).  With graphs on (the
   * default) the events bracket each replay of one RK4 step's launches;
   * with graph=0 they bracket every launch.                                */
  int32_t fine_launches;   /* number of GEMM launches timed */
  int32_t learned_restarts; /* times a learned-coarse problem restarted from
                               Step 0 with Euler after a non-finite iterate */
  double fine_ms;          /* their summed duration, milliseconds */
  double fine_flops;       /* their algorithmic flops: 2 n^3 per problem-slice
                              product */
  double fine_phase_ms;    /* duration of the whole batched fine phases */
  int32_t basis_size;      /* FM_PARAREAL_MODIFIED: blocks in the basis at
                              the end (0 for the classical variant) */
  int32_t reserved;
} fm_stats;

/*
 * Create a flow object for `batch` problems (each its own A, n and kind) whose
 * products run in `dtype`.  Stages A on the device (padded copy, A - I, the
 * dtype copies); allocates the parareal workspace lazily in the first solve.
 * options: NULL or "key=value;key=value": coarse_model=<path> loads learned
 * coarse weights (file written by the training script), autotune=0|1 (default
 * 1: on first use of an order, time the candidate tile shapes and the
 * candidate padded orders, the multiples of 64, 128 and 256 at or above n;
 * 0: the multiple of 64 and a default tile), pad=64|128|256 (fixed padding
 * multiple instead of the tuned one), coarse_f64=0|1 (default 0: coarse-step
 * products, Euler or learned, in FP64 for an FP32 or 16-bit flow, so that the
 * coarse step's own rounding does not floor the parareal increment),
 * split_b=0|1 (default 1 for FM_BF16 and FM_F16: the fixed operand of the
 * quadratic flows as hi + lo planes, see fm_dtype; 0: one plane),
 * autotune_cache=<path>,
 * timing=0|1 (default 0: fill the timing fields of fm_stats), verbose=0|1
 * (one stderr line per parareal iteration and per tile choice),
 * tile=<bm>x<bk> (fixed product tile instead of the autotuned one, for the
 * products in the flow's dtype; FM_ERR_INVALID unless compiled for that
 * dtype: FP64 128x16, 128x32, 64x16, 64x32; FP32 128x32, 128x16, 64x32;
 * BF16 and FP16 128x64, 128x32, 256x32, 256x64, 64x64; split BF16 128x64,
 * 256x32, 64x64; problems are then padded to a multiple of 64, and the tile
 * is ignored for a problem whose padded order it does not divide),
 * graph=0|1 (default 1: the launches of one RK4 step of a fine phase are
 * captured in a hipGraph and replayed for every step).
 * Tile shapes and graphs never change results; the padded order can change
 * them at rounding level only (the summation order of norms and dot products).
 * out: host; receives the handle.  Returns FM_ERR_INVALID for batch < 1,
 * n out of range, lda < n, an unknown kind/dtype or a NULL A, and
 * FM_ERR_NONFINITE when an A holds an Inf or NaN entry (nothing is created).
 */
fm_status fm_flow_create(fm_flow* out, const fm_problem* problems, int32_t batch,
                         int32_t dtype, const char* options, void* hip_stream);

/*
 * Run Alg. 1 on every problem of the flow and write f(A) (the last slice,
 * after refinement) to X_out[b].  X0: host array of device pointers to the
 * n x n initial values, or NULL for X0 = I (the choice of Sec. 2, Example 1).
 * prm: host, `batch` entries (problem b uses prm[b]).  stats: host, `batch`
 * entries, may be NULL.  Returns the worst status over the batch.
 */
fm_status fm_parareal_solve(fm_flow f, const double* const* X0, double* const* X_out,
                            const fm_params* prm, fm_stats* stats, void* hip_stream);

/*
 * Fine propagator F(t_next, t_cur, X) of Alg. 1: `steps` classical RK4 steps of
 * size (t_next - t_cur) / steps, for every problem b: X_out[b] = F(X_in[b]).
 * X_in, X_out: host arrays of device pointers (n x n each); X_out[b] may
 * equal X_in[b].
 */
fm_status fm_fine_propagate(fm_flow f, double t_next, double t_cur, int32_t steps,
                            const double* const* X_in, double* const* X_out,
                            void* hip_stream);

/* Size in bytes of the fixed device scratch of fm_fine_propagate_noalloc
 * (one copy per GPU, held for the life of the process). */
#define FM_NOALLOC_SCRATCH_BYTES (64ull << 20)

/*
 * fm_fine_propagate without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the same propagation and the same kernels, with
 * the workspace taken from a fixed device array of FM_NOALLOC_SCRATCH_BYTES
 * instead of the flow's grown workspace, no graph capture and no timing
 * events.  The workspace needs, summed over the flow's problems of padded
 * order np, np^2 (40 bytes for FM_F64, 24 for FM_F32, 18 for FM_BF16/F16
 * plus 4 for their FP32 state, 28 for FM_BF16X3) rounded up to 256 bytes
 * per matrix; more returns FM_ERR_INVALID (nothing launched).  The flow
 * itself (fm_flow_create) is allocated beforehand.  All calls on one GPU
 * share its one array: calls that overlap on a GPU (concurrent streams,
 * host threads) race and must be serialised by the caller.  The array holds
 * the last call's intermediates; every call overwrites what it reads.
 * Blocks until the item lists are staged, otherwise asynchronous.
 */
fm_status fm_fine_propagate_noalloc(fm_flow f, double t_next, double t_cur, int32_t steps,
                                    const double* const* X_in, double* const* X_out,
                                    void* hip_stream);

/*
 * Coarse propagator G(t_next, t_cur, X) of Alg. 1: `steps` forward-Euler steps
 * (coarse = FM_COARSE_EULER) or learned polynomial steps (FM_COARSE_LEARNED,
 * needs a loaded model; no fallback here), same layout as fm_fine_propagate.
 */
fm_status fm_coarse_propagate(fm_flow f, double t_next, double t_cur, int32_t steps,
                              int32_t coarse, const double* const* X_in,
                              double* const* X_out, void* hip_stream);

/* Sec. 4, Example 5, Alg. 8 (acceleration of convergence in time towards
 * A^{-1}): for every problem of the flow, all of kind FM_FLOW_INV_LINEAR,
 *     X_{k+1} = X_k + dt (I - A X_k + u_k),   u_{k+1} = (I - dt A) u_k,
 *     u_0 = E,   k = 0 .. steps-1,
 * where u_k is added only while k < accel_steps (accel_steps >= steps: at
 * every step, as Alg. 8 is printed; a smaller value switches the accelerator
 * off at t* = accel_steps dt, the cut-off control of Example 4).  With E = 0
 * this is forward-Euler time marching on dX/dt = I - A X.
 * X0, E: host arrays of `batch` device pointers to n x n FP64 row-major
 *   matrices (leading dimension n); the array itself or an entry may be NULL
 *   (zero matrix).  E approximates A^{-1} - X0 (the paper builds it from an
 *   incomplete factorisation or a thresholded inverse; the caller supplies it).
 * X_out: device n x n FP64 per problem, written with X_steps.
 * hist: NULL, or a host array of batch * (steps / every + 1) doubles that
 *   receives ||I - A X_k||_F (FP64 product) for k = 0, every, 2 every, ...:
 *   hist[i * (steps / every + 1) + j] for problem i, k = j every.
 * Products in the flow's dtype with FP64 X and u; blocks until done.
 * Errors: FM_ERR_INVALID for dt <= 0, negative counts, every < 1 with hist,
 * a flow of another kind or NULL X_out. */
fm_status fm_aima(fm_flow f, const double* const* X0, const double* const* E, double dt, int32_t steps,
                  int32_t accel_steps, int32_t every, double* const* X_out, double* hist, void* hip_stream);

/* Sec. 3, Alg. 5: cos(A) for a device n x n FP64 matrix A (row-major,
 * leading dimension lda), 1 <= n <= 8192.  m = the smallest m >= 0 with
 * 2^-m ||A||_inf <= 1 and A0 = 2^-m A; cos(A0) is the leading n x n block of
 * exp(M), M = [[0, -A0], [A0, 0]] (the sine/cosine system of Example 3 with
 * X0 = 0 in real form), computed as the FM_FLOW_EXP flow of order 2n by
 * fm_parareal_solve with *prm (T must be 1, max_refine 0; variant, grids
 * and schemes as given; products in `dtype`); then cos(2X) = 2 cos(X)^2 - I
 * is applied m times in FP64.  C_out: device n x n, leading dimension n.
 * m_out (host, may be NULL) receives m; stats (host, may be NULL) those of
 * the parareal solve.  Allocates its workspace (2n x 2n matrices) per call;
 * blocks until done.  Returns the solve's status (FM_WARN_NOT_CONVERGED
 * included) or an error. */
fm_status fm_cos(const double* A, int64_t n, int64_t lda, int32_t dtype, const fm_params* prm, double* C_out,
                 int32_t* m_out, fm_stats* stats, const char* options, void* hip_stream);

/* Release the flow and all its device memory.  NULL is accepted. */
void fm_destroy(fm_flow f);

/* Thread-local message of the last error (empty string if none). */
const char* fm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FM_H */
