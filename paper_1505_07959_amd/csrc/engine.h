// Host-side engine of libfm: the flow object, propagators, parareal driver.
#pragma once

#include <deque>
#include <string>
#include <vector>

#include "fm.h"
#include "fm_common.h"

namespace fm {

void set_error(const char* fmt, ...);
void clear_error();

fm_status hip_status(hipError_t e, const char* what);

#define FM_HIP(expr)                                                       \
  do {                                                                     \
    hipError_t e_ = (expr);                                                \
    if (e_ != hipSuccess) return ::fm::hip_status(e_, #expr);              \
  } while (0)

#define FM_TRY(expr)                                                       \
  do {                                                                     \
    fm_status s_ = (expr);                                                 \
    if (s_ != FM_OK) return s_;                                            \
  } while (0)

// Bump allocator over one device allocation; a first pass with base == null
// only measures.
struct Arena {
  char* base = nullptr;
  size_t cap = 0;
  size_t used = 0;
  bool measuring = false;
  void* take(size_t bytes) {
    size_t off = (used + 255) & ~size_t(255);
    used = off + bytes;
    return measuring ? nullptr : base + off;
  }
  fm_status reserve(size_t bytes);
  void release();
};

// Pinned host staging ring + matching device ring for per-launch item lists.
// Valid until the next reset(), which must follow a stream synchronisation.
struct Ring {
  char* host = nullptr;
  char* dev = nullptr;
  size_t cap = 0;
  size_t used = 0;
  fm_status init(size_t bytes);
  void release();
  void reset() { used = 0; }
  size_t room() const { return cap > used + 256 ? cap - used - 256 : 0; }
  // copies `bytes` to the device on `st`; returns the device address or null
  // when full (caller synchronises, resets and retries).
  void* push(const void* data, size_t bytes, hipStream_t st);
};

// Learned coarse step: network weights and input standardisation.
struct Model {
  bool loaded = false;
  int kind = 0;                 // flow kind it was trained for
  std::vector<double> theta;    // 9288 parameters, layer by layer (W out x in row-major, then b)
  double norm[12] = {0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 1};  // mean[6], std[6] of the inputs
  float* d_theta = nullptr;     // FP32 device copies used by the network kernels
  float* d_norm = nullptr;
};

// Euler coefficients of the learned step family for `kind` and step h.
void euler_coeffs(int kind, double h, double* c);

struct Inst {
  int kind = 0;
  int n = 0, np = 0;
  bool mu_ready = false;
  GemmCfg cfg{};     // product config in the flow dtype
  GemmCfg cfg64{};   // FP64 config (residual / refinement)
  double* A64 = nullptr;  // padded FP64 A
  void* Bop = nullptr;    // left operand of the first product: A - I (homotopy) or A
  void* Blo = nullptr;    // its lo plane op(B - Bop) (16-bit products, option split_b), inside Bop's allocation
  double* B64 = nullptr;  // the same in FP64 (learned-step features; made on first use)
  double mu[4] = {0, 0, 0, 0};  // tr((A - I)^j) / n
  // Crank-Nicolson operators per step size (linear flows): D = s Y A,
  // Y = (I - s h/2 A)^{-1}; E = b Y (null when b = 0); Dop = D in the
  // product dtype (== D64 for FP64)
  struct CnOp {
    double h;
    double* D64;
    void* Dop;
    double* E;
  };
  std::deque<CnOp> cn;  // deque: references stay valid as entries are added
  double norm_inf = -1.0;  // ||A||_inf (made on first use)
};

// Per-slot buffers of one propagation.
struct FineSlot {
  int inst;
  double* x;     // FP64 state, in place
  void* ya;      // operand buffers (ya holds op(x) on entry)
  void* yb;
  void* p;
  void* kacc;
  double h;
};

struct CoarseSlot {
  int inst;
  const double* xin;  // FP64 input
  double* xout;       // FP64 output (may equal xin)
  void* y0;           // operand ping-pong
  void* y1;
  void* p;
  void* k1;           // learned step scratch
  void* k2;
  void* k3;
  double t0;          // time at the slot start (learned-step network input)
  double h;           // substep size
  int learned;        // 1: learned polynomial step, 0: Euler (or Crank-Nicolson)
  const double* coef; // host: 8 coefficients per substep (learned)
  int cn = 0;         // 1: Crank-Nicolson substeps (linear flows)
};

struct Flow {
  int device = 0;
  int dt = 0;
  int batch = 0;
  std::vector<Inst> inst;
  Model model;
  bool autotune = true;
  int force_bm = 0, force_bk = 0;  // option tile=<bm>x<bk>: fixed product tile (flow dtype)
  int force_pad = 0;                // option pad=64|128|256: fixed padding multiple
  bool coarse64 = false;            // option coarse_f64=1: coarse-step products in FP64
  bool split_b = true;              // option split_b=0|1: 16-bit fixed operand as hi + lo planes
  // bytes per element of the coarse step's operand scratch
  size_t coarse_esz() const { return coarse64 ? 8 : dt_size(dt); }
  fm_status ensure_b64(int i, hipStream_t st);
  std::string autotune_cache;
  Ring ring;
  Arena work;      // parareal workspace
  Arena prop;      // propagator workspace (fm_fine/coarse_propagate)
  double* part = nullptr;   // reduction partials
  size_t part_cap = 0;
  float* x32buf = nullptr;  // FP32 states of the 16-bit fine solves
  size_t x32_cap = 0;
  double* hredu = nullptr;  // pinned host copy of reduced triples
  size_t hredu_cap = 0;

  // optional HIP-event timing of the fine propagator (option timing=1)
  bool timing = false;
  bool verbose = false;  // option verbose=1: one stderr line per parareal iteration
  bool use_graph = true; // option graph=0|1: replay the RK4 step of a fine phase from a hipGraph (timing=1 too)
  hipStream_t cap_stream = nullptr;          // capture stream (default priority)
  std::vector<hipGraphExec_t> pending_exec;  // executable graphs kept until the next synchronisation
  std::vector<hipGraph_t> pending_graph;
  std::vector<hipStream_t> pending_stream;  // stream each pending graph was launched on
  void release_graphs();
  std::vector<hipEvent_t> ev;      // event pool
  size_t ev_used = 0;
  // one timed interval: start-event index, algorithmic flops, GEMM launches
  // (one RK4 step of a fine phase, replayed from its graph, or one launch)
  struct Timed {
    int ev;
    double flops;
    int launches;
  };
  std::vector<Timed> ev_pairs;
  std::vector<int> phase_pairs;    // start-event index of each fine phase
  int64_t t_launches = 0;
  double t_ms = 0, t_flops = 0, t_phase_ms = 0;
  hipEvent_t next_event();
  fm_status collect_timing();      // after a synchronisation: fold recorded pairs into the totals

  ~Flow();
  fm_status init(const fm_problem* p, int32_t batch, int32_t dtype, const char* options, hipStream_t st);

  // launch helpers
  fm_status gemm_groups(int epi, std::vector<GItem>& items, const std::vector<int>& item_inst, bool f64,
                        hipStream_t st);
  fm_status push(const void* data, size_t bytes, void** dev, hipStream_t st);
  // make sure `bytes` of item lists can be pushed without an intermediate reset
  fm_status reserve_ring(size_t bytes, hipStream_t st);
  fm_status ensure_part(size_t count);
  fm_status ensure_x32(size_t count);
  // batched zero-padded copies in (pad = 1) or out (pad = 0) of the library layout
  fm_status pad_copy(const std::vector<double*>& dst, const std::vector<const double*>& src, int pad,
                     hipStream_t st);
  fm_status ensure_hredu(size_t count);

  // plain: no graph capture and no timing events (nothing allocated); x32_ws:
  // FP32 states of a 16-bit fine solve taken from the caller's workspace
  // instead of the flow's grown buffer
  fm_status run_fine(const std::vector<FineSlot>& slots, int steps, int method, hipStream_t st,
                     float* x32_ws = nullptr, bool plain = false);
  fm_status run_coarse(const std::vector<CoarseSlot>& slots, int steps, hipStream_t st);
  // coefficients for rows (problem, t, h): c = c_Euler(h) + net(t, h, mu)
  struct CoefRow {
    int inst;
    double t, h;
  };
  fm_status learned_table(const std::vector<CoefRow>& rows, double* coef, hipStream_t st);
  fm_status ensure_moments(hipStream_t st);
  fm_status features(double h, const double* const* X, const double* const* FX, double* G, double* bD,
                     double* fD, double* fn, int64_t row0, hipStream_t st);
  fm_status set_model(int kind, const double* theta, const double* norm);

  // ws == nullptr: workspace from the flow's propagator arena (grown on
  // demand); else the caller's ws_cap bytes at ws, and nothing is allocated
  // Crank-Nicolson operators of problem i for step size h (built once)
  fm_status ensure_cn(int i, double h, hipStream_t st, const Inst::CnOp** out);
  fm_status fine_propagate(double t1, double t0, int steps, const double* const* xin, double* const* xout,
                           hipStream_t st, char* ws = nullptr, size_t ws_cap = 0);
  fm_status coarse_propagate(double t1, double t0, int steps, int coarse, const double* const* xin,
                             double* const* xout, hipStream_t st);
  fm_status double_angle(double* C, int m, hipStream_t st);
  fm_status solve_modified(int i, const double* X0, double* Xout, const fm_params* prm, fm_stats* stats,
                           hipStream_t st);
  fm_status aima(const double* const* X0, const double* const* E, double dt, int steps, int accel_steps, int every,
                 double* const* Xout, double* hist, hipStream_t st);
  fm_status solve(const double* const* X0, double* const* Xout, const fm_params* prm, fm_stats* stats,
                  hipStream_t st);
  fm_status refine(const std::vector<int>& which, std::vector<double*>& X, const fm_params* prm,
                   fm_stats* stats, hipStream_t st);

  fm_status load_model(const std::string& path);
  GemmCfg pick_cfg(int dt, int np);
  int pick_order(int dt, int n);
};

// Scratch of the allocation-free entry point (noalloc.hip): a fixed device
// array per GPU.  noalloc_setup() looks up its address on the current device
// once (called at flow creation); noalloc_scratch() returns it (null before
// setup).
constexpr size_t kNoallocScratchBytes = FM_NOALLOC_SCRATCH_BYTES;
fm_status noalloc_setup();
char* noalloc_scratch(int device);

}  // namespace fm
