// C interface of libfm (declared in include/fm.h): argument validation and
// dispatch to the engine.  No exception crosses the interface.
#include <cmath>
#include <new>

#include "engine.h"

namespace fm {
const char* last_error();
}

struct fm_flow_s {
  fm::Flow impl;
};

using fm::set_error;

static fm_status check_flow(fm_flow f) {
  if (!f) {
    set_error("flow handle is NULL");
    return FM_ERR_INVALID;
  }
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != f->impl.device) {
    set_error("flow was created on device %d but device %d is current", f->impl.device, dev);
    return FM_ERR_INVALID;
  }
  return FM_OK;
}

static fm_status check_ptrs(const fm_flow f, const void* const* p, const char* name) {
  if (!p) {
    set_error("%s is NULL", name);
    return FM_ERR_INVALID;
  }
  for (int i = 0; i < f->impl.batch; ++i)
    if (!p[i]) {
      set_error("%s[%d] is NULL", name, i);
      return FM_ERR_INVALID;
    }
  return FM_OK;
}

extern "C" {

fm_status fm_flow_create(fm_flow* out, const fm_problem* problems, int32_t batch, int32_t dtype,
                         const char* options, void* hip_stream) {
  fm::clear_error();
  if (!out || !problems) {
    set_error("out and problems must be non-NULL");
    return FM_ERR_INVALID;
  }
  *out = nullptr;
  if (batch < 1 || batch > (1 << 20)) {
    set_error("batch %d out of range [1, 2^20]", batch);
    return FM_ERR_INVALID;
  }
  if (dtype < FM_F64 || dtype > FM_BF16X3) {
    set_error("unknown dtype %d", dtype);
    return FM_ERR_INVALID;
  }
  for (int i = 0; i < batch; ++i) {
    const fm_problem& p = problems[i];
    if (p.kind < FM_FLOW_INV_HOMOTOPY || p.kind > FM_FLOW_INV_LINEAR) {
      set_error("problem %d: unknown flow kind %d", i, p.kind);
      return FM_ERR_INVALID;
    }
    if (p.n < 1 || p.n > 16384 || p.lda < p.n || !p.A || p.reserved != 0) {
      set_error("problem %d: need 1 <= n <= 16384, lda >= n, A != NULL, reserved == 0", i);
      return FM_ERR_INVALID;
    }
  }
  fm_flow f = new (std::nothrow) fm_flow_s;
  if (!f) {
    set_error("host allocation failed");
    return FM_ERR_NOMEM;
  }
  fm_status s = f->impl.init(problems, batch, dtype, options, (hipStream_t)hip_stream);
  if (s != FM_OK) {
    delete f;
    return s;
  }
  *out = f;
  return FM_OK;
}

fm_status fm_parareal_solve(fm_flow f, const double* const* X0, double* const* X_out, const fm_params* prm,
                            fm_stats* stats, void* hip_stream) {
  fm::clear_error();
  fm_status s = check_flow(f);
  if (s != FM_OK) return s;
  if ((s = check_ptrs(f, (const void* const*)X_out, "X_out")) != FM_OK) return s;
  if (!prm) {
    set_error("prm is NULL");
    return FM_ERR_INVALID;
  }
  for (int i = 0; i < f->impl.batch; ++i) {
    const fm_params& p = prm[i];
    if (!(p.T > 0) || !std::isfinite(p.T) || p.N < 1 || p.N > 4096 || p.coarse_steps < 1 || p.fine_steps < 1 ||
        p.max_iter < 0 || p.max_refine < 0 || !(p.tol >= 0) || !(p.refine_tol >= 0) ||
        (p.coarse != FM_COARSE_EULER && p.coarse != FM_COARSE_LEARNED && p.coarse != FM_COARSE_CN) ||
        (p.fine_method != FM_FINE_RK4 && p.fine_method != FM_FINE_EULER && p.fine_method != FM_FINE_CN) ||
        (p.variant != FM_PARAREAL_CLASSICAL && p.variant != FM_PARAREAL_MODIFIED)) {
      set_error("prm[%d]: need T > 0, 1 <= N <= 4096, steps >= 1, max_iter >= 0, tol >= 0, known coarse and "
                "fine schemes and a known variant", i);
      return FM_ERR_INVALID;
    }
    if (p.variant != prm[0].variant) {
      set_error("prm[%d]: every problem of a batch must use the same parareal variant", i);
      return FM_ERR_UNSUPPORTED;
    }
    if (p.variant == FM_PARAREAL_MODIFIED &&
        ((f->impl.inst[i].kind != FM_FLOW_EXP && f->impl.inst[i].kind != FM_FLOW_INV_LINEAR) ||
         p.coarse != FM_COARSE_EULER)) {
      set_error("prm[%d]: the modified parareal needs a linear flow (FM_FLOW_EXP, FM_FLOW_INV_LINEAR) and "
                "Euler coarse steps", i);
      return FM_ERR_UNSUPPORTED;
    }
    if (f->impl.inst[i].kind == FM_FLOW_EXP && p.max_refine != 0) {
      set_error("prm[%d]: the exponential flow has no refinement (max_refine must be 0)", i);
      return FM_ERR_INVALID;
    }
    if (f->impl.inst[i].kind == FM_FLOW_INV_HOMOTOPY && p.T != 1.0) {
      set_error("prm[%d]: the homotopy flow reaches A^{-1} at T = 1 only", i);
      return FM_ERR_INVALID;
    }
    if ((p.coarse == FM_COARSE_CN || p.fine_method == FM_FINE_CN) && f->impl.inst[i].kind != FM_FLOW_EXP &&
        f->impl.inst[i].kind != FM_FLOW_INV_LINEAR) {
      set_error("prm[%d]: Crank-Nicolson steps are defined for the linear flows (FM_FLOW_EXP, FM_FLOW_INV_LINEAR)",
                i);
      return FM_ERR_INVALID;
    }
    if (p.coarse == FM_COARSE_LEARNED && f->impl.inst[i].kind != FM_FLOW_INV_HOMOTOPY &&
        f->impl.inst[i].kind != FM_FLOW_INV_STEADY) {
      set_error("prm[%d]: the learned coarse step is defined for the two quadratic inverse flows only", i);
      return FM_ERR_UNSUPPORTED;
    }
  }
  return f->impl.solve(X0, X_out, prm, stats, (hipStream_t)hip_stream);
}

static fm_status check_prop(fm_flow f, double t1, double t0, int32_t steps, const double* const* X_in,
                            double* const* X_out) {
  fm_status s = check_flow(f);
  if (s != FM_OK) return s;
  if ((s = check_ptrs(f, (const void* const*)X_in, "X_in")) != FM_OK) return s;
  if ((s = check_ptrs(f, (const void* const*)X_out, "X_out")) != FM_OK) return s;
  if (steps < 1 || !std::isfinite(t1) || !std::isfinite(t0)) {
    set_error("need steps >= 1 and finite times");
    return FM_ERR_INVALID;
  }
  return FM_OK;
}

fm_status fm_fine_propagate(fm_flow f, double t_next, double t_cur, int32_t steps, const double* const* X_in,
                            double* const* X_out, void* hip_stream) {
  fm::clear_error();
  fm_status s = check_prop(f, t_next, t_cur, steps, X_in, X_out);
  if (s != FM_OK) return s;
  return f->impl.fine_propagate(t_next, t_cur, steps, X_in, X_out, (hipStream_t)hip_stream);
}

fm_status fm_fine_propagate_noalloc(fm_flow f, double t_next, double t_cur, int32_t steps,
                                    const double* const* X_in, double* const* X_out, void* hip_stream) {
  fm::clear_error();
  fm_status s = check_prop(f, t_next, t_cur, steps, X_in, X_out);
  if (s != FM_OK) return s;
  char* ws = fm::noalloc_scratch(f->impl.device);
  if (!ws) {
    set_error("the allocation-free scratch of device %d was not set up", f->impl.device);
    return FM_ERR_DEVICE;
  }
  return f->impl.fine_propagate(t_next, t_cur, steps, X_in, X_out, (hipStream_t)hip_stream, ws,
                                fm::kNoallocScratchBytes);
}

fm_status fm_coarse_propagate(fm_flow f, double t_next, double t_cur, int32_t steps, int32_t coarse,
                              const double* const* X_in, double* const* X_out, void* hip_stream) {
  fm::clear_error();
  fm_status s = check_prop(f, t_next, t_cur, steps, X_in, X_out);
  if (s != FM_OK) return s;
  if (coarse != FM_COARSE_EULER && coarse != FM_COARSE_LEARNED && coarse != FM_COARSE_CN) {
    set_error("unknown coarse kind %d", coarse);
    return FM_ERR_INVALID;
  }
  if (coarse == FM_COARSE_CN)
    for (int i = 0; i < f->impl.batch; ++i)
      if (f->impl.inst[i].kind != FM_FLOW_EXP && f->impl.inst[i].kind != FM_FLOW_INV_LINEAR) {
        set_error("problem %d: Crank-Nicolson steps are defined for the linear flows only", i);
        return FM_ERR_INVALID;
      }
  return f->impl.coarse_propagate(t_next, t_cur, steps, coarse, X_in, X_out, (hipStream_t)hip_stream);
}

fm_status fm_aima(fm_flow f, const double* const* X0, const double* const* E, double dt, int32_t steps,
                  int32_t accel_steps, int32_t every, double* const* X_out, double* hist, void* hip_stream) {
  fm::clear_error();
  fm_status s = check_flow(f);
  if (s != FM_OK) return s;
  if ((s = check_ptrs(f, (const void* const*)X_out, "X_out")) != FM_OK) return s;
  if (!(dt > 0) || !std::isfinite(dt) || steps < 0 || accel_steps < 0 || (hist && every < 1)) {
    set_error("fm_aima: need dt > 0, steps >= 0, accel_steps >= 0 and every >= 1 with hist");
    return FM_ERR_INVALID;
  }
  for (int i = 0; i < f->impl.batch; ++i)
    if (f->impl.inst[i].kind != FM_FLOW_INV_LINEAR) {
      set_error("fm_aima: problem %d is not an FM_FLOW_INV_LINEAR flow", i);
      return FM_ERR_INVALID;
    }
  return f->impl.aima(X0, E, dt, steps, accel_steps, every, X_out, hist, (hipStream_t)hip_stream);
}

fm_status fm_cos(const double* A, int64_t n, int64_t lda, int32_t dtype, const fm_params* prm, double* C_out,
                 int32_t* m_out, fm_stats* stats, const char* options, void* hip_stream) {
  fm::clear_error();
  if (!A || !C_out || !prm || n < 1 || n > 8192 || lda < n) {
    set_error("fm_cos: need A, C_out, prm non-NULL, 1 <= n <= 8192, lda >= n");
    return FM_ERR_INVALID;
  }
  if (prm->T != 1.0 || prm->max_refine != 0) {
    set_error("fm_cos: prm.T must be 1 and prm.max_refine 0");
    return FM_ERR_INVALID;
  }
  hipStream_t st = (hipStream_t)hip_stream;
  // ||A||_inf on the device, m = smallest m >= 0 with 2^-m ||A||_inf <= 1
  double *d_norm = nullptr, *Mb = nullptr, *X = nullptr;
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(st);
    if (d_norm) (void)hipFree(d_norm);
    if (Mb) (void)hipFree(Mb);
    if (X) (void)hipFree(X);
  };
  const size_t m2 = (size_t)(2 * n) * (size_t)(2 * n);
  if (hipMalloc((void**)&d_norm, sizeof(double)) != hipSuccess || hipMalloc((void**)&Mb, m2 * 8) != hipSuccess ||
      hipMalloc((void**)&X, m2 * 8) != hipSuccess) {
    cleanup();
    set_error("fm_cos: device allocation failed");
    return FM_ERR_NOMEM;
  }
  double nrm = 0.0;
  if (fm::launch_norm_inf(A, n, lda, d_norm, st) != hipSuccess ||
      hipMemcpyAsync(&nrm, d_norm, sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess || !std::isfinite(nrm)) {
    cleanup();
    set_error("fm_cos: norm of A failed or is not finite");
    return FM_ERR_DEVICE;
  }
  int m = 0;
  while (std::ldexp(nrm, -m) > 1.0) ++m;
  if (fm::launch_rotation_generator(Mb, A, n, lda, std::ldexp(1.0, -m), st) != hipSuccess) {
    cleanup();
    set_error("fm_cos: kernel launch failed");
    return FM_ERR_DEVICE;
  }
  // exp of the 2n x 2n generator by parareal: its leading block is cos(A0)
  fm_problem big{FM_FLOW_EXP, 0, 2 * n, Mb, 2 * n};
  fm_flow fb = nullptr;
  fm_status s = fm_flow_create(&fb, &big, 1, dtype, options, hip_stream);
  if (s != FM_OK) {
    cleanup();
    return s;
  }
  double* xo[1] = {X};
  fm_status sr = fm_parareal_solve(fb, nullptr, xo, prm, stats, hip_stream);
  fm_destroy(fb);
  if (sr < 0) {
    cleanup();
    return sr;
  }
  if (hipMemcpy2DAsync(C_out, (size_t)n * 8, X, (size_t)(2 * n) * 8, (size_t)n * 8, (size_t)n,
                       hipMemcpyDeviceToDevice, st) != hipSuccess) {
    cleanup();
    set_error("fm_cos: copy of the leading block failed");
    return FM_ERR_DEVICE;
  }
  // cos(2M) = 2 cos(M)^2 - I, m times, in FP64 at order n
  fm_problem small{FM_FLOW_EXP, 0, n, A, lda};
  fm_flow fs = nullptr;
  s = fm_flow_create(&fs, &small, 1, FM_F64, nullptr, hip_stream);
  if (s != FM_OK) {
    cleanup();
    return s;
  }
  s = fs->impl.double_angle(C_out, m, st);
  fm_destroy(fs);
  cleanup();
  if (s != FM_OK) return s;
  if (m_out) *m_out = m;
  return sr;
}

void fm_destroy(fm_flow f) {
  if (!f) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(f->impl.device);
  (void)hipDeviceSynchronize();
  delete f;
  (void)hipSetDevice(cur);
}

const char* fm_last_error(void) { return fm::last_error(); }

}  // extern "C"

// ---------------------------------------------------------------- training
#include "fm_mlp.h"
#include "fm_train.h"

extern "C" {

int32_t fm_mlp_param_count(void) { return fm::mlp_param_count(); }

static fm_status launch_result(hipError_t e, const char* what) {
  if (e != hipSuccess) return fm::hip_status(e, what);
  return FM_OK;
}

fm_status fm_mlp_forward(const float* theta, const float* norm, const float* X, int64_t S, float* Y, float* acts,
                         void* hip_stream) {
  fm::clear_error();
  if (!theta || !norm || !X || !Y || S < 0) {
    set_error("fm_mlp_forward: NULL pointer or negative size");
    return FM_ERR_INVALID;
  }
  return launch_result(fm::mlp_forward(theta, norm, X, S, Y, acts, (hipStream_t)hip_stream), "mlp forward");
}

fm_status fm_mlp_loss(const float* Y, const float* cbase, const double* G, const double* bD, const double* fD,
                      const double* fn, float rho, int64_t S, float* dY, double* Ls, double* Lsum,
                      void* hip_stream) {
  fm::clear_error();
  if (!Y || !cbase || !G || !bD || !fD || !fn || !dY || !Ls || S < 0) {
    set_error("fm_mlp_loss: NULL pointer or negative size");
    return FM_ERR_INVALID;
  }
  return launch_result(fm::mlp_loss(Y, cbase, G, bD, fD, fn, rho, S, dY, Ls, Lsum, (hipStream_t)hip_stream),
                       "mlp loss");
}

fm_status fm_mlp_backward(const float* theta, const float* norm, const float* X, const float* acts,
                          const float* dY, int64_t S, float* deltas, float* grad, void* hip_stream) {
  fm::clear_error();
  if (!theta || !norm || !X || !acts || !dY || !deltas || !grad || S < 0) {
    set_error("fm_mlp_backward: NULL pointer or negative size");
    return FM_ERR_INVALID;
  }
  return launch_result(fm::mlp_backward(theta, norm, X, acts, dY, S, deltas, grad, (hipStream_t)hip_stream),
                       "mlp backward");
}

fm_status fm_mlp_adam(float* theta, const float* grad, float* m, float* v, int64_t count, int32_t t, float lr,
                      void* hip_stream) {
  fm::clear_error();
  if (!theta || !grad || !m || !v || count < 0 || t < 1) {
    set_error("fm_mlp_adam: NULL pointer, negative size or t < 1");
    return FM_ERR_INVALID;
  }
  return launch_result(fm::mlp_adam(theta, grad, m, v, count, t, lr, 0.9f, 0.999f, 1e-8f, (hipStream_t)hip_stream),
                       "adam");
}

fm_status fm_learned_features(fm_flow f, double h, const double* const* X, const double* const* FX, double* G,
                              double* bD, double* fD, double* fn, int64_t row0, void* hip_stream) {
  fm::clear_error();
  fm_status s = check_flow(f);
  if (s != FM_OK) return s;
  if ((s = check_ptrs(f, (const void* const*)X, "X")) != FM_OK) return s;
  if ((s = check_ptrs(f, (const void* const*)FX, "FX")) != FM_OK) return s;
  if (!G || !bD || !fD || !fn || row0 < 0 || !std::isfinite(h)) {
    set_error("fm_learned_features: NULL output, negative row0 or non-finite h");
    return FM_ERR_INVALID;
  }
  return f->impl.features(h, X, FX, G, bD, fD, fn, row0, (hipStream_t)hip_stream);
}

fm_status fm_trace_moments(fm_flow f, double* mu_host, void* hip_stream) {
  fm::clear_error();
  fm_status s = check_flow(f);
  if (s != FM_OK) return s;
  if (!mu_host) {
    set_error("mu_host is NULL");
    return FM_ERR_INVALID;
  }
  if ((s = f->impl.ensure_moments((hipStream_t)hip_stream)) != FM_OK) return s;
  for (int i = 0; i < f->impl.batch; ++i)
    for (int q = 0; q < 4; ++q) mu_host[i * 4 + q] = f->impl.inst[i].mu[q];
  return FM_OK;
}

fm_status fm_flow_set_coarse_model(fm_flow f, int32_t kind, const double* theta_host, const double* norm_host) {
  fm::clear_error();
  fm_status s = check_flow(f);
  if (s != FM_OK) return s;
  if (!theta_host || !norm_host || (kind != FM_FLOW_INV_HOMOTOPY && kind != FM_FLOW_INV_STEADY)) {
    set_error("fm_flow_set_coarse_model: NULL weights or a kind without learned step");
    return FM_ERR_INVALID;
  }
  return f->impl.set_model(kind, theta_host, norm_host);
}

}  // extern "C"
