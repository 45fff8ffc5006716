// Host engine of libfm: staging, propagators, the parareal driver (Alg. 1 of
// Sec. 2) and the FP64 refinement.  Device work is issued on the caller's
// stream; the only host synchronisation is one small read per parareal
// iteration (the increment) and per refinement step (the residual).
#include "engine.h"
#include "fm_mlp.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <chrono>
#include <map>
#include <mutex>
#include <tuple>

namespace fm {

static thread_local std::string g_error;

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_error = buf;
}
void clear_error() { g_error.clear(); }
const char* last_error() { return g_error.c_str(); }

fm_status hip_status(hipError_t e, const char* what) {
  set_error("%s failed: %s", what, hipGetErrorString(e));
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return FM_ERR_NOMEM;
  return FM_ERR_DEVICE;
}

// ---------------------------------------------------------------- Arena/Ring
fm_status Arena::reserve(size_t bytes) {
  if (bytes <= cap && base) {
    used = 0;
    return FM_OK;
  }
  release();
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes ? bytes : 256);
  if (e != hipSuccess) return hip_status(e, "hipMalloc(workspace)");
  base = (char*)p;
  cap = bytes;
  used = 0;
  return FM_OK;
}
void Arena::release() {
  if (base) (void)hipFree(base);
  base = nullptr;
  cap = used = 0;
}

fm_status Ring::init(size_t bytes) {
  FM_HIP(hipHostMalloc((void**)&host, bytes, hipHostMallocDefault));
  FM_HIP(hipMalloc((void**)&dev, bytes));
  cap = bytes;
  used = 0;
  return FM_OK;
}
void Ring::release() {
  if (host) (void)hipHostFree(host);
  if (dev) (void)hipFree(dev);
  host = dev = nullptr;
  cap = used = 0;
}
void* Ring::push(const void* data, size_t bytes, hipStream_t st) {
  size_t off = (used + 255) & ~size_t(255);
  if (off + bytes > cap) return nullptr;
  memcpy(host + off, data, bytes);
  if (hipMemcpyAsync(dev + off, host + off, bytes, hipMemcpyHostToDevice, st) != hipSuccess) return nullptr;
  used = off + bytes;
  return dev + off;
}

fm_status Flow::push(const void* data, size_t bytes, void** d, hipStream_t st) {
  void* p = ring.push(data, bytes, st);
  if (!p) {
    // ring full: wait for the queued copies, then start over
    FM_HIP(hipStreamSynchronize(st));
    ring.reset();
    p = ring.push(data, bytes, st);
    if (!p) {
      set_error("item list of %zu bytes exceeds the staging ring", bytes);
      return FM_ERR_NOMEM;
    }
  }
  *d = p;
  return FM_OK;
}

fm_status Flow::reserve_ring(size_t bytes, hipStream_t st) {
  if (bytes + 4096 > ring.cap) {
    set_error("item lists of %zu bytes exceed the staging ring", bytes);
    return FM_ERR_NOMEM;
  }
  if (ring.room() < bytes + 4096) {
    FM_HIP(hipStreamSynchronize(st));
    ring.reset();
  }
  return FM_OK;
}

hipEvent_t Flow::next_event() {
  if (ev_used == ev.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    ev.push_back(e);
  }
  return ev[ev_used++];
}

fm_status Flow::collect_timing() {
  for (const Timed& pr : ev_pairs) {
    float ms = 0.f;
    FM_HIP(hipEventElapsedTime(&ms, ev[pr.ev], ev[pr.ev + 1]));
    t_ms += ms;
    t_flops += pr.flops;
    t_launches += pr.launches;
  }
  for (int i : phase_pairs) {
    float ms = 0.f;
    FM_HIP(hipEventElapsedTime(&ms, ev[i], ev[i + 1]));
    t_phase_ms += ms;
  }
  ev_pairs.clear();
  phase_pairs.clear();
  ev_used = 0;
  return FM_OK;
}

void Flow::release_graphs() {
  for (auto q : pending_stream) (void)hipStreamSynchronize(q);
  pending_stream.clear();
  for (auto g : pending_exec) (void)hipGraphExecDestroy(g);
  for (auto g : pending_graph) (void)hipGraphDestroy(g);
  pending_exec.clear();
  pending_graph.clear();
}

Flow::~Flow() {
  (void)hipDeviceSynchronize();
  release_graphs();
  if (cap_stream) (void)hipStreamDestroy(cap_stream);
  for (auto e : ev) (void)hipEventDestroy(e);
  if (model.d_theta) (void)hipFree(model.d_theta);
  if (model.d_norm) (void)hipFree(model.d_norm);
  for (auto& in : inst) {
    for (auto& c : in.cn) {
      if (c.Dop && c.Dop != (void*)c.D64) (void)hipFree(c.Dop);
      if (c.D64) (void)hipFree(c.D64);
      if (c.E) (void)hipFree(c.E);
    }
    if (in.A64) (void)hipFree(in.A64);
    if (in.Bop) (void)hipFree(in.Bop);
    if (in.B64) (void)hipFree(in.B64);
  }
  ring.release();
  work.release();
  prop.release();
  if (x32buf) (void)hipFree(x32buf);
  if (part) (void)hipFree(part);
  if (hredu) (void)hipHostFree(hredu);
}

fm_status Flow::pad_copy(const std::vector<double*>& dst, const std::vector<const double*>& src, int pad,
                         hipStream_t st) {
  std::vector<PadItem> it(batch);
  for (int i = 0; i < batch; ++i) it[i] = PadItem{dst[i], src[i], inst[i].n, inst[i].np};
  void* d = nullptr;
  FM_TRY(push(it.data(), it.size() * sizeof(PadItem), &d, st));
  FM_HIP(launch_pad_copy((const PadItem*)d, batch, pad, st));
  return FM_OK;
}

fm_status Flow::ensure_part(size_t count) {
  if (count <= part_cap) return FM_OK;
  if (part) (void)hipFree(part);
  part = nullptr;
  FM_HIP(hipMalloc((void**)&part, count * sizeof(double)));
  part_cap = count;
  return FM_OK;
}
// FP64 copy of the first product's right operand (A - I for the homotopy,
// else A), made once per problem.
fm_status Flow::ensure_b64(int i, hipStream_t st) {
  if (inst[i].B64) return FM_OK;
  FM_HIP(hipMalloc((void**)&inst[i].B64, (size_t)inst[i].np * inst[i].np * 8));
  FM_HIP(convert_f64(inst[i].B64, DT_F64, inst[i].A64, inst[i].kind == FM_FLOW_INV_HOMOTOPY ? -1.0 : 0.0,
                     inst[i].n, inst[i].np, st));
  return FM_OK;
}

// Growing the buffer frees the old one: hipFree waits for the device, so no
// launch still reads it.
fm_status Flow::ensure_x32(size_t count) {
  if (count <= x32_cap) return FM_OK;
  if (x32buf) (void)hipFree(x32buf);
  x32buf = nullptr;
  x32_cap = 0;
  FM_HIP(hipMalloc((void**)&x32buf, count * sizeof(float)));
  x32_cap = count;
  return FM_OK;
}
fm_status Flow::ensure_hredu(size_t count) {
  if (count <= hredu_cap) return FM_OK;
  if (hredu) (void)hipHostFree(hredu);
  hredu = nullptr;
  FM_HIP(hipHostMalloc((void**)&hredu, count * sizeof(double), hipHostMallocDefault));
  hredu_cap = count;
  return FM_OK;
}

// Flows whose stage field takes two products (first P = B Y, then Y P).
static bool two_products(int kind) { return kind == FM_FLOW_INV_HOMOTOPY || kind == FM_FLOW_INV_STEADY; }

// ------------------------------------------------------------------ configs

static int default_bk(int dt) { return dt == DT_F64 ? 16 : (dt == DT_F32 ? 32 : 64); }  // BF16X3: 64

static GemmCfg default_cfg(int d, int np) {
  GemmCfg c;
  c.dt = d;
  c.bk = default_bk(d);
  // 128-wide tiles once a product has enough of them to fill the GPU
  c.bm = (np % 128 == 0 && np >= 512) ? 128 : 64;
  return c;
}

// ---------------------------------------------------------------- autotuner
// Tile shape per (device, dtype, padded order), chosen by timing every compiled
// configuration on a batch of products of that order: an RK4 stage pair (the
// plain product and the product with the fused stage update).  All configurations sum over k in
// the same order, so the choice changes speed only, never results.  Choices are
// kept for the process and, with autotune_cache=<file>, across processes
// (lines "device dtype np bm bk ms", ms = trial time per product).
static std::mutex g_tune_mu;
static std::map<std::tuple<int, int, int>, GemmCfg> g_tune;
static std::map<std::tuple<int, int, int>, double> g_tune_ms;
static std::map<std::string, bool> g_tune_loaded;

static void tune_load(const std::string& path) {
  if (path.empty() || g_tune_loaded.count(path)) return;
  g_tune_loaded[path] = true;
  FILE* f = fopen(path.c_str(), "r");
  if (!f) return;
  int dev, d, np, bm, bk;
  double ms;
  while (fscanf(f, "%d %d %d %d %d %lf", &dev, &d, &np, &bm, &bk, &ms) == 6)
    for (const GemmCfg& c : gemm_configs(d))
      if (c.bm == bm && c.bk == bk && np % bm == 0 && np % bk == 0) {
        g_tune[{dev, d, np}] = c;
        g_tune_ms[{dev, d, np}] = ms;
      }
  fclose(f);
}

static void tune_store(const std::string& path, int dev, int d, int np, const GemmCfg& c, double ms) {
  if (path.empty()) return;
  FILE* f = fopen(path.c_str(), "a");
  if (!f) return;
  fprintf(f, "%d %d %d %d %d %.6g\n", dev, d, np, c.bm, c.bk, ms);
  fclose(f);
}

// Time one RK4 stage pair on `nb` products: the plain product P = A B
// (EPI_AFFINE) and the product with the fused stage update (EPI_RK4, FP64
// state and stage accumulator per product), as the fine propagator runs them.
static double time_cfg(const GemmCfg& c, int np, int nb, void* A, void* B, void* C, double* X, void* Kacc,
                       GItem* d_items, int* d_ts, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  const size_t esz = dt_size(c.dt), asz = acc_size(c.dt);
  const size_t np2 = (size_t)np * np;
  std::vector<GItem> items(2 * nb);
  std::vector<int> ts(nb + 1, 0);
  for (int j = 0; j < nb; ++j) {
    GItem& g = items[j];
    memset(&g, 0, sizeof g);
    g.a = A;
    g.b = B;
    g.out0 = (char*)C + (size_t)j * np2 * esz;
    g.s[0] = 1.0;
    g.flags = F_E_NONE;
    g.np = np;
    g.n = np;
    GItem& r = items[nb + j];
    r = g;
    r.b = g.out0;
    r.out0 = (char*)C + (size_t)(nb + j) * np2 * esz;  // own next-stage operand buffer
    r.out1 = (char*)Kacc + (size_t)j * np2 * asz;
    r.x = X + (size_t)j * np2;  // FP64-sized: holds the FP32 state of 16-bit products too
    if (c.dt == DT_BF16 || c.dt == DT_F16 || c.dt == DT_BF16X3) r.flags |= F_X_F32;
    r.stage = 1;
    r.s[0] = -1.0;
    r.s[2] = 1e-3;
    ts[j + 1] = ts[j] + (np / c.bm) * (np / c.bm);
  }
  if (hipMemcpyAsync(d_items, items.data(), 2 * nb * sizeof(GItem), hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(d_ts, ts.data(), (nb + 1) * sizeof(int), hipMemcpyHostToDevice, st) != hipSuccess)
    return 1e30;
  const int total = ts[nb];
  const int grid = std::min(total, gemm_max_grid(c));
  double best = 1e30;
  for (int rep = 0; rep < 3; ++rep) {
    if (hipEventRecord(e0, st) != hipSuccess) return 1e30;
    if (launch_gemm(c, EPI_AFFINE, d_items, d_ts, nb, total, grid, nullptr, st) != hipSuccess) return 1e30;
    if (launch_gemm(c, EPI_RK4, d_items + nb, d_ts, nb, total, grid, nullptr, st) != hipSuccess) return 1e30;
    if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return 1e30;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return 1e30;
    if (rep > 0) best = std::min(best, (double)ms);  // first launch warms up
  }
  return best;
}

// Padded order of a problem of order n: the multiples of 64, 128 and 256 at
// or above n (one to three distinct orders), each with its tuned tile; the
// one with the shortest trial time per product wins.  Zero padding leaves
// the leading n x n block of every product unchanged; only the summation
// order of norms and dot products over the padded matrices depends on it.  A larger order can win
// because it admits wider tiles (n = 448: 448 takes 64-wide tiles only, 512
// the 256-wide ring).  Without autotuning, or with a fixed tile, the multiple
// of 64; with option pad=<m>, the multiple of m.
int Flow::pick_order(int d, int n) {
  if (force_pad) return (n + force_pad - 1) / force_pad * force_pad;
  const int p64 = (n + 63) / 64 * 64;
  if (!autotune || force_bm) return p64;
  std::vector<int> orders;
  for (int m : {64, 128, 256}) {
    const int o = (n + m - 1) / m * m;
    if (std::find(orders.begin(), orders.end(), o) == orders.end()) orders.push_back(o);
  }
  if (orders.size() == 1) return p64;
  int best = p64;
  double best_ms = 1e30;
  for (int o : orders) {
    (void)pick_cfg(d, o);
    double ms = 1e30;
    {
      std::lock_guard<std::mutex> lock(g_tune_mu);
      auto it = g_tune_ms.find(std::make_tuple(device, d, o));
      if (it != g_tune_ms.end()) ms = it->second;
    }
    if (verbose) fprintf(stderr, "[fm] order n=%d np=%d: %.3g ms per product\n", n, o, ms);
    if (ms < 0.95 * best_ms) {  // a larger order must be clearly faster
      best_ms = ms;
      best = o;
    }
  }
  return best;
}

GemmCfg Flow::pick_cfg(int d, int np) {
  const GemmCfg def = default_cfg(d, np);
  if (force_bm && d == dt) {
    for (const GemmCfg& c : gemm_configs(d))
      if (c.bm == force_bm && c.bk == force_bk && np % c.bm == 0 && np % c.bk == 0) {
        if (verbose) fprintf(stderr, "[fm] tile dt=%d np=%d -> bm=%d bk=%d (forced)\n", d, np, c.bm, c.bk);
        return c;
      }
    return def;
  }
  if (!autotune) return def;
  std::lock_guard<std::mutex> lock(g_tune_mu);
  tune_load(autotune_cache);
  auto key = std::make_tuple(device, d, np);
  auto it = g_tune.find(key);
  if (it != g_tune.end()) return it->second;
  std::vector<GemmCfg> cand;
  for (const GemmCfg& c : gemm_configs(d))
    if (np % c.bm == 0 && np % c.bk == 0) cand.push_back(c);
  if (cand.empty()) return def;
  // A batch of products of this order large enough that the largest
  // candidate tile fills the GPU too (>= 1024 tiles): a solve's fine phase
  // launches slices x problems products at once, and a batch that only the
  // small tiles can fill would always elect them.  That growth stops at
  // 512 MB of scratch; the base batch (up to 16 products, 128 MB of
  // operands) is kept even where it is larger, since a trial of one short
  // launch is too noisy to rank tiles.
  const size_t np2 = (size_t)np * np;
  const size_t esz = dt_size(d), asz = acc_size(d);
  int bm_max = 0;
  for (const GemmCfg& c : cand) bm_max = std::max(bm_max, c.bm);
  const size_t big_tiles = (size_t)(np / bm_max) * (np / bm_max);
  const size_t per_item = np2 * (2 * esz + asz + 8);
  const size_t base = std::max<size_t>(1, std::min<size_t>(16, ((size_t)1 << 27) / (np2 * 2)));
  const size_t fill = (1024 + big_tiles - 1) / big_tiles;
  const size_t cap = std::max<size_t>(base, ((size_t)512 << 20) / per_item);
  const int nb = (int)std::min<size_t>(std::max(base, fill), cap);
  void *A = nullptr, *B = nullptr, *C = nullptr, *Kacc = nullptr;
  double* Xs = nullptr;
  GItem* di = nullptr;
  int* dts = nullptr;
  hipStream_t st = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  GemmCfg best_c = def;
  double best = 1e30;
  bool ok = hipMalloc(&A, np2 * esz) == hipSuccess && hipMalloc(&B, np2 * esz) == hipSuccess &&
            hipMalloc(&C, np2 * esz * 2 * nb) == hipSuccess && hipMalloc(&Kacc, np2 * asz * nb) == hipSuccess &&
            hipMalloc((void**)&Xs, np2 * 8 * nb) == hipSuccess &&
            hipMalloc((void**)&di, 2 * nb * sizeof(GItem)) == hipSuccess &&
            hipMalloc((void**)&dts, (nb + 1) * sizeof(int)) == hipSuccess &&
            hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess && hipEventCreate(&e0) == hipSuccess &&
            hipEventCreate(&e1) == hipSuccess && fill_pattern(A, d, (int64_t)np2, st) == hipSuccess &&
            fill_pattern(B, d, (int64_t)np2, st) == hipSuccess &&
            fill_pattern(Xs, DT_F64, (int64_t)np2 * nb, st) == hipSuccess;
  if (ok) {
    std::vector<double> t(cand.size());
    for (size_t j = 0; j < cand.size(); ++j) {
      const GemmCfg& c = cand[j];
      t[j] = time_cfg(c, np, nb, A, B, C, Xs, Kacc, di, dts, st, e0, e1);
      if (verbose) fprintf(stderr, "[fm] autotune dt=%d np=%d bm=%d bk=%d: %.3f ms\n", d, np, c.bm, c.bk, t[j]);
      best = std::min(best, t[j]);
    }
    // Within 5 % of the fastest, the narrowest tile wins: it gives launches
    // of few products (a fine solve of one problem) more workgroups, where
    // the trial batch, which fills the GPU with any tile, cannot tell them
    // apart.
    if (best < 1e29) {
      int bm = 1 << 30;
      double chosen = best;
      for (size_t j = 0; j < cand.size(); ++j)
        if (t[j] <= 1.05 * best && cand[j].bm < bm) {
          bm = cand[j].bm;
          best_c = cand[j];
          chosen = t[j];
        }
      best = chosen;
    } else {
      best_c = def;
    }
  }
  if (st) (void)hipStreamSynchronize(st);
  if (A) (void)hipFree(A);
  if (B) (void)hipFree(B);
  if (C) (void)hipFree(C);
  if (Kacc) (void)hipFree(Kacc);
  if (Xs) (void)hipFree(Xs);
  if (di) (void)hipFree(di);
  if (dts) (void)hipFree(dts);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (st) (void)hipStreamDestroy(st);
  (void)hipGetLastError();
  g_tune[key] = best_c;
  g_tune_ms[key] = best < 1e29 ? best / nb : 1e30;
  tune_store(autotune_cache, device, d, np, best_c, g_tune_ms[key]);
  if (verbose) fprintf(stderr, "[fm] autotune dt=%d np=%d -> bm=%d bk=%d\n", d, np, best_c.bm, best_c.bk);
  return best_c;
}

// ---------------------------------------------------------------- create
static void parse_options(const char* opt, std::map<std::string, std::string>& kv) {
  if (!opt) return;
  std::string s(opt);
  size_t pos = 0;
  while (pos < s.size()) {
    size_t e = s.find(';', pos);
    if (e == std::string::npos) e = s.size();
    std::string item = s.substr(pos, e - pos);
    size_t eq = item.find('=');
    if (eq != std::string::npos) kv[item.substr(0, eq)] = item.substr(eq + 1);
    pos = e + 1;
  }
}

fm_status Flow::init(const fm_problem* p, int32_t nb, int32_t dtype, const char* options, hipStream_t st) {
  FM_HIP(hipGetDevice(&device));
  FM_TRY(noalloc_setup());
  dt = dtype;
  batch = nb;
  std::map<std::string, std::string> kv;
  parse_options(options, kv);
  if (kv.count("autotune")) autotune = kv["autotune"] != "0";
  if (kv.count("autotune_cache")) autotune_cache = kv["autotune_cache"];
  if (kv.count("timing")) timing = kv["timing"] != "0";
  if (kv.count("verbose")) verbose = kv["verbose"] != "0";
  if (kv.count("graph")) use_graph = kv["graph"] != "0";
  if (use_graph) FM_HIP(hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking));
  if (kv.count("coarse_f64")) coarse64 = kv["coarse_f64"] != "0" && dt != DT_F64;
  if (kv.count("split_b")) split_b = kv["split_b"] != "0";
  if (dt != DT_BF16 && dt != DT_F16) split_b = false;
  if (kv.count("pad")) {
    force_pad = atoi(kv["pad"].c_str());
    if (force_pad != 64 && force_pad != 128 && force_pad != 256) {
      set_error("option pad must be 64, 128 or 256");
      return FM_ERR_INVALID;
    }
  }
  if (kv.count("tile")) {
    bool known = sscanf(kv["tile"].c_str(), "%dx%d", &force_bm, &force_bk) == 2;
    bool found = false;
    if (known)
      for (const GemmCfg& c : gemm_configs(dt)) found = found || (c.bm == force_bm && c.bk == force_bk);
    if (!found) {
      set_error("option tile must read <bm>x<bk> and name a tile compiled for the flow's dtype");
      return FM_ERR_INVALID;
    }
  }
  FM_TRY(ring.init(size_t(256) << 20));
  inst.resize(nb);
  for (int i = 0; i < nb; ++i) {
    Inst& in = inst[i];
    in.kind = p[i].kind;
    in.n = (int)p[i].n;
    in.np = pick_order(dt, in.n);
    in.cfg = pick_cfg(dt, in.np);
    in.cfg64 = pick_cfg(DT_F64, in.np);
    const size_t np2 = (size_t)in.np * in.np;
    FM_HIP(hipMalloc((void**)&in.A64, np2 * sizeof(double)));
    FM_HIP(stage_pad_f64(in.A64, in.np, p[i].A, p[i].n, p[i].lda, st));
    if (in.kind != FM_FLOW_SQRT_STEADY) {
      const double shift = in.kind == FM_FLOW_INV_HOMOTOPY ? -1.0 : 0.0;
      if (split_b && two_products(in.kind)) {
        // hi plane (the operand) followed by the lo plane op(B - hi)
        FM_HIP(hipMalloc(&in.Bop, 2 * np2 * dt_size(dt)));
        FM_HIP(convert_split_f64(in.Bop, dt, in.A64, shift, in.n, in.np, st));
        in.Blo = (char*)in.Bop + np2 * dt_size(dt);
      } else {
        FM_HIP(hipMalloc(&in.Bop, np2 * dt_size(dt)));
        FM_HIP(convert_f64(in.Bop, dt, in.A64, shift, in.n, in.np, st));
      }
      if (coarse64) FM_TRY(ensure_b64(i, st));
    }
  }
  // a non-finite entry of A makes every iterate non-finite: refuse it here
  {
    constexpr int blk = 16;
    FM_TRY(ensure_part((size_t)nb * (blk + 1)));
    FM_TRY(ensure_hredu((size_t)nb));
    std::vector<DotItem> it;
    for (int i = 0; i < nb; ++i)
      it.push_back(DotItem{inst[i].A64, inst[i].A64, (int64_t)inst[i].np * inst[i].np, i, 1, nullptr});
    void* d = nullptr;
    FM_TRY(push(it.data(), it.size() * sizeof(DotItem), &d, st));
    FM_HIP(launch_dots((const DotItem*)d, nb, part, blk, part + (size_t)nb * blk, st));
    FM_HIP(hipMemcpyAsync(hredu, part + (size_t)nb * blk, nb * sizeof(double), hipMemcpyDeviceToHost, st));
    FM_HIP(hipStreamSynchronize(st));
    ring.reset();
    for (int i = 0; i < nb; ++i)
      if (hredu[i] != 0.0) {
        set_error("problem %d: A has %.0f non-finite entries", i, hredu[i]);
        return FM_ERR_NONFINITE;
      }
  }
  if (kv.count("coarse_model")) FM_TRY(load_model(kv["coarse_model"]));
  FM_HIP(hipStreamSynchronize(st));
  return FM_OK;
}

// ------------------------------------------------------------ GEMM launches
// Launch `items` (item_inst[j] = problem of item j) grouped by tile config.
fm_status Flow::gemm_groups(int epi, std::vector<GItem>& items, const std::vector<int>& item_inst, bool f64,
                            hipStream_t st) {
  if (items.empty()) return FM_OK;
  std::map<std::pair<int, int>, std::vector<int>> groups;  // (bm, bk) -> item indices
  for (size_t j = 0; j < items.size(); ++j) {
    const Inst& in = inst[item_inst[j]];
    const GemmCfg& c = f64 ? in.cfg64 : in.cfg;
    groups[{c.bm, c.bk}].push_back((int)j);
  }
  for (auto& g : groups) {
    GemmCfg cfg;
    cfg.dt = f64 ? DT_F64 : dt;
    cfg.bm = g.first.first;
    cfg.bk = g.first.second;
    std::vector<GItem> sub;
    std::vector<int> ts;
    sub.reserve(g.second.size());
    ts.reserve(g.second.size() + 1);
    int total = 0;
    ts.push_back(0);
    for (int j : g.second) {
      sub.push_back(items[j]);
      const int tpn = items[j].np / cfg.bm;
      total += tpn * tpn;
      ts.push_back(total);
    }
    void* d_items = nullptr;
    void* d_ts = nullptr;
    FM_TRY(push(sub.data(), sub.size() * sizeof(GItem), &d_items, st));
    FM_TRY(push(ts.data(), ts.size() * sizeof(int), &d_ts, st));
    const int grid = std::min(total, gemm_max_grid(cfg));
    FM_HIP(launch_gemm(cfg, epi, (const GItem*)d_items, (const int*)d_ts, (int)sub.size(), total, grid, nullptr, st));
  }
  return FM_OK;
}


// The stage-field product of item g (reading stage operand y, and P = B y
// for the two-product flows): k = s0 (a b) + s1 E + s3 I per flow kind.
static void field_item(GItem& g, const Inst& in, void* y, void* p, void* bop = nullptr) {
  if (!bop) bop = in.Bop;
  switch (in.kind) {
    case FM_FLOW_INV_HOMOTOPY:  // k = -Y (M Y)
      g.a = y;
      g.b = p;
      g.s[0] = -1.0;
      g.flags = F_E_NONE;
      break;
    case FM_FLOW_INV_STEADY:  // k = Y - Y (A Y)
      g.a = y;
      g.b = p;
      g.s[0] = -1.0;
      g.s[1] = 1.0;
      g.in0 = y;
      g.flags = 0;
      break;
    case FM_FLOW_SQRT_STEADY:  // k = A - Y Y
      g.a = y;
      g.b = y;
      g.s[0] = -1.0;
      g.s[1] = 1.0;
      g.in0 = in.A64;
      g.flags = F_E_F64;
      break;
    case FM_FLOW_EXP:  // k = A Y
      g.a = bop;
      g.b = y;
      g.s[0] = 1.0;
      g.flags = F_E_NONE;
      break;
    default:  // FM_FLOW_INV_LINEAR: k = I - A Y
      g.a = bop;
      g.b = y;
      g.s[0] = -1.0;
      g.s[3] = 1.0;
      g.flags = F_E_NONE;
  }
}

static GItem blank_item(const Inst& in, int i) {
  GItem it;
  memset(&it, 0, sizeof it);
  it.np = in.np;
  it.n = in.n;
  it.inst = i;
  return it;
}

// First product of a two-product stage field, out = s0 B Y, onto the item
// list.  With the lo plane of B (16-bit products, option split_b, stored
// right after the hi plane) the product runs over both planes in one
// launch, out = s0 (B_hi Y + B_lo Y) with one FP32 accumulation: B carries
// 2 x 8 (or 2 x 11) significant bits.
static void first_product(std::vector<GItem>& items, std::vector<int>& ii, const Inst& in, int i,
                          const void* b, bool split, const void* y, void* out, double s0, double s2 = 0.0) {
  GItem g = blank_item(in, i);
  g.a = b;
  g.b = y;
  g.out0 = out;
  g.flags = F_E_NONE | (split ? F_SPLIT_A : 0);
  g.s[0] = s0;
  g.s[2] = s2;  // identity term on the leading n x n diagonal
  items.push_back(g);
  ii.push_back(i);
}

// ------------------------------------------------- Crank-Nicolson operators
// For dX/dt = s A X + b I the Crank-Nicolson step (Sec. 2, Example 2) is
// X+ = Y ((I + s h/2 A) X + h b I), Y = (I - s h/2 A)^{-1}, which equals
// X + h (D X + b Y) with D = s Y A.  Y comes from the FP64 Newton-Schulz
// iteration Y <- Y (2I - M Y), M = I - s h/2 A, from Y = I: its residual
// I - M Y is squared by every step and starts at s h/2 A, so with
// rho = (h/2) ||A||_inf < 0.75 the iteration count k with rho^(2^k) < 1e-17
// reaches FP64 rounding.  Built once per (problem, h); kept with the flow.
fm_status Flow::ensure_cn(int i, double h, hipStream_t st, const Inst::CnOp** out) {
  Inst& in = inst[i];
  for (const auto& c : in.cn)
    if (c.h == h) {
      *out = &c;
      return FM_OK;
    }
  if (in.kind != FM_FLOW_EXP && in.kind != FM_FLOW_INV_LINEAR) {
    set_error("Crank-Nicolson steps are defined for the linear flows only");
    return FM_ERR_INVALID;
  }
  const double s = in.kind == FM_FLOW_EXP ? 1.0 : -1.0;
  const bool affine = in.kind == FM_FLOW_INV_LINEAR;
  const size_t np2 = (size_t)in.np * in.np;
  FM_HIP(hipStreamSynchronize(st));
  release_graphs();
  ring.reset();
  FM_TRY(ensure_hredu(1));
  double* tmp = nullptr;  // M, Y0, Y1, T and one scalar
  FM_HIP(hipMalloc((void**)&tmp, (4 * np2 + 1) * sizeof(double)));
  double *M = tmp, *Y[2] = {tmp + np2, tmp + 2 * np2}, *T = tmp + 3 * np2, *dn = tmp + 4 * np2;
  auto fail = [&](fm_status r) {
    (void)hipStreamSynchronize(st);
    (void)hipFree(tmp);
    return r;
  };
  if (in.norm_inf < 0) {
    hipError_t e = launch_norm_inf(in.A64, in.n, in.np, dn, st);
    if (e == hipSuccess) e = hipMemcpyAsync(hredu, dn, sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(hip_status(e, "Crank-Nicolson: ||A||_inf"));
    in.norm_inf = hredu[0];
  }
  const double rho = 0.5 * std::fabs(h) * in.norm_inf;
  if (!(rho < 0.75)) {
    set_error("Crank-Nicolson step h = %g: (h/2) ||A||_inf = %g, the Newton-Schulz inverse needs < 0.75", h, rho);
    return fail(FM_ERR_UNSUPPORTED);
  }
  int k = 0;
  for (double r = rho; r > 1e-17 && k < 64; r *= r) ++k;
  Inst::CnOp op{h, nullptr, nullptr, nullptr};
  auto product = [&](const void* a, const void* b, void* o, double s0, double s2) -> fm_status {
    std::vector<GItem> items(1);
    std::vector<int> ii(1, i);
    GItem& g = items[0];
    g = blank_item(in, i);
    g.a = a;
    g.b = b;
    g.out0 = o;
    g.s[0] = s0;
    g.s[2] = s2;
    g.flags = F_E_NONE | F_OUT0_F64;
    return gemm_groups(EPI_AFFINE, items, ii, true, st);
  };
  fm_status r = FM_OK;
  {
    hipError_t e = set_identity(Y[0], in.n, in.np, st);
    LinItem li{nullptr, nullptr, nullptr, Y[0], in.A64, M, nullptr, -0.5 * s * h, (int64_t)np2, 0, LIN_AXPY};
    if (e == hipSuccess) e = launch_lincomb(li, st);
    if (e != hipSuccess) return fail(hip_status(e, "Crank-Nicolson: M = I - s h/2 A"));
  }
  int cur = 0;
  for (int j = 0; j < k && r == FM_OK; ++j) {
    r = product(M, Y[cur], T, -1.0, 2.0);               // T = 2I - M Y
    if (r == FM_OK) r = product(Y[cur], T, Y[cur ^ 1], 1.0, 0.0);  // Y <- Y T
    cur ^= 1;
  }
  if (r != FM_OK) return fail(r);
  {
    hipError_t e = hipMalloc((void**)&op.D64, np2 * 8);
    if (e != hipSuccess) return fail(hip_status(e, "Crank-Nicolson: hipMalloc(D)"));
  }
  r = product(Y[cur], in.A64, op.D64, s, 0.0);          // D = s Y A
  if (r == FM_OK && affine) {
    hipError_t e = hipMalloc((void**)&op.E, np2 * 8);
    if (e == hipSuccess) e = copy_f64(op.E, Y[cur], (int64_t)np2, st);
    if (e != hipSuccess) r = hip_status(e, "Crank-Nicolson: E");
  }
  if (r == FM_OK) {
    if (dt == DT_F64) {
      op.Dop = op.D64;
    } else {
      hipError_t e = hipMalloc(&op.Dop, np2 * dt_size(dt));
      if (e == hipSuccess) e = convert_f64(op.Dop, dt, op.D64, 0.0, in.n, in.np, st);
      if (e != hipSuccess) r = hip_status(e, "Crank-Nicolson: D in the product dtype");
    }
  }
  if (r != FM_OK) {
    (void)hipStreamSynchronize(st);
    if (op.Dop && op.Dop != (void*)op.D64) (void)hipFree(op.Dop);
    if (op.D64) (void)hipFree(op.D64);
    if (op.E) (void)hipFree(op.E);
    return fail(r);
  }
  FM_HIP(hipStreamSynchronize(st));
  (void)hipFree(tmp);
  ring.reset();
  in.cn.push_back(op);
  *out = &in.cn.back();
  return FM_OK;
}

// The Crank-Nicolson step as an Euler-form item: k = D Y + b E, X+ = X + h k.
static void cn_item(GItem& g, const Inst::CnOp& op, const void* dop, void* y) {
  g.a = dop;
  g.b = y;
  g.s[0] = 1.0;
  if (op.E) {
    g.in0 = op.E;
    g.s[1] = 1.0;
    g.flags = F_E_F64;
  } else {
    g.flags = F_E_NONE;
  }
}

// ------------------------------------------------------- fine propagator
// `steps` classical RK4 steps of size slot.h on every slot, in place on
// slot.x; slot.ya must hold op(x) on entry.  One grouped launch per product:
// stage s reads Y from ya (s odd) or yb (s even) and writes the next stage
// operand to the other buffer, so after 4 stages Y is back in ya.
fm_status Flow::run_fine(const std::vector<FineSlot>& slots, int steps, int method, hipStream_t st,
                         float* x32_ws, bool plain) {
  if (slots.empty() || steps <= 0) return FM_OK;
  const bool timed = timing && !plain;
  // Build the 8 item lists once; they are identical for every step.
  // RK4: one unit = one step of 4 stages (operands ya -> yb -> ya -> yb -> ya).
  // Forward Euler: one unit = two steps (ya -> yb -> ya); an odd step count
  // ends with one more step on the first list (result operand in yb).
  const bool cn = method == FM_FINE_CN;
  const bool euler = method == FM_FINE_EULER || cn;  // one product per step, FP64 state
  const int nst = euler ? 2 : 4;
  // Crank-Nicolson operators of every slot (built before any list is staged)
  std::vector<const Inst::CnOp*> cnop(slots.size(), nullptr);
  if (cn)
    for (size_t k = 0; k < slots.size(); ++k) FM_TRY(ensure_cn(slots[k].inst, slots[k].h, st, &cnop[k]));
  const int units = euler ? steps / 2 : steps;
  const bool tail = euler && (steps % 2 == 1);
  const int fepi = euler ? EPI_EULER : EPI_RK4;
  // 16-bit products with RK4: the steps carry the state in FP32 (a stage
  // increment is an FP32 accumulation of 16-bit operands, so FP64 would hold
  // digits no step produces, at 20 more bytes per element and step); it is
  // narrowed from and widened back to the slot's FP64 state around the steps.
  const bool x32 = !euler && (dt == DT_BF16 || dt == DT_F16 || dt == DT_BF16X3);
  std::vector<float*> xs(slots.size(), nullptr);
  std::vector<CastItem> narrow, widen;
  if (x32) {
    size_t need = 0;
    for (const FineSlot& sl : slots) need += ((size_t)inst[sl.inst].np * inst[sl.inst].np + 63) / 64 * 64;
    if (!x32_ws) FM_TRY(ensure_x32(need));
    float* xbase = x32_ws ? x32_ws : x32buf;
    size_t off = 0;
    for (size_t k = 0; k < slots.size(); ++k) {
      const int64_t np2 = (int64_t)inst[slots[k].inst].np * inst[slots[k].inst].np;
      xs[k] = xbase + off;
      off += ((size_t)np2 + 63) / 64 * 64;
      narrow.push_back(CastItem{slots[k].x, xs[k], np2, 1, 0});
      widen.push_back(CastItem{xs[k], slots[k].x, np2, 0, 0});
    }
  }
  std::vector<GItem> l1[4], l2[4];
  std::vector<int> i1[4], i2[4];
  for (int s = 0; s < nst; ++s) {
    for (size_t k = 0; k < slots.size(); ++k) {
      const FineSlot& sl = slots[k];
      const Inst& in = inst[sl.inst];
      void* ycur = (s % 2 == 0) ? sl.ya : sl.yb;
      void* ynext = (s % 2 == 0) ? sl.yb : sl.ya;
      if (two_products(in.kind)) first_product(l1[s], i1[s], in, sl.inst, in.Bop, in.Blo != nullptr, ycur, sl.p, 1.0);
      GItem g = blank_item(in, sl.inst);
      if (cn) cn_item(g, *cnop[k], cnop[k]->Dop, ycur);
      else field_item(g, in, ycur, sl.p);
      g.out0 = ynext;
      g.out1 = euler ? (void*)sl.x : sl.kacc;
      g.x = x32 ? (double*)(void*)xs[k] : sl.x;
      if (x32) g.flags |= F_X_F32;
      g.stage = s + 1;
      g.s[2] = sl.h;
      l2[s].push_back(g);
      i2[s].push_back(sl.inst);
    }
  }
  // Push the lists once and replay the launches for every step.
  struct Launch {
    GemmCfg cfg;
    int epi;
    const GItem* items;
    const int* ts;
    int n;
    int total;
    int grid;
    double flops;  // algorithmic: 2 n^3 per item (unpadded order)
  };
  std::vector<Launch> seq;
  {
    // every list below is launched `steps` times: no ring reset in between
    size_t need = 0;
    for (int s = 0; s < nst; ++s)
      need += (l1[s].size() + l2[s].size()) * (sizeof(GItem) + sizeof(int)) + 8 * 512;
    need += 2 * (slots.size() * sizeof(CastItem) + 512);
    FM_TRY(reserve_ring(need, st));
  }
  const CastItem* d_widen = nullptr;
  if (x32) {
    void* dn = nullptr;
    void* dw = nullptr;
    FM_TRY(push(narrow.data(), narrow.size() * sizeof(CastItem), &dn, st));
    FM_TRY(push(widen.data(), widen.size() * sizeof(CastItem), &dw, st));
    FM_HIP(launch_cast((const CastItem*)dn, (int)narrow.size(), st));
    d_widen = (const CastItem*)dw;
  }
  auto widen_back = [&]() -> fm_status {
    if (x32) FM_HIP(launch_cast(d_widen, (int)widen.size(), st));
    return FM_OK;
  };
  auto prepare = [&](std::vector<GItem>& items, const std::vector<int>& ii, int epi) -> fm_status {
    if (items.empty()) return FM_OK;
    std::map<std::pair<int, int>, std::vector<int>> groups;
    for (size_t j = 0; j < items.size(); ++j) {
      const GemmCfg& c = inst[ii[j]].cfg;
      groups[{c.bm, c.bk}].push_back((int)j);
    }
    for (auto& g : groups) {
      Launch L;
      L.cfg.dt = dt;
      L.cfg.bm = g.first.first;
      L.cfg.bk = g.first.second;
      L.epi = epi;
      std::vector<GItem> sub;
      std::vector<int> ts(1, 0);
      int total = 0;
      L.flops = 0;
      for (int j : g.second) {
        sub.push_back(items[j]);
        const int tpn = items[j].np / L.cfg.bm;
        total += tpn * tpn;
        ts.push_back(total);
        L.flops += 2.0 * (double)items[j].n * items[j].n * items[j].n;
      }
      void* di = nullptr;
      void* dts = nullptr;
      FM_TRY(push(sub.data(), sub.size() * sizeof(GItem), &di, st));
      FM_TRY(push(ts.data(), ts.size() * sizeof(int), &dts, st));
      L.items = (const GItem*)di;
      L.ts = (const int*)dts;
      L.n = (int)sub.size();
      L.total = total;
      L.grid = std::min(total, gemm_max_grid(L.cfg));
      seq.push_back(L);
    }
    return FM_OK;
  };
  size_t first_stage_end = 0;  // launches of the first list (the Euler tail)
  for (int s = 0; s < nst; ++s) {
    FM_TRY(prepare(l1[s], i1[s], EPI_AFFINE));
    FM_TRY(prepare(l2[s], i2[s], fepi));
    if (s == 0) first_stage_end = seq.size();
  }
  int phase_ev = -1;
  if (timed) {
    phase_ev = (int)ev_used;
    hipEvent_t e0 = next_event(), e1 = next_event();
    if (!e0 || !e1) timing = false;
    else FM_HIP(hipEventRecord(e0, st));
  }
  auto launch_tail = [&]() -> fm_status {
    if (tail)
      for (size_t j = 0; j < first_stage_end; ++j) {
        const Launch& L = seq[j];
        FM_HIP(launch_gemm(L.cfg, L.epi, L.items, L.ts, L.n, L.total, L.grid, nullptr, st));
      }
    return FM_OK;
  };
  if (use_graph && cap_stream && units > 1 && !plain) {
    // capture the launches of one unit once, replay the graph for every unit
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    FM_HIP(hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (const Launch& L : seq) {
      e = launch_gemm(L.cfg, L.epi, L.items, L.ts, L.n, L.total, L.grid, nullptr, cap_stream);
      if (e != hipSuccess) break;
    }
    hipError_t e2 = hipStreamEndCapture(cap_stream, &g);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return hip_status(e, "fine-step graph capture");
    }
    pending_graph.push_back(g);
    pending_exec.push_back(ge);
    pending_stream.push_back(st);
    // with timing=1 each replay (one step: every GEMM launch of the unit) is
    // bracketed by events on the solve's stream
    double unit_flops = 0;
    for (const Launch& L : seq) unit_flops += L.flops;
    for (int u = 0; u < units; ++u) {
      int idx = -1;
      if (timed) {
        idx = (int)ev_used;
        hipEvent_t a = next_event(), b = next_event();
        if (a && b) FM_HIP(hipEventRecord(a, st));
        else idx = -1;
      }
      FM_HIP(hipGraphLaunch(ge, st));
      if (idx >= 0) {
        FM_HIP(hipEventRecord(ev[idx + 1], st));
        ev_pairs.push_back(Timed{idx, unit_flops, (int)seq.size()});
      }
    }
    FM_TRY(launch_tail());
    FM_TRY(widen_back());
    if (timed && phase_ev >= 0) {
      FM_HIP(hipEventRecord(ev[phase_ev + 1], st));
      phase_pairs.push_back(phase_ev);
    }
    return FM_OK;
  }
  for (int u = 0; u < units; ++u)
    for (const Launch& L : seq) {
      const bool rec = timed;
      int idx = -1;
      if (rec) {
        idx = (int)ev_used;
        hipEvent_t a = next_event(), b = next_event();
        if (a && b) FM_HIP(hipEventRecord(a, st));
        else idx = -1;
      }
      FM_HIP(launch_gemm(L.cfg, L.epi, L.items, L.ts, L.n, L.total, L.grid, nullptr, st));
      if (idx >= 0) {
        FM_HIP(hipEventRecord(ev[idx + 1], st));
        ev_pairs.push_back(Timed{idx, L.flops, 1});
      }
    }
  FM_TRY(launch_tail());
  FM_TRY(widen_back());
  if (timed && phase_ev >= 0) {
    FM_HIP(hipEventRecord(ev[phase_ev + 1], st));
    phase_pairs.push_back(phase_ev);
  }
  return FM_OK;
}

// ----------------------------------------------------- coarse propagator
// `steps` forward-Euler (or learned polynomial) substeps of size slot.h from
// slot.xin to slot.xout.  Operands ping-pong between y0 and y1.
fm_status Flow::run_coarse(const std::vector<CoarseSlot>& slots, int steps, hipStream_t st) {
  if (slots.empty() || steps <= 0) return FM_OK;
  // option coarse_f64: operands, products and B in FP64 (B64 is made at
  // flow creation)
  auto cbop = [&](const Inst& in) -> void* { return coarse64 ? (void*)in.B64 : in.Bop; };
  std::vector<const Inst::CnOp*> cnop(slots.size(), nullptr);
  for (size_t k = 0; k < slots.size(); ++k)
    if (slots[k].cn) FM_TRY(ensure_cn(slots[k].inst, slots[k].h, st, &cnop[k]));
  {
    std::vector<PrepItem> prep;
    for (const CoarseSlot& sl : slots) {
      const Inst& in = inst[sl.inst];
      PrepItem p;
      p.u = sl.xin;
      p.fo = nullptr;
      p.y = sl.y0;
      p.count = (int64_t)in.np * in.np;
      p.inst = sl.inst;
      p.pad_ = 0;
      prep.push_back(p);
    }
    void* d = nullptr;
    FM_TRY(push(prep.data(), prep.size() * sizeof(PrepItem), &d, st));
    FM_HIP(launch_prep((const PrepItem*)d, (int)prep.size(), coarse64 ? DT_F64 : dt, nullptr, st));
  }
  // B as two planes for the first product (not with FP64 coarse products)
  auto csplit = [&](const Inst& in) -> bool { return !coarse64 && in.Blo != nullptr; };
  for (int j = 0; j < steps; ++j) {
    std::vector<GItem> l1, l2, l3, l4;
    std::vector<int> i1, i2, i3, i4;
    for (size_t sk = 0; sk < slots.size(); ++sk) {
      const CoarseSlot& sl = slots[sk];
      const Inst& in = inst[sl.inst];
      void* yin = (j % 2 == 0) ? sl.y0 : sl.y1;
      void* yout = (j % 2 == 0) ? sl.y1 : sl.y0;
      const double* x = (j == 0) ? sl.xin : sl.xout;
      if (!sl.learned) {
        if (two_products(in.kind)) first_product(l1, i1, in, sl.inst, cbop(in), csplit(in), yin, sl.p, 1.0);
        GItem g = blank_item(in, sl.inst);
        if (sl.cn) cn_item(g, *cnop[sk], coarse64 ? (void*)cnop[sk]->D64 : cnop[sk]->Dop, yin);
        else field_item(g, in, yin, sl.p, cbop(in));
        g.out0 = yout;
        g.out1 = sl.xout;
        g.x = const_cast<double*>(x);
        g.s[2] = sl.h;
        l2.push_back(g);
        i2.push_back(sl.inst);
      } else {
        // K = h B Y ; K2 = K K ; P = c0 I + c1 K + c2 K2 + c3 K2 K (and K3) ;
        // X+ = Y P + c4 I + c5 K + c6 K2 + c7 K3
        const double* c = sl.coef + 8 * j;
        // K = h (A - I) Y (homotopy) or h (A Y - I) (X - X A X, centred on the root)
        first_product(l1, i1, in, sl.inst, cbop(in), csplit(in), yin, sl.k1, sl.h,
                      in.kind == FM_FLOW_INV_STEADY ? -sl.h : 0.0);
        GItem g2 = blank_item(in, sl.inst);
        g2.a = sl.k1;
        g2.b = sl.k1;
        g2.out0 = sl.k2;
        g2.flags = F_E_NONE;
        g2.s[0] = 1.0;
        l2.push_back(g2);
        i2.push_back(sl.inst);
        GItem g3 = blank_item(in, sl.inst);
        g3.a = sl.k2;
        g3.b = sl.k1;
        g3.out0 = sl.p;
        g3.out1 = sl.k3;
        g3.in0 = sl.k1;
        g3.in1 = sl.k2;
        for (int q = 0; q < 8; ++q) g3.s[q] = c[q];
        l3.push_back(g3);
        i3.push_back(sl.inst);
        GItem g4 = blank_item(in, sl.inst);
        g4.a = yin;
        g4.b = sl.p;
        g4.out0 = yout;
        g4.out1 = sl.xout;
        g4.in0 = sl.k1;
        g4.in1 = sl.k2;
        g4.in2 = sl.k3;
        for (int q = 0; q < 8; ++q) g4.s[q] = c[q];
        l4.push_back(g4);
        i4.push_back(sl.inst);
      }
    }
    // Euler items go to l1 (first product) / l2 (EPI_EULER); learned items
    // use l1..l4.  A call mixes both kinds only through separate lists.
    bool any_learned = false, any_euler = false;
    for (const CoarseSlot& sl : slots) (sl.learned ? any_learned : any_euler) = true;
    if (any_euler && any_learned) {
      set_error("internal: mixed coarse kinds in one call");
      return FM_ERR_INVALID;
    }
    if (!any_learned) {
      FM_TRY(gemm_groups(EPI_AFFINE, l1, i1, coarse64, st));
      FM_TRY(gemm_groups(EPI_EULER, l2, i2, coarse64, st));
    } else {
      FM_TRY(gemm_groups(EPI_AFFINE, l1, i1, coarse64, st));
      FM_TRY(gemm_groups(EPI_AFFINE, l2, i2, coarse64, st));
      FM_TRY(gemm_groups(EPI_POLYP, l3, i3, coarse64, st));
      FM_TRY(gemm_groups(EPI_POLYX, l4, i4, coarse64, st));
    }
  }
  return FM_OK;
}

// ------------------------------------------------- standalone propagators
fm_status Flow::fine_propagate(double t1, double t0, int steps, const double* const* xin, double* const* xout,
                               hipStream_t st, char* ws, size_t ws_cap) {
  // workspace: per problem x (FP64), ya, yb, p (op), kacc (acc); with a
  // caller's workspace also the FP32 states of the 16-bit products
  const bool ext = ws != nullptr;
  const bool x32 = dt == DT_BF16 || dt == DT_F16 || dt == DT_BF16X3;
  Arena own;
  Arena& ar = ext ? own : prop;
  std::vector<FineSlot> slots(batch);
  float* x32_ws = nullptr;
  for (int pass = 0; pass < 2; ++pass) {
    ar.measuring = (pass == 0);
    ar.used = 0;
    for (int i = 0; i < batch; ++i) {
      const size_t np2 = (size_t)inst[i].np * inst[i].np;
      FineSlot& s = slots[i];
      s.inst = i;
      s.x = (double*)ar.take(np2 * 8);
      s.ya = ar.take(np2 * dt_size(dt));
      s.yb = ar.take(np2 * dt_size(dt));
      s.p = ar.take(np2 * dt_size(dt));
      s.kacc = ar.take(np2 * acc_size(dt));
      s.h = (t1 - t0) / steps;
    }
    if (ext && x32) {
      size_t need = 0;
      for (int i = 0; i < batch; ++i) need += ((size_t)inst[i].np * inst[i].np + 63) / 64 * 64;
      x32_ws = (float*)ar.take(need * sizeof(float));
    }
    if (pass == 0) {
      if (!ext) {
        FM_TRY(prop.reserve(prop.used));
      } else {
        if (ar.used > ws_cap) {
          set_error("workspace of %zu bytes needed, the allocation-free scratch holds %zu", ar.used, ws_cap);
          return FM_ERR_INVALID;
        }
        own.base = ws;
        own.cap = ws_cap;
      }
    }
  }
  FM_HIP(hipStreamSynchronize(st));
  if (ext) {
    // earlier graphs stay alive (destroying them frees memory); only wait
    // for their streams before the item ring is reused
    for (auto q : pending_stream) FM_HIP(hipStreamSynchronize(q));
  } else {
    release_graphs();
  }
  ring.reset();
  {
    std::vector<double*> dst(batch);
    std::vector<const double*> src(batch);
    for (int i = 0; i < batch; ++i) {
      dst[i] = slots[i].x;
      src[i] = xin[i];
    }
    FM_TRY(pad_copy(dst, src, 1, st));
  }
  std::vector<PrepItem> prep;
  for (int i = 0; i < batch; ++i) {
    PrepItem p{slots[i].x, nullptr, slots[i].ya, (int64_t)inst[i].np * inst[i].np, i, 0};
    prep.push_back(p);
  }
  void* d = nullptr;
  FM_TRY(push(prep.data(), prep.size() * sizeof(PrepItem), &d, st));
  FM_HIP(launch_prep((const PrepItem*)d, (int)prep.size(), dt, nullptr, st));
  FM_TRY(run_fine(slots, steps, FM_FINE_RK4, st, x32_ws, ext));
  {
    std::vector<double*> dst(batch);
    std::vector<const double*> src(batch);
    for (int i = 0; i < batch; ++i) {
      dst[i] = xout[i];
      src[i] = slots[i].x;
    }
    FM_TRY(pad_copy(dst, src, 0, st));
  }
  return FM_OK;
}

fm_status Flow::coarse_propagate(double t1, double t0, int steps, int coarse, const double* const* xin,
                                 double* const* xout, hipStream_t st) {
  if (coarse == FM_COARSE_LEARNED && !model.loaded) {
    set_error("learned coarse step requested but no coarse_model is loaded");
    return FM_ERR_INVALID;
  }
  std::vector<CoarseSlot> slots(batch);
  std::vector<double> coefs((size_t)batch * 8 * steps);
  for (int pass = 0; pass < 2; ++pass) {
    prop.measuring = (pass == 0);
    prop.used = 0;
    for (int i = 0; i < batch; ++i) {
      const size_t np2 = (size_t)inst[i].np * inst[i].np;
      const size_t e = coarse_esz();
      CoarseSlot& s = slots[i];
      s.inst = i;
      double* xi = (double*)prop.take(np2 * 8);
      s.xin = xi;
      s.xout = xi;
      s.y0 = prop.take(np2 * e);
      s.y1 = prop.take(np2 * e);
      s.p = prop.take(np2 * e);
      s.k1 = prop.take(np2 * e);
      s.k2 = prop.take(np2 * e);
      s.k3 = prop.take(np2 * e);
      s.t0 = t0;
      s.h = (t1 - t0) / steps;
      s.learned = coarse == FM_COARSE_LEARNED;
      s.cn = coarse == FM_COARSE_CN;
      s.coef = coefs.data() + (size_t)i * 8 * steps;
    }
    if (pass == 0) FM_TRY(prop.reserve(prop.used));
  }
  if (coarse == FM_COARSE_LEARNED) {
    std::vector<CoefRow> rows;
    for (int i = 0; i < batch; ++i)
      for (int j = 0; j < steps; ++j) rows.push_back(CoefRow{i, t0 + j * slots[i].h, slots[i].h});
    FM_TRY(learned_table(rows, coefs.data(), st));
  }
  ring.reset();
  FM_HIP(hipStreamSynchronize(st));
  std::vector<double*> pd(batch), od(batch);
  std::vector<const double*> ps(batch), os(batch);
  for (int i = 0; i < batch; ++i) {
    pd[i] = slots[i].xout;
    ps[i] = xin[i];
    od[i] = xout[i];
    os[i] = slots[i].xout;
  }
  FM_TRY(pad_copy(pd, ps, 1, st));
  FM_TRY(run_coarse(slots, steps, st));
  FM_TRY(pad_copy(od, os, 0, st));
  return FM_OK;
}

// ------------------------------------------------------------ parareal
fm_status Flow::solve(const double* const* X0, double* const* Xout, const fm_params* prm, fm_stats* stats,
                      hipStream_t st) {
  if (prm[0].variant == FM_PARAREAL_MODIFIED) {
    fm_status worst = FM_OK;
    for (int i = 0; i < batch; ++i) {
      const fm_status r = solve_modified(i, X0 ? X0[i] : nullptr, Xout[i], prm, stats, st);
      if (r < 0 && r != FM_ERR_NONFINITE) return r;
      if (r < 0 && (worst >= 0 || r < worst)) worst = r;
      else if (worst == FM_OK && r != FM_OK) worst = r;
    }
    return worst;
  }
  // operand scratch that the coarse step shares (its own, and the slices'
  // buffers that the learned candidates borrow) holds FP64 with coarse_f64
  const size_t e = std::max<size_t>(dt_size(dt), coarse_esz()), ea = std::max<size_t>(acc_size(dt), coarse_esz());
  int Nmax = 0;
  for (int i = 0; i < batch; ++i) Nmax = std::max(Nmax, prm[i].N);
  bool any_learned = false;
  for (int i = 0; i < batch; ++i) any_learned |= prm[i].coarse == FM_COARSE_LEARNED;
  if (any_learned && !model.loaded) {
    set_error("coarse = FM_COARSE_LEARNED needs a loaded coarse_model");
    return FM_ERR_INVALID;
  }

  // ---- workspace layout
  struct IW {
    std::vector<double*> U, Fo, Go;
    std::vector<void*> ya, yb, p, kacc;
    double* gnew;
    void *cy0, *cy1, *cp, *ck1, *ck2, *ck3;
    // learned: coarse choice per slice and coefficient table
    std::vector<double> coef;    // N * coarse_steps * 8
    std::vector<int> use_learned;
    std::vector<void*> lk2, lk3;  // per-slice scratch of the candidate steps
    std::vector<double*> gl;      // per-slice learned candidate G_L(U^k_n)
  };
  std::vector<IW> w(batch);
  for (int pass = 0; pass < 2; ++pass) {
    work.measuring = (pass == 0);
    work.used = 0;
    for (int i = 0; i < batch; ++i) {
      const size_t np2 = (size_t)inst[i].np * inst[i].np;
      const int N = prm[i].N;
      IW& q = w[i];
      q.U.resize(N + 1);
      q.Fo.resize(N);
      q.Go.resize(N);
      q.ya.resize(N);
      q.yb.resize(N);
      q.p.resize(N);
      q.kacc.resize(N);
      for (int s = 0; s <= N; ++s) q.U[s] = (double*)work.take(np2 * 8);
      for (int s = 0; s < N; ++s) {
        q.Fo[s] = (double*)work.take(np2 * 8);
        q.Go[s] = (double*)work.take(np2 * 8);
        q.ya[s] = work.take(np2 * e);
        q.yb[s] = work.take(np2 * e);
        q.p[s] = work.take(np2 * e);
        q.kacc[s] = work.take(np2 * ea);
      }
      q.gnew = (double*)work.take(np2 * 8);
      q.cy0 = work.take(np2 * e);
      q.cy1 = work.take(np2 * e);
      q.cp = work.take(np2 * e);
      const bool lrn = prm[i].coarse == FM_COARSE_LEARNED;
      q.ck1 = lrn ? work.take(np2 * e) : nullptr;
      q.ck2 = lrn ? work.take(np2 * e) : nullptr;
      q.ck3 = lrn ? work.take(np2 * e) : nullptr;
      q.lk2.assign(N, nullptr);
      q.lk3.assign(N, nullptr);
      q.gl.assign(N, nullptr);
      if (lrn)
        for (int s = 0; s < N; ++s) {
          q.lk2[s] = work.take(np2 * e);
          q.lk3[s] = work.take(np2 * e);
          q.gl[s] = (double*)work.take(np2 * 8);
        }
    }
    if (pass == 0) FM_TRY(work.reserve(work.used));
  }
  FM_HIP(hipStreamSynchronize(st));
  const auto t_start = std::chrono::steady_clock::now();
  ring.reset();
  t_launches = 0;
  t_ms = t_flops = t_phase_ms = 0;
  ev_pairs.clear();
  phase_pairs.clear();
  ev_used = 0;

  // learned coefficient tables: one batched network evaluation for every
  // (problem, slice, substep); inputs (t, h, mu_1..4)
  {
    std::vector<CoefRow> rows;
    for (int i = 0; i < batch; ++i) {
      if (prm[i].coarse != FM_COARSE_LEARNED) continue;
      const int N = prm[i].N, C = prm[i].coarse_steps;
      w[i].use_learned.assign(N, 1);
      for (int s = 0; s < N; ++s) {
        const double ta = s * prm[i].T / N, tb = (s + 1) * prm[i].T / N;
        const double h = (tb - ta) / C;
        for (int j = 0; j < C; ++j) rows.push_back(CoefRow{i, ta + j * h, h});
      }
    }
    std::vector<double> table(rows.size() * 8);
    FM_TRY(learned_table(rows, table.data(), st));
    size_t r = 0;
    for (int i = 0; i < batch; ++i) {
      if (prm[i].coarse != FM_COARSE_LEARNED) continue;
      const size_t cnt = (size_t)prm[i].N * prm[i].coarse_steps;
      w[i].coef.assign(table.begin() + r * 8, table.begin() + (r + cnt) * 8);
      r += cnt;
    }
  }

  // ---- Step 0: U_0 = X0, U_{n+1} = G(U_n), G_old cached
  for (int i = 0; i < batch; ++i) {
    if (X0 && X0[i]) FM_HIP(copy_in(w[i].U[0], inst[i].np, X0[i], inst[i].n, st));
    else FM_HIP(set_identity(w[i].U[0], inst[i].n, inst[i].np, st));
  }
  // coarse propagator in use per problem: learned problems fall back to Euler
  // for good when an iteration produced a non-finite iterate
  std::vector<int> cmode(batch);
  for (int i = 0; i < batch; ++i) cmode[i] = prm[i].coarse;
  auto coarse_slot = [&](int i, int s, const double* xin, double* xout, bool learned) {
    CoarseSlot c;
    const int N = prm[i].N, C = prm[i].coarse_steps;
    const double ta = s * prm[i].T / N, tb = (s + 1) * prm[i].T / N;
    c.inst = i;
    c.xin = xin;
    c.xout = xout;
    c.y0 = w[i].cy0;
    c.y1 = w[i].cy1;
    c.p = w[i].cp;
    c.k1 = w[i].ck1;
    c.k2 = w[i].ck2;
    c.k3 = w[i].ck3;
    c.t0 = ta;
    c.h = (tb - ta) / C;
    c.learned = learned ? 1 : 0;
    c.coef = learned ? &w[i].coef[(size_t)s * C * 8] : nullptr;
    c.cn = prm[i].coarse == FM_COARSE_CN ? 1 : 0;
    return c;
  };
  // coarse steps of one sweep position, split by coarse kind and step count
  auto run_coarse_mixed = [&](std::vector<CoarseSlot>& all) -> fm_status {
    std::map<std::pair<int, int>, std::vector<CoarseSlot>> by;
    for (auto& c : all) by[{c.learned, prm[c.inst].coarse_steps}].push_back(c);
    for (auto& g : by) FM_TRY(run_coarse(g.second, g.first.second, st));
    return FM_OK;
  };
  const size_t npairs = (size_t)Nmax * batch;
  FM_TRY(ensure_hredu(npairs * 3));
  double* s0sums = nullptr;
  double* s0part = nullptr;
  if (any_learned) {
    for (int pass = 0; pass < 2; ++pass) {
      prop.measuring = (pass == 0);
      prop.used = 0;
      s0sums = (double*)prop.take(npairs * 8);
      s0part = (double*)prop.take(npairs * 16 * 8);
      if (pass == 0) {
        FM_HIP(hipStreamSynchronize(st));
        FM_TRY(prop.reserve(prop.used));
      }
    }
  }
  // number of non-finite entries of G_old of the listed (problem, slice) pairs
  auto nonfinite = [&](const std::vector<std::pair<int, int>>& is) -> fm_status {
    std::vector<DotItem> it;
    for (auto& q : is) {
      const int i = q.first, t = q.second;
      it.push_back(DotItem{w[i].Go[t], w[i].Go[t], (int64_t)inst[i].np * inst[i].np, t * batch + i, 1, nullptr});
    }
    if (it.empty()) return FM_OK;
    void* d = nullptr;
    FM_TRY(push(it.data(), it.size() * sizeof(DotItem), &d, st));
    FM_HIP(launch_dots((const DotItem*)d, (int)it.size(), s0part, 16, s0sums, st));
    FM_HIP(hipMemcpyAsync(hredu, s0sums, npairs * sizeof(double), hipMemcpyDeviceToHost, st));
    FM_HIP(hipStreamSynchronize(st));
    ring.reset();
    return FM_OK;
  };
  // Step 0 for the listed problems.  The learned step is kept unless it is not
  // finite: the first non-finite slice of a learned problem is redone with
  // Euler and the sweep continues from there (rare path, one check per slice).
  auto step0 = [&](const std::vector<int>& ids) -> fm_status {
    for (int s = 0; s < Nmax; ++s) {
      std::vector<CoarseSlot> cs;
      for (int i : ids)
        if (s < prm[i].N) cs.push_back(coarse_slot(i, s, w[i].U[s], w[i].Go[s], cmode[i] == FM_COARSE_LEARNED));
      FM_TRY(run_coarse_mixed(cs));
      for (int i : ids)
        if (s < prm[i].N) FM_HIP(copy_f64(w[i].U[s + 1], w[i].Go[s], (int64_t)inst[i].np * inst[i].np, st));
    }
    std::vector<std::pair<int, int>> all;
    for (int i : ids)
      if (cmode[i] == FM_COARSE_LEARNED)
        for (int t = 0; t < prm[i].N; ++t) all.push_back({i, t});
    if (all.empty()) return FM_OK;
    FM_TRY(nonfinite(all));
    for (int i : ids) {
      if (cmode[i] != FM_COARSE_LEARNED) continue;
      int first_bad = -1;
      for (int t = 0; t < prm[i].N && first_bad < 0; ++t)
        if (hredu[(size_t)t * batch + i] != 0.0) first_bad = t;
      if (first_bad < 0) continue;
      for (int t = first_bad; t < prm[i].N; ++t) {
        std::vector<CoarseSlot> one(1, coarse_slot(i, t, w[i].U[t], w[i].Go[t], true));
        FM_TRY(run_coarse(one, prm[i].coarse_steps, st));
        FM_TRY(nonfinite({{i, t}}));
        w[i].use_learned[t] = hredu[(size_t)t * batch + i] == 0.0;
        if (!w[i].use_learned[t]) {
          one[0] = coarse_slot(i, t, w[i].U[t], w[i].Go[t], false);
          FM_TRY(run_coarse(one, prm[i].coarse_steps, st));
        }
        FM_HIP(copy_f64(w[i].U[t + 1], w[i].Go[t], (int64_t)inst[i].np * inst[i].np, st));
      }
    }
    return FM_OK;
  };
  {
    std::vector<int> ids(batch);
    for (int i = 0; i < batch; ++i) ids[i] = i;
    FM_TRY(step0(ids));
  }

  // ---- iterations (each problem counts its own: kk[i] iterations since its
  // last Step 0, which is also the number of leading slices that equal the
  // serial fine solution; total[i] iterations including those before a
  // restart, the count that max_iter bounds and the stats report)
  std::vector<int> live(batch, 0), kk(batch, 0), total(batch, 0), restarts(batch, 0);
  std::vector<fm_status> ist(batch, FM_OK);
  std::vector<double> lastinc(batch, 0.0);
  std::vector<std::vector<double>> hist(batch);
  std::vector<int> learned_count(batch, 0);
  for (int i = 0; i < batch; ++i) live[i] = prm[i].max_iter > 0 && prm[i].N > 0;
  int nblk = 1;
  for (int i = 0; i < batch; ++i) {
    int64_t np2 = (int64_t)inst[i].np * inst[i].np;
    nblk = std::max<int>(nblk, (int)std::min<int64_t>(256, (np2 + 4095) / 4096));
  }
  // partials: the correction's (3 per block and pair) or the learned
  // candidates' defect dots (two per pair, 16 blocks each), then the reduced
  // triples and the candidate defects
  const int cand_blk = 16;
  const size_t part_n = npairs * (size_t)std::max(3 * nblk, 2 * cand_blk);
  FM_TRY(ensure_part(part_n + npairs * 3 + npairs * 2));
  double* d_red = part + part_n;
  double* d_cand = d_red + npairs * 3;  // defects of the learned / Euler candidates

  for (int round = 0;; ++round) {
    bool any = false;
    int kmin = Nmax;
    for (int i = 0; i < batch; ++i)
      if (live[i]) {
        any = true;
        kmin = std::min(kmin, kk[i]);
      }
    if (!any) break;
    FM_HIP(hipStreamSynchronize(st));
    release_graphs();
    ring.reset();
    // fine solves of all live (problem, slice >= k) pairs in one launch per product;
    // slices below k are already the serial fine solution
    std::vector<FineSlot> fs;
    std::vector<PrepItem> prep;
    for (int s = kmin; s < Nmax; ++s)
      for (int i = 0; i < batch; ++i) {
        if (!live[i] || s >= prm[i].N || s < kk[i]) continue;
        const int N = prm[i].N;
        const double ta = s * prm[i].T / N, tb = (s + 1) * prm[i].T / N;
        FineSlot f{i, w[i].Fo[s], w[i].ya[s], w[i].yb[s], w[i].p[s], w[i].kacc[s], (tb - ta) / prm[i].fine_steps};
        fs.push_back(f);
        prep.push_back(PrepItem{w[i].U[s], w[i].Fo[s], w[i].ya[s], (int64_t)inst[i].np * inst[i].np, i, 0});
      }
    {
      void* d = nullptr;
      FM_TRY(push(prep.data(), prep.size() * sizeof(PrepItem), &d, st));
      FM_HIP(launch_prep((const PrepItem*)d, (int)prep.size(), dt, nullptr, st));
    }
    {
      std::map<std::pair<int, int>, std::vector<FineSlot>> by;  // (steps, scheme)
      for (auto& f : fs) by[{prm[f.inst].fine_steps, prm[f.inst].fine_method}].push_back(f);
      for (auto& g : by) FM_TRY(run_fine(g.second, g.first.first, g.first.second, st));
    }
    // learned coarse: choose per slice between the learned and the Euler step
    // by their defect against F(U^k_n) (the Euler fallback), and set G_old to
    // the chosen step at U^k_n.  Candidates of all slices run in parallel on
    // the slices' own scratch.
    {
      std::vector<CoarseSlot> ce, cl;
      std::vector<std::pair<int, int>> cl_is;  // (problem, slice) of each candidate
      std::vector<DotItem> di;
      for (int s = kmin; s < Nmax; ++s)
        for (int i = 0; i < batch; ++i) {
          if (!live[i] || s >= prm[i].N || s < kk[i] || cmode[i] != FM_COARSE_LEARNED) continue;
          CoarseSlot c = coarse_slot(i, s, w[i].U[s], w[i].Go[s], false);
          c.y0 = w[i].ya[s];
          c.y1 = w[i].yb[s];
          c.p = w[i].p[s];
          c.k1 = w[i].kacc[s];
          c.k2 = w[i].lk2[s];
          c.k3 = w[i].lk3[s];
          ce.push_back(c);
          c.learned = 1;
          c.xout = w[i].gl[s];
          c.coef = &w[i].coef[(size_t)s * prm[i].coarse_steps * 8];
          cl.push_back(c);
          cl_is.push_back({i, s});
          const int64_t cnt = (int64_t)inst[i].np * inst[i].np;
          di.push_back(DotItem{w[i].gl[s], w[i].gl[s], cnt, (int)(s * batch + i), 0, w[i].Fo[s]});
          di.push_back(DotItem{w[i].Go[s], w[i].Go[s], cnt, (int)(npairs + s * batch + i), 0, w[i].Fo[s]});
        }
      if (!ce.empty()) {
        FM_TRY(run_coarse_mixed(ce));
        FM_TRY(run_coarse_mixed(cl));
        void* d = nullptr;
        if (di.size() * cand_blk > part_n || di.size() > 2 * npairs) {
          set_error("internal: %zu candidate dots exceed the partials buffer", di.size());
          return FM_ERR_INVALID;
        }
        FM_TRY(push(di.data(), di.size() * sizeof(DotItem), &d, st));
        FM_HIP(launch_dots((const DotItem*)d, (int)di.size(), part, cand_blk, d_cand, st));
        FM_HIP(hipMemcpyAsync(hredu, d_cand, npairs * 2 * sizeof(double), hipMemcpyDeviceToHost, st));
        FM_HIP(hipStreamSynchronize(st));
        ring.reset();
        for (const auto& q : cl_is) {
          const int i = q.first, s2 = q.second;
          const double dl = hredu[(size_t)s2 * batch + i], de = hredu[npairs + (size_t)s2 * batch + i];
          w[i].use_learned[s2] = (std::isfinite(dl) && dl <= de) ? 1 : 0;
          if (w[i].use_learned[s2])
            FM_HIP(copy_f64(w[i].Go[s2], w[i].gl[s2], (int64_t)inst[i].np * inst[i].np, st));
        }
        for (int i = 0; i < batch; ++i)
          if (live[i] && cmode[i] == FM_COARSE_LEARNED) {
            int c2 = 0;
            for (int s2 = kk[i]; s2 < prm[i].N; ++s2) c2 += w[i].use_learned[s2];
            learned_count[i] = c2;
          }
      }
    }
    // sequential correction sweep: U^{k+1}_{n+1} = G(U^{k+1}_n) + F(U^k_n) - G(U^k_n);
    // at n = k both coarse values are of the exact slice, so U^{k+1}_{k+1} = F(U^k_k)
    for (int s = kmin; s < Nmax; ++s) {
      std::vector<CoarseSlot> cs;
      std::vector<CorrItem> ci;
      for (int i = 0; i < batch; ++i) {
        if (!live[i] || s >= prm[i].N || s < kk[i]) continue;
        if (s > kk[i])
          cs.push_back(coarse_slot(i, s, w[i].U[s], w[i].gnew,
                                   cmode[i] == FM_COARSE_LEARNED && w[i].use_learned[s]));
        CorrItem c;
        c.u = w[i].U[s + 1];
        c.f = w[i].Fo[s];
        c.gnew = (s > kk[i]) ? w[i].gnew : w[i].Go[s];
        c.gold = w[i].Go[s];
        c.count = (int64_t)inst[i].np * inst[i].np;
        c.inst = i;
        c.slot = s * batch + i;
        ci.push_back(c);
      }
      FM_TRY(run_coarse_mixed(cs));
      if (!ci.empty()) {
        void* d = nullptr;
        FM_TRY(push(ci.data(), ci.size() * sizeof(CorrItem), &d, st));
        FM_HIP(launch_correction((const CorrItem*)d, (int)ci.size(), part, nblk, nullptr, st));
      }
    }
    FM_HIP(launch_reduce_pairs(part, (int)npairs, nblk, d_red, st));
    FM_HIP(hipMemcpyAsync(hredu, d_red, npairs * 3 * sizeof(double), hipMemcpyDeviceToHost, st));
    FM_HIP(hipStreamSynchronize(st));
    if (timing) FM_TRY(collect_timing());
    std::vector<int> restart;
    for (int i = 0; i < batch; ++i) {
      if (!live[i]) continue;
      double inc = 0.0;
      bool bad = false;
      for (int s = kk[i]; s < prm[i].N; ++s) {
        const double* r = hredu + ((size_t)s * batch + i) * 3;
        const double d = r[0] > 0 ? std::sqrt(r[0]) : 0.0;
        const double u = r[1] > 0 ? std::sqrt(r[1]) : 0.0;
        const double q = u > 0 ? d / u : d;
        if (!(q == q)) bad = true;
        inc = std::max(inc, q);
        if (r[2] != 0.0) bad = true;
      }
      kk[i]++;
      total[i]++;
      lastinc[i] = inc;
      hist[i].push_back(inc);
      if (bad) {
        if (cmode[i] == FM_COARSE_LEARNED && total[i] < prm[i].max_iter) {
          // the learned step diverged in a sweep: restart from Step 0 with
          // Euler; the iterations so far still count against max_iter
          cmode[i] = FM_COARSE_EULER;
          learned_count[i] = 0;
          restarts[i]++;
          kk[i] = 0;
          restart.push_back(i);
        } else {
          ist[i] = FM_ERR_NONFINITE;
          live[i] = 0;
        }
        continue;
      }
      if (inc <= prm[i].tol || kk[i] >= prm[i].N) {
        live[i] = 0;
      } else if (total[i] >= prm[i].max_iter) {
        live[i] = 0;
        ist[i] = FM_WARN_NOT_CONVERGED;
      }
    }
    if (!restart.empty()) FM_TRY(step0(restart));
    if (verbose) {
      double worst = 0.0;
      int nlive = 0;
      for (int i = 0; i < batch; ++i) {
        if (live[i] || total[i] > 0) worst = std::max(worst, lastinc[i]);
        nlive += live[i];
      }
      const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
      fprintf(stderr, "[fm] round %d: max increment %.3e, %d problems still iterating, %.2f s\n", round + 1,
              worst, nlive, sec);
      fflush(stderr);
    }
  }
  std::vector<int> iters = total;

  // ---- result, residual and refinement
  std::vector<double*> X(batch);
  std::vector<int> which;
  for (int i = 0; i < batch; ++i) {
    X[i] = w[i].U[prm[i].N];
    if (ist[i] != FM_ERR_NONFINITE && inst[i].kind != FM_FLOW_EXP) which.push_back(i);
  }
  if (stats) {
    for (int i = 0; i < batch; ++i) {
      memset(&stats[i], 0, sizeof(fm_stats));
      stats[i].iters = iters[i];
      stats[i].increment = lastinc[i];
      for (size_t j = 0; j < hist[i].size() && j < 64; ++j) stats[i].hist[j] = hist[i][j];
      stats[i].residual_before = stats[i].residual = NAN;
      stats[i].learned_slices = learned_count[i];
      stats[i].learned_restarts = restarts[i];
      stats[i].fine_launches = (int32_t)t_launches;
      stats[i].fine_ms = t_ms;
      stats[i].fine_flops = t_flops;
      stats[i].fine_phase_ms = t_phase_ms;
    }
  }
  FM_TRY(refine(which, X, prm, stats, st));
  fm_status worst = FM_OK;
  for (int i = 0; i < batch; ++i) {
    if (ist[i] != FM_ERR_NONFINITE) FM_HIP(copy_out(Xout[i], inst[i].n, X[i], inst[i].np, st));
    if (stats) stats[i].status = ist[i];
    if (ist[i] < 0 && (worst >= 0 || ist[i] < worst)) worst = ist[i];
    else if (worst == FM_OK && ist[i] != FM_OK) worst = ist[i];
  }
  FM_HIP(hipStreamSynchronize(st));
  if (worst == FM_ERR_NONFINITE) set_error("an iterate became non-finite (A(t) singular or the flow diverged)");
  return worst;
}

// ------------------------------------------------------ double angle
// Alg. 5 (Sec. 3): C <- 2 C^2 - I, m times, in FP64, for problem 0's order
// (C: device n x n, leading dimension n, overwritten).  One FP64 product
// per step with the affine epilogue 2 (C C) - I; operands ping-pong between
// two zero-padded buffers.
fm_status Flow::double_angle(double* C, int m, hipStream_t st) {
  const Inst& in = inst[0];
  const size_t np2 = (size_t)in.np * in.np;
  double* P[2] = {nullptr, nullptr};
  for (int pass = 0; pass < 2; ++pass) {
    prop.measuring = (pass == 0);
    prop.used = 0;
    P[0] = (double*)prop.take(np2 * 8);
    P[1] = (double*)prop.take(np2 * 8);
    if (pass == 0) FM_TRY(prop.reserve(prop.used));
  }
  FM_HIP(hipStreamSynchronize(st));
  release_graphs();
  ring.reset();
  FM_HIP(copy_in(P[0], in.np, C, in.n, st));
  for (int j = 0; j < m; ++j) {
    std::vector<GItem> items(1);
    std::vector<int> ii(1, 0);
    GItem& g = items[0];
    g = blank_item(in, 0);
    g.a = P[j & 1];
    g.b = P[j & 1];
    g.out0 = P[(j & 1) ^ 1];
    g.s[0] = 2.0;
    g.s[2] = -1.0;
    g.flags = F_E_NONE | F_OUT0_F64;
    FM_TRY(gemm_groups(EPI_AFFINE, items, ii, true, st));
  }
  FM_HIP(copy_out(C, in.n, P[m & 1], in.np, st));
  FM_HIP(hipStreamSynchronize(st));
  return FM_OK;
}

// -------------------------------------------------- modified parareal
// Alg. 3 / Alg. 4 (Sec. 3) for problem i of a linear flow.  Layout: the
// iterates of two consecutive iterations (Ua, Ub), the basis Q and its fine
// images FQ (FP64, at most `cap` blocks, device pointer tables for the
// combination kernel), one FP64 work block per candidate, and the operand
// buffers of one fine propagation per possible new block and of one coarse
// propagation.  Every step is a grouped GEMM launch or an FP64 stream kernel;
// the host reads back two norms per basis candidate (accept / drop) and the
// slice increments once per iteration.
fm_status Flow::solve_modified(int i, const double* X0, double* Xout, const fm_params* prm, fm_stats* stats,
                               hipStream_t st) {
  const fm_params& p = prm[i];
  const Inst& in = inst[i];
  const int N = p.N;
  const int K = std::min(p.max_iter, N);
  const bool affine = in.kind == FM_FLOW_INV_LINEAR;
  const size_t np2 = (size_t)in.np * in.np;
  const int64_t cnt = (int64_t)np2;
  // operand scratch that the coarse step shares (its own, and the slices'
  // buffers that the learned candidates borrow) holds FP64 with coarse_f64
  const size_t e = std::max<size_t>(dt_size(dt), coarse_esz()), ea = std::max<size_t>(acc_size(dt), coarse_esz());
  const int64_t cap64 = std::min<int64_t>((int64_t)(K + 1) * (N + 1), (int64_t)in.n * in.n);
  const int cap = (int)std::max<int64_t>(1, cap64);
  constexpr int NB = 32;  // dot partial blocks
  constexpr double DROP = 1e-7;  // remainders below: rounding-dominated directions
  std::vector<double*> Ua(N + 1), Ub(N + 1), Q(cap), FQ(cap);
  std::vector<void*> fya(N + 1), fyb(N + 1), fp(N + 1), fk(N + 1);
  double *W = nullptr, *R = nullptr, *GR = nullptr, *F0 = nullptr, *G0 = nullptr, *C = nullptr;
  double *alpha = nullptr, *nrm = nullptr, *part_d = nullptr, *incs = nullptr;
  double **qptr = nullptr, **fqptr = nullptr;
  void *cy0 = nullptr, *cy1 = nullptr, *cp = nullptr;
  for (int pass = 0; pass < 2; ++pass) {
    work.measuring = (pass == 0);
    work.used = 0;
    for (int n = 0; n <= N; ++n) {
      Ua[n] = (double*)work.take(np2 * 8);
      Ub[n] = (double*)work.take(np2 * 8);
      fya[n] = work.take(np2 * e);
      fyb[n] = work.take(np2 * e);
      fp[n] = work.take(np2 * e);
      fk[n] = work.take(np2 * ea);
    }
    for (int j = 0; j < cap; ++j) {
      Q[j] = (double*)work.take(np2 * 8);
      FQ[j] = (double*)work.take(np2 * 8);
    }
    W = (double*)work.take(np2 * 8);
    R = (double*)work.take(np2 * 8);
    GR = (double*)work.take(np2 * 8);
    F0 = affine ? (double*)work.take(np2 * 8) : nullptr;
    G0 = affine ? (double*)work.take(np2 * 8) : nullptr;
    C = affine ? (double*)work.take(np2 * 8) : nullptr;
    cy0 = work.take(np2 * e);
    cy1 = work.take(np2 * e);
    cp = work.take(np2 * e);
    alpha = (double*)work.take(sizeof(double) * (cap + 2));
    nrm = (double*)work.take(sizeof(double) * 4);
    part_d = (double*)work.take(sizeof(double) * (size_t)(cap + 2 * (N + 1)) * NB);
    incs = (double*)work.take(sizeof(double) * 2 * (N + 1));
    qptr = (double**)work.take(sizeof(double*) * cap);
    fqptr = (double**)work.take(sizeof(double*) * cap);
    if (pass == 0) FM_TRY(work.reserve(work.used));
  }
  FM_HIP(hipStreamSynchronize(st));
  release_graphs();
  ring.reset();
  FM_HIP(hipMemcpyAsync(qptr, Q.data(), sizeof(double*) * cap, hipMemcpyHostToDevice, st));
  FM_HIP(hipMemcpyAsync(fqptr, FQ.data(), sizeof(double*) * cap, hipMemcpyHostToDevice, st));
  const double H = p.T / N;
  auto coarse = [&](const double* xin, double* xout) -> fm_status {
    std::vector<CoarseSlot> cs(1);
    cs[0] = CoarseSlot{i, xin, xout, cy0, cy1, cp, nullptr, nullptr, nullptr, 0.0, H / p.coarse_steps, 0, nullptr};
    return run_coarse(cs, p.coarse_steps, st);
  };
  // fine images of blocks src[j] into dst[j], all in one grouped propagation
  auto fine = [&](const std::vector<const double*>& src, const std::vector<double*>& dst) -> fm_status {
    if (src.empty()) return FM_OK;
    std::vector<FineSlot> fs;
    std::vector<PrepItem> prep;
    for (size_t j = 0; j < src.size(); ++j) {
      FM_HIP(copy_f64(dst[j], src[j], cnt, st));
      fs.push_back(FineSlot{i, dst[j], fya[j], fyb[j], fp[j], fk[j], H / p.fine_steps});
      prep.push_back(PrepItem{dst[j], nullptr, fya[j], cnt, i, 0});
    }
    void* d = nullptr;
    FM_TRY(push(prep.data(), prep.size() * sizeof(PrepItem), &d, st));
    FM_HIP(launch_prep((const PrepItem*)d, (int)prep.size(), dt, nullptr, st));
    return run_fine(fs, p.fine_steps, p.fine_method, st);
  };
  // <q_j, x> for j < s into alpha[0..s)
  auto project = [&](const double* x, int s) -> fm_status {
    if (s == 0) return FM_OK;
    std::vector<DotItem> it;
    for (int j = 0; j < s; ++j) it.push_back(DotItem{Q[j], x, cnt, j, 0, nullptr});
    void* d = nullptr;
    FM_TRY(push(it.data(), it.size() * sizeof(DotItem), &d, st));
    FM_HIP(launch_dots((const DotItem*)d, s, part_d, NB, alpha, st));
    return FM_OK;
  };
  auto lin = [&](int mode, const double* z, double* out1, double* out2, const double* c, double scale,
                 int s) -> fm_status {
    LinItem it{(const double* const*)qptr, (const double* const*)fqptr, alpha, z, c, out1, out2, scale, cnt, s, mode};
    FM_HIP(launch_lincomb(it, st));
    return FM_OK;
  };
  auto norms2 = [&](const double* a, const double* b, double* h2) -> fm_status {  // ||a||^2, ||b||^2 to host
    DotItem it[2] = {DotItem{a, a, cnt, 0, 0, nullptr}, DotItem{b, b, cnt, 1, 0, nullptr}};
    void* d = nullptr;
    FM_TRY(push(it, sizeof it, &d, st));
    FM_HIP(launch_dots((const DotItem*)d, 2, part_d, NB, nrm, st));
    FM_HIP(hipMemcpyAsync(h2, nrm, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    FM_HIP(hipStreamSynchronize(st));
    return FM_OK;
  };

  // ---- U_0 and Step 0 (coarse sweep); Step -1 for the affine flow
  std::vector<double*>* U = &Ua;
  std::vector<double*>* V = &Ub;
  if (X0) FM_HIP(copy_in((*U)[0], in.np, X0, in.n, st));
  else FM_HIP(set_identity((*U)[0], in.n, in.np, st));
  FM_HIP(copy_f64((*V)[0], (*U)[0], cnt, st));
  for (int n = 0; n < N; ++n) FM_TRY(coarse((*U)[n], (*U)[n + 1]));
  if (affine) {
    FM_HIP(hipMemsetAsync(W, 0, np2 * 8, st));
    FM_TRY(fine({W}, {F0}));
    FM_TRY(coarse(W, G0));
    FM_TRY(lin(LIN_AXPY, F0, C, nullptr, G0, -1.0, 0));  // C = F(0) - G(0)
  }
  int s = 0, k = 0;
  double inc = NAN;
  std::vector<double> hist;
  fm_status status = FM_OK;
  while (k < K) {
    // ---- enlarge the basis with U^k_0 .. U^k_N (CGS, applied twice)
    const int s0 = s;
    for (int c = 0; c <= N; ++c) {
      if (s == cap) break;
      const double* z = (*U)[c];
      FM_TRY(project(z, s));
      FM_TRY(lin(LIN_ORTH, z, W, nullptr, nullptr, 0.0, s));
      FM_TRY(project(W, s));
      FM_TRY(lin(LIN_ORTH, W, W, nullptr, nullptr, 0.0, s));
      double h2[2];
      FM_TRY(norms2(z, W, h2));
      if (!std::isfinite(h2[0]) || !std::isfinite(h2[1])) {
        status = FM_ERR_NONFINITE;
        break;
      }
      const double nz = std::sqrt(h2[0]), rw = std::sqrt(h2[1]);
      if (rw > DROP * nz && rw > 0) {
        FM_TRY(lin(LIN_SCALE, W, Q[s], nullptr, nullptr, 1.0 / rw, 0));
        ++s;
      }
    }
    if (status != FM_OK) break;
    // ---- fine images of the new blocks (in parallel); affine: minus F(0)
    {
      std::vector<const double*> src;
      std::vector<double*> dst;
      for (int j = s0; j < s; ++j) {
        src.push_back(Q[j]);
        dst.push_back(FQ[j]);
      }
      FM_TRY(fine(src, dst));
      if (affine)
        for (int j = s0; j < s; ++j) FM_TRY(lin(LIN_AXPY, FQ[j], FQ[j], nullptr, F0, -1.0, 0));
    }
    // ---- sweep: U^{k+1}_{n+1} = sum alpha FQ [+ F(0) - G(0)] + G(U - sum alpha Q)
    for (int n = 0; n < N; ++n) {
      FM_TRY(project((*V)[n], s));
      FM_TRY(lin(LIN_SWEEP, (*V)[n], R, (*V)[n + 1], C, 0.0, s));
      FM_TRY(coarse(R, GR));
      FM_TRY(lin(LIN_AXPY, (*V)[n + 1], (*V)[n + 1], nullptr, GR, 1.0, 0));
    }
    // ---- increment of the iteration
    {
      std::vector<DotItem> it;
      for (int n = 1; n <= N; ++n) {
        it.push_back(DotItem{(*V)[n], (*V)[n], cnt, 2 * (n - 1), 0, (*U)[n]});
        it.push_back(DotItem{(*V)[n], (*V)[n], cnt, 2 * (n - 1) + 1, 0, nullptr});
      }
      void* d = nullptr;
      FM_TRY(push(it.data(), it.size() * sizeof(DotItem), &d, st));
      FM_HIP(launch_dots((const DotItem*)d, (int)it.size(), part_d, NB, incs, st));
      std::vector<double> h(2 * N);
      FM_HIP(hipMemcpyAsync(h.data(), incs, 2 * N * sizeof(double), hipMemcpyDeviceToHost, st));
      FM_HIP(hipStreamSynchronize(st));
      inc = 0.0;
      bool finite = true;
      for (int n = 0; n < N; ++n) {
        finite &= std::isfinite(h[2 * n]) && std::isfinite(h[2 * n + 1]);
        const double d2 = std::sqrt(h[2 * n]), s2 = std::sqrt(h[2 * n + 1]);
        inc = std::max(inc, s2 > 0 ? d2 / s2 : d2);
      }
      if (!finite) {
        status = FM_ERR_NONFINITE;
        break;
      }
    }
    std::swap(U, V);
    ring.reset();  // all pushed lists were consumed (the last host read synchronised)
    ++k;
    hist.push_back(inc);
    if (verbose) fprintf(stderr, "[fm] modified parareal problem %d iteration %d: basis %d, increment %.3e\n", i, k, s, inc);
    if (inc <= p.tol) break;
  }
  if (status == FM_OK && K > 0 && k == K && K < N && !(inc <= p.tol)) status = FM_WARN_NOT_CONVERGED;
  if (stats) {
    fm_stats& o = stats[i];
    memset(&o, 0, sizeof o);
    o.iters = k;
    o.increment = inc;
    for (size_t j = 0; j < hist.size() && j < 64; ++j) o.hist[j] = hist[j];
    o.residual_before = o.residual = NAN;
    o.basis_size = s;
  }
  std::vector<double*> X(batch, nullptr);
  X[i] = (*U)[N];
  if (status != FM_ERR_NONFINITE) {
    if (in.kind != FM_FLOW_EXP) FM_TRY(refine({i}, X, prm, stats, st));
    FM_HIP(copy_out(Xout, in.n, X[i], in.np, st));
  }
  if (stats) stats[i].status = status;
  FM_HIP(hipStreamSynchronize(st));
  if (status == FM_ERR_NONFINITE) set_error("an iterate became non-finite");
  return status;
}

// ------------------------------------------------- accelerated marching
// Alg. 8 (Sec. 4, Example 5) for every problem of the flow:
//   X_{k+1} = X_k + dt (I - A X_k + u_k),  u_{k+1} = u_k - dt A u_k,  u_0 = E,
// with u applied while k < accel_steps.  One grouped launch per step holds
// the product A X_k (Euler epilogue adding I and u_k) and A u_k (Euler
// epilogue); X is updated in place (each element by its own thread), u and
// both product operands ping-pong between two buffers because the epilogue
// of one tile must not overwrite what another tile still reads.  Every
// `every` steps R = I - A X is formed in FP64 and ||R||_F^2 reduced into a
// device table read back once at the end.
fm_status Flow::aima(const double* const* X0, const double* const* E, double step, int steps, int accel_steps,
                     int every, double* const* Xout, double* hist, hipStream_t st) {
  struct AW {
    double *x, *u[2], *r;
    void *xo[2], *uo[2];
  };
  std::vector<AW> b(batch);
  const int nh = hist ? steps / every + 1 : 0;
  double *hdev = nullptr, *hpart = nullptr;
  constexpr int HBLK = 16;
  for (int pass = 0; pass < 2; ++pass) {
    prop.measuring = (pass == 0);
    prop.used = 0;
    for (int i = 0; i < batch; ++i) {
      const size_t np2 = (size_t)inst[i].np * inst[i].np;
      b[i].x = (double*)prop.take(np2 * 8);
      b[i].u[0] = (double*)prop.take(np2 * 8);
      b[i].u[1] = (double*)prop.take(np2 * 8);
      b[i].r = hist ? (double*)prop.take(np2 * 8) : nullptr;
      for (int q = 0; q < 2; ++q) {
        b[i].xo[q] = prop.take(np2 * dt_size(dt));
        b[i].uo[q] = prop.take(np2 * dt_size(dt));
      }
    }
    hdev = (double*)prop.take(sizeof(double) * (size_t)std::max(1, batch * nh));
    hpart = (double*)prop.take(sizeof(double) * (size_t)batch * HBLK);
    if (pass == 0) FM_TRY(prop.reserve(prop.used));
  }
  FM_HIP(hipStreamSynchronize(st));
  release_graphs();
  ring.reset();
  // initial values (absent: zero), op-dtype copies of X_0 and u_0
  for (int i = 0; i < batch; ++i) {
    const size_t np2 = (size_t)inst[i].np * inst[i].np;
    FM_HIP(hipMemsetAsync(b[i].x, 0, np2 * 8, st));
    FM_HIP(hipMemsetAsync(b[i].u[0], 0, np2 * 8, st));
  }
  {
    std::vector<double*> dx, du;
    std::vector<const double*> sx, su;
    for (int i = 0; i < batch; ++i) {
      dx.push_back(b[i].x);
      sx.push_back(X0 ? X0[i] : nullptr);
      du.push_back(b[i].u[0]);
      su.push_back(E ? E[i] : nullptr);
    }
    // pad_copy of a subset: copy the present entries one batch at a time
    std::vector<PadItem> it;
    for (int i = 0; i < batch; ++i) {
      if (sx[i]) it.push_back(PadItem{dx[i], sx[i], inst[i].n, inst[i].np});
      if (su[i]) it.push_back(PadItem{du[i], su[i], inst[i].n, inst[i].np});
    }
    if (!it.empty()) {
      void* d = nullptr;
      FM_TRY(push(it.data(), it.size() * sizeof(PadItem), &d, st));
      FM_HIP(launch_pad_copy((const PadItem*)d, (int)it.size(), 1, st));
    }
    std::vector<PrepItem> prep;
    for (int i = 0; i < batch; ++i) {
      const int64_t cnt = (int64_t)inst[i].np * inst[i].np;
      prep.push_back(PrepItem{b[i].x, nullptr, b[i].xo[0], cnt, i, 0});
      prep.push_back(PrepItem{b[i].u[0], nullptr, b[i].uo[0], cnt, i, 0});
    }
    void* d = nullptr;
    FM_TRY(push(prep.data(), prep.size() * sizeof(PrepItem), &d, st));
    FM_HIP(launch_prep((const PrepItem*)d, (int)prep.size(), dt, nullptr, st));
  }
  // launch lists: [accelerated?][parity]; residual list
  struct L {
    GemmCfg cfg;
    const GItem* items;
    const int* ts;
    int n, total, grid;
  };
  auto prepare = [&](std::vector<GItem>& items, bool f64, std::vector<L>& out) -> fm_status {
    std::map<std::pair<int, int>, std::vector<int>> groups;
    for (size_t j = 0; j < items.size(); ++j) {
      const GemmCfg& c = f64 ? inst[items[j].inst].cfg64 : inst[items[j].inst].cfg;
      groups[{c.bm, c.bk}].push_back((int)j);
    }
    for (auto& g : groups) {
      L l;
      l.cfg.dt = f64 ? DT_F64 : dt;
      l.cfg.bm = g.first.first;
      l.cfg.bk = g.first.second;
      std::vector<GItem> sub;
      std::vector<int> ts(1, 0);
      int total = 0;
      for (int j : g.second) {
        sub.push_back(items[j]);
        const int tpn = items[j].np / l.cfg.bm;
        total += tpn * tpn;
        ts.push_back(total);
      }
      void *di = nullptr, *dts = nullptr;
      FM_TRY(push(sub.data(), sub.size() * sizeof(GItem), &di, st));
      FM_TRY(push(ts.data(), ts.size() * sizeof(int), &dts, st));
      l.items = (const GItem*)di;
      l.ts = (const int*)dts;
      l.n = (int)sub.size();
      l.total = total;
      l.grid = std::min(total, gemm_max_grid(l.cfg));
      out.push_back(l);
    }
    return FM_OK;
  };
  std::vector<L> step_l[2][2], res_l;
  for (int acc = 0; acc < 2; ++acc)
    for (int par = 0; par < 2; ++par) {
      std::vector<GItem> items;
      for (int i = 0; i < batch; ++i) {
        const Inst& in = inst[i];
        GItem g = blank_item(in, i);  // X_{k+1} = X_k + dt (I - A X_k [+ u_k])
        g.a = in.Bop;
        g.b = b[i].xo[par];
        g.s[0] = -1.0;
        g.s[2] = step;
        g.s[3] = 1.0;
        g.x = b[i].x;
        g.out1 = b[i].x;
        g.out0 = b[i].xo[par ^ 1];
        if (acc) {
          g.in0 = b[i].u[par];
          g.s[1] = 1.0;
          g.flags = F_E_F64;
        } else {
          g.flags = F_E_NONE;
        }
        items.push_back(g);
        if (acc) {
          GItem q = blank_item(in, i);  // u_{k+1} = u_k - dt A u_k
          q.a = in.Bop;
          q.b = b[i].uo[par];
          q.s[0] = -1.0;
          q.s[2] = step;
          q.flags = F_E_NONE;
          q.x = b[i].u[par];
          q.out1 = b[i].u[par ^ 1];
          q.out0 = b[i].uo[par ^ 1];
          items.push_back(q);
        }
      }
      FM_TRY(prepare(items, false, step_l[acc][par]));
    }
  const DotItem* dots_dev = nullptr;  // per evaluation j: batch items at dots_dev + j * batch
  if (hist) {
    std::vector<GItem> items;
    for (int i = 0; i < batch; ++i) {
      GItem g = blank_item(inst[i], i);  // R = I - A X in FP64
      g.a = inst[i].A64;
      g.b = b[i].x;
      g.s[0] = -1.0;
      g.s[2] = 1.0;
      g.flags = F_E_NONE | F_OUT0_F64;
      g.out0 = b[i].r;
      items.push_back(g);
    }
    FM_TRY(prepare(items, true, res_l));
    std::vector<DotItem> it;
    for (int j = 0; j < nh; ++j)
      for (int i = 0; i < batch; ++i)
        it.push_back(DotItem{b[i].r, b[i].r, (int64_t)inst[i].np * inst[i].np, i * nh + j, 0, nullptr});
    void* d = nullptr;
    FM_TRY(push(it.data(), it.size() * sizeof(DotItem), &d, st));
    dots_dev = (const DotItem*)d;
  }
  auto residual = [&](int j) -> fm_status {
    for (const L& l : res_l) FM_HIP(launch_gemm(l.cfg, EPI_AFFINE, l.items, l.ts, l.n, l.total, l.grid, nullptr, st));
    FM_HIP(launch_dots(dots_dev + (size_t)j * batch, batch, hpart, HBLK, hdev, st));
    return FM_OK;
  };
  // the X and u operands alternate buffers every step (the u buffers stay in
  // step with X even after the cut-off, where they are no longer read)
  for (int k = 0; k < steps; ++k) {
    if (hist && k % every == 0) FM_TRY(residual(k / every));
    const int acc = k < accel_steps ? 1 : 0;
    for (const L& l : step_l[acc][k & 1])
      FM_HIP(launch_gemm(l.cfg, EPI_EULER, l.items, l.ts, l.n, l.total, l.grid, nullptr, st));
  }
  if (hist && steps % every == 0) FM_TRY(residual(steps / every));
  {
    std::vector<double*> dst(batch);
    std::vector<const double*> src(batch);
    for (int i = 0; i < batch; ++i) {
      dst[i] = Xout[i];
      src[i] = b[i].x;
    }
    FM_TRY(pad_copy(dst, src, 0, st));
  }
  if (hist) {
    std::vector<double> h((size_t)batch * nh);
    FM_HIP(hipMemcpyAsync(h.data(), hdev, h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    FM_HIP(hipStreamSynchronize(st));
    for (size_t j = 0; j < h.size(); ++j) hist[j] = std::sqrt(h[j]);
  }
  FM_HIP(hipStreamSynchronize(st));
  return FM_OK;
}

// ----------------------------------------------------------- refinement
// Inverse flows: R = I - A X, X <- X + X R (Newton-Schulz, I - A X+ = R^2).
// Square root: R = A - X^2, X <- X + H with X H + H X = R (full Newton step),
// H by conjugate gradients on the operator H -> X H + H X, which is symmetric
// positive definite in the Frobenius inner product for symmetric positive
// definite X; two FP64 products per CG iteration.  All problems of the batch
// advance together; the relative residual (||R||_F / sqrt(n) for the inverse,
// ||R||_F / ||A||_F for the root) is read back once per refinement step.
static constexpr int REF_DOT_BLOCKS = 32;

fm_status Flow::refine(const std::vector<int>& which, std::vector<double*>& X, const fm_params* prm,
                       fm_stats* stats, hipStream_t st) {
  if (which.empty()) return FM_OK;
  std::vector<double*> R(batch, nullptr), X2(batch, nullptr), H(batch, nullptr), r(batch, nullptr),
      p(batch, nullptr), Ap(batch, nullptr), T(batch, nullptr);
  double *sc = nullptr, *dpart = nullptr;
  for (int pass = 0; pass < 2; ++pass) {
    prop.measuring = (pass == 0);
    prop.used = 0;
    for (int i : which) {
      const size_t np2 = (size_t)inst[i].np * inst[i].np;
      R[i] = (double*)prop.take(np2 * 8);
      X2[i] = (double*)prop.take(np2 * 8);
      if (inst[i].kind == FM_FLOW_SQRT_STEADY) {
        H[i] = (double*)prop.take(np2 * 8);
        r[i] = (double*)prop.take(np2 * 8);
        p[i] = (double*)prop.take(np2 * 8);
        Ap[i] = (double*)prop.take(np2 * 8);
        T[i] = (double*)prop.take(np2 * 8);
      }
    }
    sc = (double*)prop.take((size_t)batch * 6 * 8);  // nrm | rrA | rrB | pap | rr0 | spare
    dpart = (double*)prop.take((size_t)batch * REF_DOT_BLOCKS * 8);
    if (pass == 0) {
      FM_HIP(hipStreamSynchronize(st));
      FM_TRY(prop.reserve(prop.used));
    }
  }
  double* nrm = sc;
  double* rrA = sc + batch;
  double* rrB = sc + 2 * batch;
  double* pap = sc + 3 * batch;
  FM_TRY(ensure_hredu((size_t)batch * 2 + 2));

  auto dots = [&](const std::vector<int>& ids, const std::vector<const double*>& a,
                  const std::vector<const double*>& b, double* out) -> fm_status {
    std::vector<DotItem> it;
    for (size_t j = 0; j < ids.size(); ++j) {
      const int i = ids[j];
      it.push_back(DotItem{a[j], b[j], (int64_t)inst[i].np * inst[i].np, i, 0, nullptr});
    }
    if (it.empty()) return FM_OK;
    void* d = nullptr;
    FM_TRY(push(it.data(), it.size() * sizeof(DotItem), &d, st));
    FM_HIP(launch_dots((const DotItem*)d, (int)it.size(), dpart, REF_DOT_BLOCKS, out, st));
    return FM_OK;
  };
  auto fetch = [&](const double* d) -> fm_status {
    FM_HIP(hipMemcpyAsync(hredu, d, batch * sizeof(double), hipMemcpyDeviceToHost, st));
    FM_HIP(hipStreamSynchronize(st));
    ring.reset();
    return FM_OK;
  };

  std::vector<double> scale(batch, 1.0);
  {
    std::vector<int> ids;
    std::vector<const double*> a;
    for (int i : which)
      if (inst[i].kind == FM_FLOW_SQRT_STEADY) {
        ids.push_back(i);
        a.push_back(inst[i].A64);
      }
    FM_TRY(dots(ids, a, a, nrm));
    FM_TRY(fetch(nrm));
    for (int i : which)
      scale[i] = inst[i].kind == FM_FLOW_SQRT_STEADY ? std::sqrt(hredu[i]) : std::sqrt((double)inst[i].n);
  }

  std::vector<int> active = which;
  std::vector<int> steps(batch, 0);
  bool first = true;
  while (!active.empty()) {
    // residuals
    std::vector<GItem> items;
    std::vector<int> ii;
    for (int i : active) {
      const Inst& in = inst[i];
      GItem g = blank_item(in, i);
      g.out0 = R[i];
      if (in.kind == FM_FLOW_SQRT_STEADY) {  // R = A - X X
        g.a = X[i];
        g.b = X[i];
        g.in0 = in.A64;
        g.s[0] = -1.0;
        g.s[1] = 1.0;
        g.flags = F_OUT0_F64 | F_E_F64;
      } else {  // R = I - A X
        g.a = in.A64;
        g.b = X[i];
        g.s[0] = -1.0;
        g.s[2] = 1.0;
        g.flags = F_OUT0_F64 | F_E_NONE;
      }
      items.push_back(g);
      ii.push_back(i);
    }
    FM_TRY(gemm_groups(EPI_AFFINE, items, ii, true, st));
    {
      std::vector<const double*> a;
      for (int i : active) a.push_back(R[i]);
      FM_TRY(dots(active, a, a, nrm));
      FM_TRY(fetch(nrm));
    }
    std::vector<int> next, next_inv, next_sqrt;
    for (int i : active) {
      const double res = std::sqrt(hredu[i]) / scale[i];
      if (stats) {
        if (first) stats[i].residual_before = res;
        stats[i].residual = res;
        stats[i].refine_steps = steps[i];
      }
      if (res > prm[i].refine_tol && steps[i] < prm[i].max_refine) {
        next.push_back(i);
        (inst[i].kind == FM_FLOW_SQRT_STEADY ? next_sqrt : next_inv).push_back(i);
      }
    }
    first = false;
    if (next.empty()) break;
    // Newton-Schulz: X2 = X + X R
    {
      std::vector<GItem> upd;
      std::vector<int> ui;
      for (int i : next_inv) {
        GItem g = blank_item(inst[i], i);
        g.a = X[i];
        g.b = R[i];
        g.in0 = X[i];
        g.out0 = X2[i];
        g.s[0] = 1.0;
        g.s[1] = 1.0;
        g.flags = F_OUT0_F64 | F_E_F64;
        upd.push_back(g);
        ui.push_back(i);
      }
      FM_TRY(gemm_groups(EPI_AFFINE, upd, ui, true, st));
    }
    // Newton for the root: CG on X H + H X = R, then X2 = X + H
    if (!next_sqrt.empty()) {
      std::vector<CgItem> cg;
      for (int i : next_sqrt) cg.push_back(CgItem{H[i], r[i], p[i], R[i], (int64_t)inst[i].np * inst[i].np, i, 0});
      void* d = nullptr;
      FM_TRY(push(cg.data(), cg.size() * sizeof(CgItem), &d, st));
      FM_HIP(launch_cg_init((const CgItem*)d, (int)cg.size(), st));
      std::vector<int> cg_act = next_sqrt;
      {
        std::vector<const double*> a;
        for (int i : cg_act) a.push_back(r[i]);
        FM_TRY(dots(cg_act, a, a, rrA));
        FM_TRY(fetch(rrA));
      }
      std::vector<double> rr0(batch, 0.0);
      for (int i : cg_act) rr0[i] = hredu[i];
      double* rr_cur = rrA;
      double* rr_nxt = rrB;
      const int max_cg = 600;
      const double cg_tol = 1e-13;
      for (int it = 0; it < max_cg && !cg_act.empty(); ++it) {
        std::vector<GItem> g1, g2;
        std::vector<int> i1;
        std::vector<CgItem> ci;
        std::vector<const double*> pa, apa, ra;
        for (int i : cg_act) {
          GItem a = blank_item(inst[i], i);  // T = X p
          a.a = X[i];
          a.b = p[i];
          a.out0 = T[i];
          a.s[0] = 1.0;
          a.flags = F_OUT0_F64 | F_E_NONE;
          g1.push_back(a);
          GItem b = blank_item(inst[i], i);  // Ap = p X + T
          b.a = p[i];
          b.b = X[i];
          b.in0 = T[i];
          b.out0 = Ap[i];
          b.s[0] = 1.0;
          b.s[1] = 1.0;
          b.flags = F_OUT0_F64 | F_E_F64;
          g2.push_back(b);
          i1.push_back(i);
          ci.push_back(CgItem{H[i], r[i], p[i], Ap[i], (int64_t)inst[i].np * inst[i].np, i, 0});
          pa.push_back(p[i]);
          apa.push_back(Ap[i]);
          ra.push_back(r[i]);
        }
        FM_TRY(gemm_groups(EPI_AFFINE, g1, i1, true, st));
        FM_TRY(gemm_groups(EPI_AFFINE, g2, i1, true, st));
        FM_TRY(dots(cg_act, pa, apa, pap));
        void* dci = nullptr;
        FM_TRY(push(ci.data(), ci.size() * sizeof(CgItem), &dci, st));
        FM_HIP(launch_cg_step1((const CgItem*)dci, (int)ci.size(), rr_cur, pap, st));
        FM_TRY(dots(cg_act, ra, ra, rr_nxt));
        if (it % 8 == 7 || it == max_cg - 1) {
          FM_TRY(fetch(rr_nxt));
          std::vector<int> keep;
          for (int i : cg_act)
            if (!(std::sqrt(hredu[i]) <= cg_tol * std::sqrt(rr0[i]))) keep.push_back(i);
          // continue with the unconverged problems only; the ring was reset
          // by the read-back, so the list is pushed again
          cg_act = keep;
          ci.clear();
          for (int i : cg_act) ci.push_back(CgItem{H[i], r[i], p[i], Ap[i], (int64_t)inst[i].np * inst[i].np, i, 0});
          if (!ci.empty()) FM_TRY(push(ci.data(), ci.size() * sizeof(CgItem), &dci, st));
        }
        if (!ci.empty()) FM_HIP(launch_cg_step2((const CgItem*)dci, (int)ci.size(), rr_nxt, rr_cur, st));
        std::swap(rr_cur, rr_nxt);
      }
      std::vector<CgItem> add;
      for (int i : next_sqrt) {
        FM_HIP(copy_f64(X2[i], X[i], (int64_t)inst[i].np * inst[i].np, st));
        add.push_back(CgItem{X2[i], nullptr, nullptr, H[i], (int64_t)inst[i].np * inst[i].np, i, 0});
      }
      void* da = nullptr;
      FM_TRY(push(add.data(), add.size() * sizeof(CgItem), &da, st));
      FM_HIP(launch_add((const CgItem*)da, (int)add.size(), st));
    }
    for (int i : next) {
      std::swap(X[i], X2[i]);
      steps[i]++;
    }
    active = next;
  }
  // X[i] may now point into the refinement scratch; the caller copies it out
  // before the scratch is reused.
  return FM_OK;
}

// Forward Euler in the learned step family: X+ = X (I - K) for both flows
// (K = h (A - I) X for the homotopy, h (A X - I) for X - X A X).
void euler_coeffs(int kind, double h, double* c) {
  (void)kind;
  (void)h;
  for (int q = 0; q < 8; ++q) c[q] = 0.0;
  c[0] = 1.0;
  c[1] = -1.0;
}

fm_status Flow::set_model(int kind, const double* theta, const double* norm) {
  const int np = mlp_param_count();
  model.kind = kind;
  model.theta.assign(theta, theta + np);
  for (int q = 0; q < 12; ++q) model.norm[q] = norm[q];
  for (int q = 6; q < 12; ++q)
    if (!(model.norm[q] > 0)) {
      set_error("network input std must be positive");
      return FM_ERR_INVALID;
    }
  std::vector<float> tf(theta, theta + np), nf(norm, norm + 12);
  if (!model.d_theta) FM_HIP(hipMalloc((void**)&model.d_theta, np * sizeof(float)));
  if (!model.d_norm) FM_HIP(hipMalloc((void**)&model.d_norm, 12 * sizeof(float)));
  FM_HIP(hipMemcpy(model.d_theta, tf.data(), np * sizeof(float), hipMemcpyHostToDevice));
  FM_HIP(hipMemcpy(model.d_norm, nf.data(), 12 * sizeof(float), hipMemcpyHostToDevice));
  model.loaded = true;
  return FM_OK;
}

// Weight file: 8-byte magic "FMMLP001", int32 kind, int32 count (9288),
// double norm[12] (input mean[6], std[6]), double theta[count]; little endian.
fm_status Flow::load_model(const std::string& path) {
  FILE* f = fopen(path.c_str(), "rb");
  if (!f) {
    set_error("cannot open coarse model %s", path.c_str());
    return FM_ERR_INVALID;
  }
  char magic[8];
  int32_t kind = 0, count = 0;
  double norm[12];
  bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, "FMMLP001", 8) == 0 && fread(&kind, 4, 1, f) == 1 &&
            fread(&count, 4, 1, f) == 1 && count == mlp_param_count() && fread(norm, 8, 12, f) == 12;
  std::vector<double> th(count > 0 ? count : 0);
  ok = ok && fread(th.data(), 8, count, f) == (size_t)count;
  fclose(f);
  if (!ok) {
    set_error("coarse model %s is not a valid weight file", path.c_str());
    return FM_ERR_INVALID;
  }
  return set_model(kind, th.data(), norm);
}

// mu_j = tr((A - I)^j) / n from M = A - I and M^2 (one FP64 product each).
fm_status Flow::ensure_moments(hipStream_t st) {
  for (int i = 0; i < batch; ++i) {
    Inst& in = inst[i];
    if (in.mu_ready) continue;
    const size_t np2 = (size_t)in.np * in.np;
    double *M = nullptr, *M2 = nullptr, *out = nullptr;
    FM_HIP(hipMalloc((void**)&M, np2 * 8));
    FM_HIP(hipMalloc((void**)&M2, np2 * 8));
    FM_HIP(hipMalloc((void**)&out, 4 * 8));
    fm_status s = FM_OK;
    hipError_t e = convert_f64(M, DT_F64, in.A64, -1.0, in.n, in.np, st);
    if (e == hipSuccess) {
      std::vector<GItem> it(1, GItem{});
      it[0].np = in.np;
      it[0].n = in.n;
      it[0].inst = i;
      it[0].a = M;
      it[0].b = M;
      it[0].out0 = M2;
      it[0].s[0] = 1.0;
      it[0].flags = F_OUT0_F64 | F_E_NONE;
      std::vector<int> ii(1, i);
      s = gemm_groups(EPI_AFFINE, it, ii, true, st);
      if (s == FM_OK) e = trace_moments(M, M2, in.n, in.np, out, st);
      if (s == FM_OK && e == hipSuccess) e = hipMemcpyAsync(in.mu, out, 4 * 8, hipMemcpyDeviceToHost, st);
      if (s == FM_OK && e == hipSuccess) e = hipStreamSynchronize(st);
    }
    (void)hipFree(M);
    (void)hipFree(M2);
    (void)hipFree(out);
    if (s != FM_OK) return s;
    if (e != hipSuccess) return hip_status(e, "trace moments");
    in.mu_ready = true;
  }
  ring.reset();
  return FM_OK;
}

fm_status Flow::learned_table(const std::vector<CoefRow>& rows, double* coef, hipStream_t st) {
  if (rows.empty()) return FM_OK;
  if (!model.loaded) {
    set_error("learned coarse step requested but no coarse model is loaded");
    return FM_ERR_INVALID;
  }
  FM_TRY(ensure_moments(st));
  const int64_t S = (int64_t)rows.size();
  std::vector<float> X(S * 6);
  for (int64_t r = 0; r < S; ++r) {
    const Inst& in = inst[rows[r].inst];
    X[r * 6 + 0] = (float)rows[r].t;
    X[r * 6 + 1] = (float)rows[r].h;
    for (int q = 0; q < 4; ++q) X[r * 6 + 2 + q] = (float)in.mu[q];
  }
  float *dX = nullptr, *dY = nullptr;
  FM_HIP(hipMalloc((void**)&dX, S * 6 * sizeof(float)));
  hipError_t e = hipMalloc((void**)&dY, S * 8 * sizeof(float));
  std::vector<float> Y(S * 8);
  if (e == hipSuccess) e = hipMemcpyAsync(dX, X.data(), S * 6 * sizeof(float), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = mlp_forward(model.d_theta, model.d_norm, dX, S, dY, nullptr, st);
  if (e == hipSuccess) e = hipMemcpyAsync(Y.data(), dY, S * 8 * sizeof(float), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(dX);
  if (dY) (void)hipFree(dY);
  if (e != hipSuccess) return hip_status(e, "network inference");
  for (int64_t r = 0; r < S; ++r) {
    euler_coeffs(inst[rows[r].inst].kind, rows[r].h, coef + r * 8);
    for (int q = 0; q < 8; ++q) coef[r * 8 + q] += (double)Y[r * 8 + q];
  }
  return FM_OK;
}

// Fitting features of the learned step family for state/target pairs, one per
// problem: K = h B X, K^2, K^3, X K, X K^2, X K^3 by FP64 products, then the
// Gram data of the basis (see mlp.hip).
fm_status Flow::features(double h, const double* const* X, const double* const* FX, double* G, double* bD,
                         double* fD, double* fn, int64_t row0, hipStream_t st) {
  for (int i = 0; i < batch; ++i)
    if (inst[i].kind == FM_FLOW_SQRT_STEADY) {
      set_error("learned-step features are defined for the inverse flows only");
      return FM_ERR_UNSUPPORTED;
    }
  struct Buf {
    double *B, *x, *f, *k[3], *xk[3];
  };
  std::vector<Buf> b(batch);
  double* part = nullptr;
  const int nblk = 16;
  for (int i = 0; i < batch; ++i) FM_TRY(ensure_b64(i, st));
  for (int pass = 0; pass < 2; ++pass) {
    prop.measuring = (pass == 0);
    prop.used = 0;
    for (int i = 0; i < batch; ++i) {
      const size_t np2 = (size_t)inst[i].np * inst[i].np * 8;
      b[i].B = inst[i].B64;
      b[i].x = (double*)prop.take(np2);
      b[i].f = (double*)prop.take(np2);
      for (int q = 0; q < 3; ++q) {
        b[i].k[q] = (double*)prop.take(np2);
        b[i].xk[q] = (double*)prop.take(np2);
      }
    }
    part = (double*)prop.take((size_t)batch * nblk * 46 * 8);
    if (pass == 0) {
      FM_HIP(hipStreamSynchronize(st));
      FM_TRY(prop.reserve(prop.used));
    }
  }
  ring.reset();
  std::vector<int> ii(batch);
  {
    std::vector<double*> dx(batch), df(batch);
    std::vector<const double*> sx(batch), sf(batch);
    for (int i = 0; i < batch; ++i) {
      ii[i] = i;
      dx[i] = b[i].x;
      sx[i] = X[i];
      df[i] = b[i].f;
      sf[i] = FX[i];
    }
    FM_TRY(pad_copy(dx, sx, 1, st));
    FM_TRY(pad_copy(df, sf, 1, st));
  }
  auto prod = [&](int which, double scale) -> fm_status {
    std::vector<GItem> it;
    for (int i = 0; i < batch; ++i) {
      GItem g = blank_item(inst[i], i);
      g.s[0] = scale;
      g.flags = F_OUT0_F64 | F_E_NONE;
      switch (which) {
        case 0:  // K = h (A - I) X, or h (A X - I) for X - X A X
          g.a = b[i].B;
          g.b = b[i].x;
          g.out0 = b[i].k[0];
          if (inst[i].kind == FM_FLOW_INV_STEADY) g.s[2] = -scale;
          break;
        case 1: g.a = b[i].k[0]; g.b = b[i].k[0]; g.out0 = b[i].k[1]; break;  // K^2
        case 2: g.a = b[i].k[1]; g.b = b[i].k[0]; g.out0 = b[i].k[2]; break;  // K^3
        default: g.a = b[i].x; g.b = b[i].k[which - 3]; g.out0 = b[i].xk[which - 3];  // X K^j
      }
      it.push_back(g);
    }
    return gemm_groups(EPI_AFFINE, it, ii, true, st);
  };
  FM_TRY(prod(0, h));
  for (int w = 1; w < 6; ++w) FM_TRY(prod(w, 1.0));
  std::vector<FeatItem> fi(batch);
  for (int i = 0; i < batch; ++i) {
    FeatItem& q = fi[i];
    q.x = b[i].x;
    for (int j = 0; j < 3; ++j) {
      q.xk[j] = b[i].xk[j];
      q.k[j] = b[i].k[j];
    }
    q.f = b[i].f;
    euler_coeffs(inst[i].kind, h, q.ce);
    q.np = inst[i].np;
    q.n = inst[i].n;
    q.out = row0 + i;
  }
  void* d = nullptr;
  FM_TRY(push(fi.data(), fi.size() * sizeof(FeatItem), &d, st));
  FM_HIP(::fm::features((const FeatItem*)d, batch, part, nblk, G, bD, fD, fn, st));
  return FM_OK;
}

}  // namespace fm
