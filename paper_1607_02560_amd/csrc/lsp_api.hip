// Host side of liblsp: argument validation, the problem object and its
// workspaces, the stencil-setup launch sequence and the GMRES driver.
// Every entry point declared in include/lsp.h is defined here.
#include <math.h>
#include <stdlib.h>
#include <stdio.h>
#include <string.h>

#include <complex>
#include <new>
#include <string>
#include <vector>

#include "lsp_internal.h"

namespace {
thread_local std::string g_last_error;

bool is_pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

// Free a device pointer and null it.
template <typename T>
void dfree(T*& ptr) {
  if (ptr) (void)hipFree(ptr);
  ptr = nullptr;
}

int dalloc(void** ptr, size_t bytes, const char* what) {
  hipError_t e = hipMalloc(ptr, bytes);
  if (e != hipSuccess) {
    *ptr = nullptr;
    (void)hipGetLastError();
    return lsp::set_error(LSP_ENOMEM, std::string("device allocation failed: ") + what + " (" +
                                          std::to_string(bytes) + " bytes)");
  }
  return LSP_OK;
}

void free_workspace(lsp_problem* p) {
  lsp::Workspace& w = p->ws;
  dfree(w.minmax_part);
  dfree(w.S);
  dfree(w.nS);
  dfree(w.vrange);
  dfree(w.green_part);
  dfree(w.gtab);
  dfree(w.gamtab);
  dfree(w.Mtab);
  dfree(w.alpha);
  dfree(w.Ctab);
  dfree(w.sigma);
  dfree(w.rho);
  dfree(w.actab);
  dfree(w.status);
  w.cap_shifts = w.cap_m = w.cap_w = 0;
  w.green_part_cap = 0;
}

int ensure_workspace(lsp_problem* p, int shifts, int t, int m, int wd) {
  lsp::Workspace& w = p->ws;
  int rc = LSP_OK;
  if (!w.minmax_part) {
    if ((rc = dalloc((void**)&w.minmax_part, sizeof(double) * 3 * lsp::kMinMaxBlocks, "minmax")))
      return rc;
    if ((rc = dalloc((void**)&w.S, sizeof(double) * lsp::kMaxShifts, "S"))) return rc;
    if ((rc = dalloc((void**)&w.nS, sizeof(int), "nS"))) return rc;
    if ((rc = dalloc((void**)&w.vrange, sizeof(double) * 2, "vrange"))) return rc;
    if (hipMemsetAsync(w.nS, 0, sizeof(int), p->stream) != hipSuccess)
      return lsp::set_error(LSP_EHIP, "hipMemsetAsync(nS) failed");
  }
  const size_t gneed = lsp::green_partial_doubles(p->d, p->n, t, shifts);
  if (gneed > w.green_part_cap) {
    ++p->ws_gen;
    (void)hipStreamSynchronize(p->stream);
    dfree(w.green_part);
    if ((rc = dalloc((void**)&w.green_part, sizeof(double) * gneed, "green partial sums")))
      return rc;
    w.green_part_cap = gneed;
  }
  if (shifts > w.cap_shifts || m > w.cap_m || wd > w.cap_w) {
    ++p->ws_gen;
    (void)hipStreamSynchronize(p->stream);
    dfree(w.gtab);
    dfree(w.gamtab);
    dfree(w.Mtab);
    dfree(w.alpha);
    dfree(w.Ctab);
    dfree(w.sigma);
    dfree(w.rho);
    dfree(w.actab);
    dfree(w.status);
    const int cs = shifts > w.cap_shifts ? shifts : w.cap_shifts;
    const int cm = m > w.cap_m ? m : w.cap_m;
    const int cw = wd > w.cap_w ? wd : w.cap_w;
    if ((rc = dalloc((void**)&w.gtab, sizeof(double) * cs * cw, "g table"))) return rc;
    if ((rc = dalloc((void**)&w.gamtab, sizeof(double) * cs * cw, "g*g table"))) return rc;
    if ((rc = dalloc((void**)&w.Mtab, sizeof(double) * cs * cm * cm, "Gram matrices"))) return rc;
    if ((rc = dalloc((void**)&w.alpha, sizeof(double) * cs * cm, "alpha"))) return rc;
    if ((rc = dalloc((void**)&w.Ctab, sizeof(double) * cs * cm, "C"))) return rc;
    if ((rc = dalloc((void**)&w.sigma, sizeof(double) * cs, "sigma"))) return rc;
    if ((rc = dalloc((void**)&w.rho, sizeof(double) * cs, "rho*"))) return rc;
    if ((rc = dalloc((void**)&w.actab, sizeof(double) * 2 * cs * cm, "alpha/C"))) return rc;
    if ((rc = dalloc((void**)&w.status, sizeof(int) * cs, "status"))) return rc;
    w.cap_shifts = cs;
    w.cap_m = cm;
    w.cap_w = cw;
  }
  return LSP_OK;
}

// cw[k][delta] = w(k) cos(2 pi k delta / n), k in [0, n/2], delta in [0, W):
// the folded cosine weights of the Green's sums (w = 1 at k = 0, n/2; else 2),
// computed on the device; in 3D also the Green's-sum work units.
int upload_cos_table(lsp_problem* p, int W) {
  ++p->ws_gen;
  int rc = dalloc((void**)&p->cosT, sizeof(double) * (size_t)lsp::cos_table_doubles(p->n, W),
                  "cos table");
  if (rc) return rc;
  hipError_t e = lsp::launch_cos_table(p->n, W, p->cosT, p->stream);
  if (e != hipSuccess) return lsp::hip_check(e, "cosine table");
  if (p->d == 3 && !p->green_units) {
    std::vector<int> units;
    lsp::green_units(p->d, p->n, units);
    if ((rc = dalloc((void**)&p->green_units, sizeof(int) * units.size(), "green units")))
      return rc;
    if (hipMemcpy(p->green_units, units.data(), sizeof(int) * units.size(),
                  hipMemcpyHostToDevice) != hipSuccess)
      return lsp::set_error(LSP_EHIP, "upload of the Green's-sum units failed");
    p->green_nunits = (int)units.size();
  }
  return LSP_OK;
}

int check_finite_device(lsp_problem* p, const double* x, int64_t count, const char* what) {
  hipError_t e = lsp::launch_count_nonfinite(x, count, p->flag, p->stream);
  if (e != hipSuccess) return lsp::hip_check(e, "non-finite check");
  int bad = 0;
  e = hipMemcpyAsync(&bad, p->flag, sizeof(int), hipMemcpyDeviceToHost, p->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return lsp::hip_check(e, "non-finite check readback");
  if (bad)
    return lsp::set_error(LSP_ENONFINITE,
                          std::string(what) + " has " + std::to_string(bad) + " non-finite values");
  return LSP_OK;
}

// Eigen-solver status of the last setup's shifts: LSP_ERESONANT when the
// Gram block of some shift could not be factorised (its null vector, and so
// its rows, are not valid). Synchronises the stream.
int check_setup_status(lsp_problem* p) {
  hipError_t e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return lsp::hip_check(e, "synchronise");
  int ns = 0;
  e = hipMemcpy(&ns, p->ws.nS, sizeof(int), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return lsp::hip_check(e, "read |S|");
  if (ns <= 0) return LSP_OK;
  std::vector<int> st(ns);
  e = hipMemcpy(st.data(), p->ws.status, sizeof(int) * ns, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return lsp::hip_check(e, "status copy");
  for (int i = 0; i < ns; ++i)
    if (st[i] < 0)
      return lsp::set_error(LSP_ERESONANT, "Gram matrix of shift " + std::to_string(i) +
                                               " could not be factorised");
  if (p->nd_leaf > 0 && p->nd1.status && ns <= p->nd1_shifts) {
    // the radius-1 tables of a per-point-radius setup
    e = hipMemcpy(st.data(), p->nd1.status, sizeof(int) * ns, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return lsp::hip_check(e, "status copy");
    for (int i = 0; i < ns; ++i)
      if (st[i] < 0)
        return lsp::set_error(LSP_ERESONANT, "radius-1 Gram matrix of shift " +
                                                 std::to_string(i) + " could not be factorised");
  }
  return LSP_OK;
}

void drop_graph(lsp_problem::GraphCache& gc) {
  if (gc.exec) (void)hipGraphExecDestroy(gc.exec);
  gc.exec = nullptr;
  gc.valid = false;
}

// Run a launch sequence through a cached HIP graph: replay it when the key
// (arguments and workspace generation) matches the captured one, otherwise
// capture it anew. For a single problem graphs are opt-in (LSP_GRAPHS=1): on
// this platform a graph launch of the setup's four kernels costs about 6 us
// more than launching them directly (73 us against 67 us at n = 1024), and
// the apply's three about 7 us more. Without graphs (the default, profiling,
// the legacy default stream) the sequence is launched directly.
hipError_t run_graph(lsp_problem* p, lsp_problem::GraphCache& gc, const uint64_t (&key)[6],
                     const std::function<hipError_t()>& launch) {
  if (!p->use_graphs || p->profiling || p->stream == nullptr) return launch();
  bool same = gc.valid;
  for (int i = 0; i < 6 && same; ++i) same = (gc.key[i] == key[i]);
  if (!same) {
    drop_graph(gc);
    hipError_t e = hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      p->use_graphs = false;
      return launch();
    }
    const hipError_t le = launch();
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(p->stream, &graph);
    if (le != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return le;
    }
    if (e != hipSuccess) return e;
    e = hipGraphInstantiate(&gc.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      gc.exec = nullptr;
      return e;
    }
    for (int i = 0; i < 6; ++i) gc.key[i] = key[i];
    gc.valid = true;
  }
  return hipGraphLaunch(gc.exec, p->stream);
}

}  // namespace

namespace lsp {

void free_device_gmres(lsp_problem* p) {
  for (lsp_problem::GraphCache& gc : p->g_arnoldi) drop_graph(gc);
  p->g_arnoldi.clear();
  dfree(p->dk);
  p->dk_doubles = 0;
  if (p->dk_host) (void)hipHostFree(p->dk_host);
  p->dk_host = nullptr;
}

bool graphs_enabled(bool by_default) {
  const char* g = getenv("LSP_GRAPHS");
  if (!g || !g[0]) return by_default;
  return g[0] != '0';
}

int set_error(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return LSP_OK;
  return set_error(LSP_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

static hipEvent_t next_event(lsp_problem* p) {
  if (p->ev_used == p->ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    p->ev_pool.push_back(e);
  }
  return p->ev_pool[p->ev_used++];
}

// Fold finished event pairs into the totals and recycle the pool.
static void drain_events(lsp_problem* p) {
  (void)hipStreamSynchronize(p->stream);
  for (const auto& pr : p->ev_pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p->ev_pool[pr.second], p->ev_pool[pr.second + 1]) ==
        hipSuccess) {
      p->prof_ms[pr.first] += ms;
      p->prof_count[pr.first] += 1;
    }
  }
  p->ev_pending.clear();
  p->ev_used = 0;
}

int stage_begin(lsp_problem* p, int stage) {
  if (!p->profiling) return -1;
  const size_t i0 = p->ev_used;
  hipEvent_t a = next_event(p);
  hipEvent_t b = next_event(p);
  if (!a || !b) return -1;
  (void)hipEventRecord(a, p->stream);
  p->ev_pending.emplace_back(stage, (int)i0);
  return (int)p->ev_pending.size() - 1;
}

void stage_end(lsp_problem* p, int token) {
  if (token < 0 || !p->profiling) return;
  const int i0 = p->ev_pending[token].second;
  (void)hipEventRecord(p->ev_pool[i0 + 1], p->stream);
}

}  // namespace lsp

extern "C" {

const char* lsp_strerror(int code) {
  switch (code) {
    case LSP_OK: return "ok";
    case LSP_NOT_CONVERGED: return "not converged";
    case LSP_EINVAL: return "invalid argument";
    case LSP_ENONFINITE: return "non-finite input";
    case LSP_ERESONANT: return "resonant shift";
    case LSP_ENOMEM: return "out of memory";
    case LSP_EHIP: return "HIP runtime error";
    case LSP_ESOLVER: return "host P-solve failed";
    case LSP_ESTATE: return "invalid call order";
    default: return "unknown status";
  }
}

const char* lsp_last_error(void) { return g_last_error.c_str(); }

const char* lsp_version(void) { return "liblsp 0.1 (gfx950)"; }

int lsp_create(int d, int n, const double* v_dev, void* stream, lsp_problem** out) {
  if (!out) return lsp::set_error(LSP_EINVAL, "out is NULL");
  *out = nullptr;
  if (d != 2 && d != 3) return lsp::set_error(LSP_EINVAL, "d must be 2 or 3");
  const int nmax = (d == 2) ? 1024 : 256;
  if (!is_pow2(n) || n < 8 || n > nmax)
    return lsp::set_error(LSP_EINVAL, "n must be a power of two in [8, " +
                                          std::to_string(nmax) + "] for d = " + std::to_string(d));
  if (!v_dev) return lsp::set_error(LSP_EINVAL, "v_dev is NULL");
  lsp_problem* p = new (std::nothrow) lsp_problem();
  if (!p) return lsp::set_error(LSP_ENOMEM, "host allocation failed");
  p->d = d;
  p->n = n;
  p->N = 1;
  for (int i = 0; i < d; ++i) p->N *= n;
  p->stream = reinterpret_cast<hipStream_t>(stream);
  p->use_graphs = lsp::graphs_enabled(false);
  p->krylov_graphs = lsp::graphs_enabled(true);
  (void)hipGetDevice(&p->device);
  if (hipDeviceGetAttribute(&p->cus, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess)
    p->cus = 0;
  int rc = LSP_OK;
  if ((rc = dalloc((void**)&p->v, sizeof(double) * p->N, "potential")) ||
      (rc = dalloc((void**)&p->z, sizeof(double) * 2 * p->N, "apply scratch")) ||
      (rc = dalloc((void**)&p->tw, sizeof(double) * 2 * n, "twiddles")) ||
      (rc = dalloc((void**)&p->flag, sizeof(int), "flag"))) {
    lsp_destroy(p);
    return rc;
  }
  // twiddles exp(-2 pi i j / n)
  std::vector<double> tw(2 * (size_t)n);
  for (int j = 0; j < n; ++j) {
    tw[2 * j] = cos(2.0 * M_PI * j / n);
    tw[2 * j + 1] = -sin(2.0 * M_PI * j / n);
  }
  hipError_t e = hipMemcpy(p->tw, tw.data(), sizeof(double) * 2 * n, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    rc = lsp::hip_check(e, "twiddle upload");
    lsp_destroy(p);
    return rc;
  }
  e = hipMemcpyAsync(p->v, v_dev, sizeof(double) * p->N, hipMemcpyDeviceToDevice, p->stream);
  if (e != hipSuccess) {
    rc = lsp::hip_check(e, "potential copy");
    lsp_destroy(p);
    return rc;
  }
  if ((rc = check_finite_device(p, p->v, p->N, "v"))) {
    lsp_destroy(p);
    return rc;
  }
  *out = p;
  return LSP_OK;
}

int lsp_set_potential(lsp_problem* p, const double* v_dev) {
  if (!p || !v_dev) return lsp::set_error(LSP_EINVAL, "NULL argument");
  hipError_t e =
      hipMemcpyAsync(p->v, v_dev, sizeof(double) * p->N, hipMemcpyDeviceToDevice, p->stream);
  if (e != hipSuccess) return lsp::hip_check(e, "potential copy");
  p->have_setup = false;
  return check_finite_device(p, p->v, p->N, "v");
}

void lsp_destroy(lsp_problem* p) {
  if (!p) return;
  (void)hipStreamSynchronize(p->stream);
  dfree(p->v);
  dfree(p->z);
  dfree(p->tw);
  for (double*& c : p->cos_by_t) dfree(c);
  p->cosT = nullptr;
  dfree(p->green_units);
  dfree(p->c_rows);
  dfree(p->nd_t1);
  dfree(p->learn_buf);
  dfree(p->flag);
  drop_graph(p->g_setup);
  drop_graph(p->g_apply);
  for (hipEvent_t e : p->ev_pool) (void)hipEventDestroy(e);
  p->ev_pool.clear();
  dfree(p->kry);
  dfree(p->red);
  if (p->red_host) (void)hipHostFree(p->red_host);
  lsp::free_psolve(p);
  lsp::free_device_gmres(p);
  free_workspace(p);
  delete p;
}

namespace {
// the candidates of each tuned shape (0: the default)
bool tune_value_ok(int knob, int v) {
  switch (knob) {
    case LSP_TUNE_GREEN_WAVES:
      return v == 0 || v == 512 || v == 1024 || v == 1536 || v == 2048 || v == 3072;
    case LSP_TUNE_ASSEMBLY_TILE: return v == 0 || v == 1 || v == 32 || v == 64 || v == 128;
    case LSP_TUNE_APPLY_FORM: return v == 0 || v == 8 || v == 16;
    default: return false;
  }
}
}  // namespace

int lsp_set_tuning(lsp_problem* p, const int* choice_host) {
  if (!p || !choice_host) return lsp::set_error(LSP_EINVAL, "NULL argument");
  for (int k = 0; k < LSP_TUNE_COUNT; ++k)
    if (!tune_value_ok(k, choice_host[k]))
      return lsp::set_error(LSP_EINVAL, "tuning value " + std::to_string(choice_host[k]) +
                                            " is not a candidate of shape " + std::to_string(k));
  (void)hipStreamSynchronize(p->stream);
  for (int k = 0; k < LSP_TUNE_COUNT; ++k) p->tune[k] = choice_host[k];
  ++p->ws_gen;  // cached graphs hold the old shapes
  return LSP_OK;
}

int lsp_get_tuning(const lsp_problem* p, int* choice_host) {
  if (!p || !choice_host) return lsp::set_error(LSP_EINVAL, "NULL argument");
  for (int k = 0; k < LSP_TUNE_COUNT; ++k) choice_host[k] = p->tune[k];
  return LSP_OK;
}

int lsp_autotune(lsp_problem* p, int t, int num_shifts, int precision, void* P_dev,
                 const double* u_dev, double* y_dev, int reps, int* choice_host,
                 double* ms_host) {
  if (!p || !P_dev || !u_dev || !y_dev) return lsp::set_error(LSP_EINVAL, "NULL argument");
  if (reps < 1 || reps > 1000) return lsp::set_error(LSP_EINVAL, "reps must be in 1..1000");
  hipStream_t s = p->stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return lsp::set_error(LSP_EHIP, "event creation failed");
  }
  // mean time of reps calls of one candidate (after one untimed call)
  auto time_it = [&](bool setup, double* ms) -> int {
    auto call = [&]() -> int {
      return setup ? lsp_stencil_setup(p, t, num_shifts, precision, P_dev, nullptr)
                   : lsp_ps_apply(p, u_dev, y_dev);
    };
    int rc = call();
    if (rc < 0) return rc;
    if (hipEventRecord(e0, s) != hipSuccess) return lsp::set_error(LSP_EHIP, "event record");
    for (int i = 0; i < reps; ++i)
      if ((rc = call()) < 0) return rc;
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
      return lsp::set_error(LSP_EHIP, "event wait");
    float f = 0.f;
    if (hipEventElapsedTime(&f, e0, e1) != hipSuccess) return lsp::set_error(LSP_EHIP, "event time");
    *ms = (double)f / reps;
    return LSP_OK;
  };
  const int n = p->n;
  std::vector<int> cand[LSP_TUNE_COUNT];
  if (p->d == 2) cand[LSP_TUNE_GREEN_WAVES] = {512, 1024, 1536, 2048, 3072};
  if (p->d == 2 && n >= 128) cand[LSP_TUNE_ASSEMBLY_TILE] = {32, 64, 128, 1};
  if (n == 256 || n == 512 || n == 1024) cand[LSP_TUNE_APPLY_FORM] = {8, 16};
  int rc = LSP_OK;
  double best_ms[LSP_TUNE_COUNT] = {0.0, 0.0, 0.0};
  for (int k = 0; k < LSP_TUNE_COUNT && rc == LSP_OK; ++k) {
    const bool setup = (k != LSP_TUNE_APPLY_FORM);
    if (cand[k].empty()) {
      p->tune[k] = 0;
      rc = time_it(setup, &best_ms[k]);
      continue;
    }
    int best = 0;
    double bms = 0.0;
    for (int v : cand[k]) {
      p->tune[k] = v;
      ++p->ws_gen;
      double ms = 0.0;
      if ((rc = time_it(setup, &ms)) != LSP_OK) break;
      if (best == 0 || ms < bms) {
        best = v;
        bms = ms;
      }
    }
    p->tune[k] = best;
    ++p->ws_gen;
    best_ms[k] = bms;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != LSP_OK) return rc;
  for (int k = 0; k < LSP_TUNE_COUNT; ++k) {
    if (choice_host) choice_host[k] = p->tune[k];
    if (ms_host) ms_host[k] = best_ms[k];
  }
  return LSP_OK;
}

int lsp_stencil_size(const lsp_problem* p) { return (p && p->have_setup) ? p->m : 0; }

int lsp_profile(lsp_problem* p, int enable) {
  if (!p) return lsp::set_error(LSP_EINVAL, "problem is NULL");
  if (enable) {
    lsp::drain_events(p);
    for (int i = 0; i < LSP_NUM_STAGES; ++i) {
      p->prof_ms[i] = 0.0;
      p->prof_count[i] = 0;
    }
    p->profiling = true;
  } else {
    lsp::drain_events(p);
    p->profiling = false;
  }
  return LSP_OK;
}

int lsp_profile_read(lsp_problem* p, int nstages, double* ms_host, int* count_host) {
  if (!p || nstages < 0) return lsp::set_error(LSP_EINVAL, "invalid argument");
  lsp::drain_events(p);
  for (int i = 0; i < nstages && i < LSP_NUM_STAGES; ++i) {
    if (ms_host) ms_host[i] = p->prof_ms[i];
    if (count_host) count_host[i] = p->prof_count[i];
  }
  return LSP_OK;
}

int lsp_default_num_shifts(int d, int n) {
  if ((d != 2 && d != 3) || n < 1) return lsp::set_error(LSP_EINVAL, "invalid d or n");
  const int s = (d == 2) ? n / 16 : n / 4;
  return s < 1 ? 1 : s;
}

}  // extern "C"

namespace lsp {

// Validation, workspaces and the cosine table shared by the exact, the
// learned and the batched setup; num_shifts is replaced by the effective request.
int prepare_setup(lsp_problem* p, int t, int* num_shifts_io) {
  int num_shifts = *num_shifts_io;
  if (t < 1) return lsp::set_error(LSP_EINVAL, "t must be >= 1");
  const int W = 2 * t + 1;
  int m = 1;
  for (int i = 0; i < p->d; ++i) m *= W;
  if (m > lsp::kMaxStencil)
    return lsp::set_error(LSP_EINVAL, "stencil size (2t+1)^d = " + std::to_string(m) +
                                          " exceeds " + std::to_string(lsp::kMaxStencil));
  if (W >= p->n) return lsp::set_error(LSP_EINVAL, "2t+1 must be smaller than n");
  if (p->N < 2 * (int64_t)m) return lsp::set_error(LSP_EINVAL, "N must be at least 2m");
  if (p->d == 3 && W != 3 && W != 5)
    return lsp::set_error(LSP_EINVAL, "d = 3 supports t = 1, 2");
  if (p->d == 2 && W > 7) return lsp::set_error(LSP_EINVAL, "d = 2 supports t = 1, 2, 3");
  if (num_shifts == 0) num_shifts = lsp_default_num_shifts(p->d, p->n);
  if (num_shifts < 1) return lsp::set_error(LSP_EINVAL, "num_shifts must be >= 0");
  if (num_shifts > lsp::kMaxShifts)
    return lsp::set_error(LSP_EINVAL, "num_shifts exceeds " + std::to_string(lsp::kMaxShifts));
  int rc = ensure_workspace(p, num_shifts, t, m, m);
  if (rc) return rc;
  // one cosine table per t, uploaded once: switching t (the per-point-radius
  // setup does so twice per call) only repoints cosT
  if (!p->cos_by_t[t]) {
    (void)hipStreamSynchronize(p->stream);
    if ((rc = upload_cos_table(p, W))) return rc;
    p->cos_by_t[t] = p->cosT;
  }
  p->cosT = p->cos_by_t[t];
  p->t = t;
  p->m = m;
  p->num_shifts = num_shifts;
  p->have_setup = false;
  p->learned = false;
  p->nd_leaf = 0;
  *num_shifts_io = num_shifts;
  return LSP_OK;
}

}  // namespace lsp

extern "C" {

int lsp_stencil_setup(lsp_problem* p, int t, int num_shifts, int precision, void* P_dev,
                      int32_t* idx_dev) {
  if (!p) return lsp::set_error(LSP_EINVAL, "problem is NULL");
  if (!P_dev) return lsp::set_error(LSP_EINVAL, "P_dev is NULL");
  if (precision != LSP_FP64 && precision != LSP_FP32_REFINE)
    return lsp::set_error(LSP_EINVAL, "unsupported precision");
  int rc = lsp::prepare_setup(p, t, &num_shifts);
  if (rc) return rc;
  auto launch = [&]() -> hipError_t {
    const int tk_all = lsp::stage_begin(p, LSP_STAGE_SETUP);
    int tk = lsp::stage_begin(p, LSP_STAGE_SHIFTS);
    hipError_t e = lsp::launch_minmax(p);
    if (e != hipSuccess) return e;
    lsp::stage_end(p, tk);
    tk = lsp::stage_begin(p, LSP_STAGE_GREEN);
    e = lsp::launch_green_sums(p, num_shifts);
    if (e != hipSuccess) return e;
    lsp::stage_end(p, tk);
    tk = lsp::stage_begin(p, LSP_STAGE_NULL);
    e = lsp::launch_null_vectors(p, num_shifts);
    if (e != hipSuccess) return e;
    lsp::stage_end(p, tk);
    tk = lsp::stage_begin(p, LSP_STAGE_ASSEMBLE);
    e = lsp::launch_assemble(p, P_dev, precision == LSP_FP32_REFINE, idx_dev);
    if (e != hipSuccess) return e;
    lsp::stage_end(p, tk);
    lsp::stage_end(p, tk_all);
    return hipSuccess;
  };
  const uint64_t key[6] = {(uint64_t)t, (uint64_t)num_shifts, (uint64_t)(uintptr_t)P_dev,
                           (uint64_t)(uintptr_t)idx_dev, p->ws_gen, (uint64_t)precision};
  const hipError_t e = run_graph(p, p->g_setup, key, launch);
  if (e != hipSuccess) return lsp::hip_check(e, "stencil setup launch");
  p->have_setup = true;
  return LSP_OK;
}

int lsp_stencil_setup_global(lsp_problem* p, int t, int precision, void* P_dev,
                             int32_t* idx_dev) {
  if (!p) return lsp::set_error(LSP_EINVAL, "problem is NULL");
  if (!P_dev) return lsp::set_error(LSP_EINVAL, "P_dev is NULL");
  if (precision != LSP_FP64 && precision != LSP_FP32_REFINE)
    return lsp::set_error(LSP_EINVAL, "unsupported precision");
  int num_shifts = 1;
  int rc = lsp::prepare_setup(p, t, &num_shifts);
  if (rc) return rc;
  auto launch = [&]() -> hipError_t {
    const int tk_all = lsp::stage_begin(p, LSP_STAGE_SETUP);
    int tk = lsp::stage_begin(p, LSP_STAGE_SHIFTS);
    hipError_t e = lsp::launch_minmax(p, true);
    if (e != hipSuccess) return e;
    lsp::stage_end(p, tk);
    tk = lsp::stage_begin(p, LSP_STAGE_GREEN);
    e = lsp::launch_green_sums(p, 1, true);
    if (e != hipSuccess) return e;
    lsp::stage_end(p, tk);
    tk = lsp::stage_begin(p, LSP_STAGE_NULL);
    e = lsp::launch_null_vectors(p, 1);
    if (e != hipSuccess) return e;
    lsp::stage_end(p, tk);
    tk = lsp::stage_begin(p, LSP_STAGE_ASSEMBLE);
    e = lsp::launch_assemble(p, P_dev, precision == LSP_FP32_REFINE, idx_dev);
    if (e != hipSuccess) return e;
    lsp::stage_end(p, tk);
    lsp::stage_end(p, tk_all);
    return hipSuccess;
  };
  // the all-ones word keeps this graph apart from a localized setup's
  const uint64_t key[6] = {(uint64_t)t, ~(uint64_t)0, (uint64_t)(uintptr_t)P_dev,
                           (uint64_t)(uintptr_t)idx_dev, p->ws_gen, (uint64_t)precision};
  const hipError_t e = run_graph(p, p->g_setup, key, launch);
  if (e != hipSuccess) return lsp::hip_check(e, "non-localized setup launch");
  p->have_setup = true;
  return LSP_OK;
}

int lsp_stencil_setup_nd(lsp_problem* p, int leaf, int num_shifts, double* P_dev,
                         int32_t* idx_dev) {
  if (!p) return lsp::set_error(LSP_EINVAL, "problem is NULL");
  if (!P_dev) return lsp::set_error(LSP_EINVAL, "P_dev is NULL");
  if (leaf < 2 || p->n % leaf != 0)
    return lsp::set_error(LSP_EINVAL, "the leaf box must be >= 2 and divide n");
  // one shift list and one radius-2 Green's pass; the radius-2 tables go to
  // the workspace and the radius-1 tables (their Green's values are the
  // radius-2 pass's at offsets [0, 2]^d) to the problem's radius-1 area
  int ns = num_shifts;
  int rc = lsp::prepare_setup(p, 2, &ns);
  if (rc) return rc;
  const int d = p->d;
  const size_t m1 = (d == 2) ? 9 : 27;
  const size_t m2 = (d == 2) ? 25 : 125;  // the (alpha, C) pairs in the radius-2 layout
  const size_t per = sizeof(double) * (2 * m1 + m1 * m1 + 2 * m1 + 2) + sizeof(double2) * m2 +
                     sizeof(int);
  const size_t bytes = per * (size_t)ns + 16 * 256;
  if (p->nd_t1_bytes < bytes) {
    (void)hipStreamSynchronize(p->stream);
    dfree(p->nd_t1);
    p->nd_t1_bytes = 0;
    p->nd1 = lsp::NdTables1{};
    if ((rc = dalloc((void**)&p->nd_t1, bytes, "radius-1 tables"))) return rc;
    p->nd_t1_bytes = bytes;
    ++p->ws_gen;
  }
  {
    size_t off = 0;
    auto take = [&](size_t b) {
      char* at = p->nd_t1 + off;
      off = (off + b + 255) / 256 * 256;
      return at;
    };
    const size_t S = (size_t)ns;
    lsp::NdTables1& t1 = p->nd1;
    t1.gtab = reinterpret_cast<double*>(take(sizeof(double) * S * m1));
    t1.gamtab = reinterpret_cast<double*>(take(sizeof(double) * S * m1));
    t1.Mtab = reinterpret_cast<double*>(take(sizeof(double) * S * m1 * m1));
    t1.alpha = reinterpret_cast<double*>(take(sizeof(double) * S * m1));
    t1.C = reinterpret_cast<double*>(take(sizeof(double) * S * m1));
    t1.sigma = reinterpret_cast<double*>(take(sizeof(double) * S));
    t1.rho = reinterpret_cast<double*>(take(sizeof(double) * S));
    t1.actab = reinterpret_cast<double2*>(take(sizeof(double2) * S * m2));
    t1.status = reinterpret_cast<int*>(take(sizeof(int) * S));
    p->nd1_shifts = ns;
  }
  hipError_t e = lsp::launch_minmax(p);
  if (e == hipSuccess) e = lsp::launch_green_sums(p, ns);
  if (e == hipSuccess) e = lsp::launch_null_nd(p, ns, p->nd1);
  if (e == hipSuccess) e = lsp::launch_assemble_nd(p, p->nd1.actab, leaf, P_dev, idx_dev);
  if (e != hipSuccess) return lsp::hip_check(e, "per-point-radius setup");
  p->nd_leaf = leaf;
  p->have_setup = true;
  return LSP_OK;
}

int lsp_training_rows(lsp_problem* p, const double* P_dev, const int64_t* points_dev,
                      int count, float* X_dev, float* T_dev) {
  if (!p || !P_dev || !points_dev || !X_dev || !T_dev)
    return lsp::set_error(LSP_EINVAL, "NULL argument");
  if (!p->have_setup || p->learned)
    return lsp::set_error(LSP_ESTATE, "training rows need a completed exact FP64 setup");
  if (count < 1) return lsp::set_error(LSP_EINVAL, "count must be >= 1");
  hipError_t e = lsp::launch_features(p, points_dev, 0, count, X_dev);
  if (e == hipSuccess) e = lsp::launch_targets(p, P_dev, points_dev, count, T_dev);
  return lsp::hip_check(e, "training rows");
}

int lsp_stencil_setup_learned(lsp_problem* p, lsp_mlp* mlp, int t, int num_shifts,
                              double threshold, double* P_dev, int32_t* fallback_dev,
                              int* n_fallback_host) {
  if (!p || !mlp || !P_dev || !fallback_dev) return lsp::set_error(LSP_EINVAL, "NULL argument");
  if (!(threshold >= 0.0)) return lsp::set_error(LSP_EINVAL, "threshold must be >= 0");
  if (p->d == 3 && t != 1)
    return lsp::set_error(LSP_EINVAL, "the learned setup supports d = 3 with t = 1");
  int rc = lsp::prepare_setup(p, t, &num_shifts);
  if (rc) return rc;
  const int m = p->m;
  if (lsp::mlp_inputs(mlp) != m + 2 || lsp::mlp_outputs(mlp) != 2 * m)
    return lsp::set_error(LSP_EINVAL, "the surrogate needs m + 2 inputs and 2m outputs");
  // per-point C rows and the chunk buffers of the inference
  const size_t need = (size_t)p->N * m;
  if (p->c_rows_cap < need) {
    (void)hipStreamSynchronize(p->stream);
    dfree(p->c_rows);
    p->c_rows_cap = 0;
    if ((rc = dalloc((void**)&p->c_rows, sizeof(double) * need, "learned C rows"))) return rc;
    p->c_rows_cap = need;
  }
  // one buffer: the fallback count and, for the chunked path, the network's
  // inputs [B][m+2] and outputs [B][2m] of one chunk (each part 256-byte
  // aligned)
  const lsp::MlpView mv = lsp::mlp_view(mlp);
  const bool fused = lsp::learned_fused_supported(p, mv);
  const int B = lsp::mlp_batch_rows(mlp);
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t off_nf = 0;
  const size_t off_x = off_nf + 256;
  const size_t off_y = off_x + (fused ? 0 : up(sizeof(float) * (size_t)B * (m + 2)));
  const size_t bytes = off_y + (fused ? 0 : up(sizeof(float) * (size_t)B * 2 * m));
  if (p->learn_cap < bytes) {
    (void)hipStreamSynchronize(p->stream);
    dfree(p->learn_buf);
    p->learn_cap = 0;
    if ((rc = dalloc((void**)&p->learn_buf, bytes, "learned-setup buffers"))) return rc;
    p->learn_cap = bytes;
  }
  const double* rho_star = p->ws.rho;  // written by the null-vector kernel
  int* nfall = reinterpret_cast<int*>(p->learn_buf + off_nf);
  float* X = reinterpret_cast<float*>(p->learn_buf + off_x);
  float* Y = reinterpret_cast<float*>(p->learn_buf + off_y);
  // the network's kernels run on the problem's stream below; work queued on
  // the network's own stream must be finished first
  if (lsp::mlp_stream(mlp) != p->stream) {
    const hipError_t es = hipStreamSynchronize(lsp::mlp_stream(mlp));
    if (es != hipSuccess) return lsp::hip_check(es, "surrogate stream");
  }
  // exact tables (shift list, Green's sums, Gram matrices, null vectors and
  // rho*(s)); the null-vector kernel also clears the fallback counter
  const int tk_all = lsp::stage_begin(p, LSP_STAGE_SETUP);
  int tk = lsp::stage_begin(p, LSP_STAGE_SHIFTS);
  hipError_t e = lsp::launch_minmax(p);
  lsp::stage_end(p, tk);
  tk = lsp::stage_begin(p, LSP_STAGE_GREEN);
  if (e == hipSuccess) e = lsp::launch_green_sums(p, num_shifts);
  lsp::stage_end(p, tk);
  tk = lsp::stage_begin(p, LSP_STAGE_NULL);
  if (e == hipSuccess) e = lsp::launch_null_vectors(p, num_shifts, nfall);
  lsp::stage_end(p, tk);
  // the learned rows take the place of the assembly in the stage timing
  tk = lsp::stage_begin(p, LSP_STAGE_ASSEMBLE);
  if (fused) {
    // one pass: network, check against eq. (A) and rows
    if (e == hipSuccess)
      e = lsp::launch_learned_fused(p, mv, threshold, rho_star, P_dev, p->c_rows, fallback_dev,
                                    nfall);
  } else {
    // learned rows in chunks of B points, each checked against the exact tables
    for (int64_t j0 = 0; e == hipSuccess && j0 < p->N; j0 += B) {
      const int rows = (int)std::min<int64_t>(B, p->N - j0);
      e = lsp::launch_features(p, nullptr, j0, rows, X);
      if (e == hipSuccess) e = lsp::mlp_forward_raw(mlp, X, rows, Y, p->stream);
      if (e == hipSuccess)
        e = lsp::launch_learned_rows(p, rho_star, Y, j0, rows, threshold, P_dev, p->c_rows,
                                     fallback_dev, nfall);
    }
  }
  lsp::stage_end(p, tk);
  lsp::stage_end(p, tk_all);
  int nf = 0;
  if (n_fallback_host) {
    if (e == hipSuccess)
      e = hipMemcpyAsync(&nf, nfall, sizeof(int), hipMemcpyDeviceToHost, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  }
  if (e != hipSuccess) return lsp::hip_check(e, "learned setup");
  if (n_fallback_host) {
    // synchronous call: report a shift whose Gram block failed
    if ((rc = check_setup_status(p))) return rc;
    *n_fallback_host = nf;
  }
  p->have_setup = true;
  p->learned = true;
  return LSP_OK;
}

int lsp_ps_apply(lsp_problem* p, const double* u_dev, double* y_dev) {
  if (!p || !u_dev || !y_dev) return lsp::set_error(LSP_EINVAL, "NULL argument");
  if (u_dev == y_dev) return lsp::set_error(LSP_EINVAL, "u and y must not alias");
  auto launch = [&]() -> hipError_t {
    const int tk = lsp::stage_begin(p, LSP_STAGE_APPLY);
    const hipError_t e = lsp::launch_ps_apply(p, u_dev, y_dev);
    lsp::stage_end(p, tk);
    return e;
  };
  const uint64_t key[6] = {(uint64_t)(uintptr_t)u_dev, (uint64_t)(uintptr_t)y_dev, p->ws_gen,
                           0, 0, 0};
  return lsp::hip_check(run_graph(p, p->g_apply, key, launch), "ps_apply launch");
}

int lsp_c_apply(lsp_problem* p, const double* r_dev, double* z_dev) {
  if (!p || !r_dev || !z_dev) return lsp::set_error(LSP_EINVAL, "NULL argument");
  if (r_dev == z_dev) return lsp::set_error(LSP_EINVAL, "r and z must not alias");
  if (!p->have_setup) return lsp::set_error(LSP_ESTATE, "c_apply needs a completed setup");
  const int tk = lsp::stage_begin(p, LSP_STAGE_CAPPLY);
  const int rc = lsp::hip_check(lsp::launch_c_apply(p, r_dev, z_dev), "c_apply launch");
  lsp::stage_end(p, tk);
  return rc;
}

int lsp_get_tables_nd1(lsp_problem* p, int capacity, int* nS, double* alpha_host,
                       double* C_host, double* sigma_host, double* g_host, double* gam_host) {
  if (!p) return lsp::set_error(LSP_EINVAL, "problem is NULL");
  if (!p->have_setup || p->nd_leaf <= 0 || !p->nd1.status)
    return lsp::set_error(LSP_ESTATE, "the last setup was not a per-point-radius setup");
  hipError_t e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return lsp::hip_check(e, "synchronise");
  int ns = 0;
  e = hipMemcpy(&ns, p->ws.nS, sizeof(int), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return lsp::hip_check(e, "read |S|");
  if (nS) *nS = ns;
  if (capacity < ns) return lsp::set_error(LSP_EINVAL, "capacity smaller than |S|");
  const size_t m1 = (p->d == 2) ? 9 : 27;
  const lsp::NdTables1& t1 = p->nd1;
  struct Copy {
    void* dst;
    const void* src;
    size_t bytes;
  } copies[] = {
      {alpha_host, t1.alpha, sizeof(double) * ns * m1},
      {C_host, t1.C, sizeof(double) * ns * m1},
      {sigma_host, t1.sigma, sizeof(double) * ns},
      {g_host, t1.gtab, sizeof(double) * ns * m1},
      {gam_host, t1.gamtab, sizeof(double) * ns * m1},
  };
  for (const Copy& c : copies) {
    if (!c.dst || c.bytes == 0) continue;
    e = hipMemcpy(c.dst, c.src, c.bytes, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return lsp::hip_check(e, "table copy");
  }
  return check_setup_status(p);
}

int lsp_get_tables(lsp_problem* p, int capacity, int* nS, double* S_host, double* alpha_host,
                   double* C_host, double* sigma_host, double* g_host, double* gam_host,
                   double* M_host) {
  if (!p) return lsp::set_error(LSP_EINVAL, "problem is NULL");
  if (!p->have_setup) return lsp::set_error(LSP_ESTATE, "no setup has been run");
  hipError_t e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return lsp::hip_check(e, "synchronise");
  int ns = 0;
  e = hipMemcpy(&ns, p->ws.nS, sizeof(int), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return lsp::hip_check(e, "read |S|");
  if (nS) *nS = ns;
  if (capacity < ns) return lsp::set_error(LSP_EINVAL, "capacity smaller than |S|");
  const int m = p->m;
  const int W = 2 * p->t + 1;
  int wd = 1;
  for (int i = 0; i < p->d; ++i) wd *= W;
  struct Copy {
    void* dst;
    const void* src;
    size_t bytes;
  } copies[] = {
      {S_host, p->ws.S, sizeof(double) * ns},
      {alpha_host, p->ws.alpha, sizeof(double) * ns * m},
      {C_host, p->ws.Ctab, sizeof(double) * ns * m},
      {sigma_host, p->ws.sigma, sizeof(double) * ns},
      {g_host, p->ws.gtab, sizeof(double) * ns * wd},
      {gam_host, p->ws.gamtab, sizeof(double) * ns * wd},
  };
  for (const Copy& c : copies) {
    if (!c.dst || c.bytes == 0) continue;
    e = hipMemcpy(c.dst, c.src, c.bytes, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return lsp::hip_check(e, "table copy");
  }
  if (M_host && ns > 0) {
    // the device keeps the Gram matrices as packed parity blocks
    std::vector<double> packed((size_t)ns * m * m);
    e = hipMemcpy(packed.data(), p->ws.Mtab, sizeof(double) * packed.size(),
                  hipMemcpyDeviceToHost);
    if (e != hipSuccess) return lsp::hip_check(e, "Gram copy");
    for (int i = 0; i < ns; ++i)
      if (lsp::expand_gram_host(p->d, p->t, packed.data() + (size_t)i * m * m,
                                M_host + (size_t)i * m * m) != 0)
        return lsp::set_error(LSP_EINVAL, "unsupported stencil for the Gram expansion");
  }
  // eigen-solver status: report a failed elimination
  return check_setup_status(p);
}

int lsp_export_pattern(int d, int n, int t, int64_t* col_host) {
  if (!col_host) return lsp::set_error(LSP_EINVAL, "col_host is NULL");
  if ((d != 2 && d != 3) || n < 1 || t < 1 || 2 * t + 1 > n)
    return lsp::set_error(LSP_EINVAL, "invalid d, n or t");
  const int W = 2 * t + 1;
  int m = 1;
  int64_t N = 1;
  for (int i = 0; i < d; ++i) {
    m *= W;
    N *= n;
  }
  int64_t out = 0;
  for (int64_t j = 0; j < N; ++j) {
    int jc[3] = {0, 0, 0};
    int64_t rem = j;
    for (int i = d - 1; i >= 0; --i) {
      jc[i] = (int)(rem % n);
      rem /= n;
    }
    for (int a = 0; a < m; ++a) {
      int ra = a;
      int ac[3] = {0, 0, 0};
      for (int i = d - 1; i >= 0; --i) {
        ac[i] = ra % W - t;
        ra /= W;
      }
      int64_t col = 0;
      for (int i = 0; i < d; ++i) col = col * n + (((jc[i] + ac[i]) % n) + n) % n;
      col_host[out++] = col;
    }
  }
  return LSP_OK;
}

// ---------------------------------------------------------------------------
// GMRES(restart) with right preconditioner P^-1 C. Basis V and preconditioned
// vectors Z = P^-1 C V are kept on the device (flexible form, so the update
// x += Z y needs no second preconditioner application). Orthogonalisation is
// classical Gram-Schmidt applied twice; the small Hessenberg least-squares
// problem is updated with Givens rotations on the host.
// ---------------------------------------------------------------------------
int lsp_precond_solve(lsp_problem* p, const double* f_dev, double* u_dev, double rtol,
                      int restart, int maxit, lsp_host_solve_fn solveP, void* user, int* iters,
                      double* relres) {
  using cplx = std::complex<double>;
  if (!p || !f_dev || !u_dev || !solveP) return lsp::set_error(LSP_EINVAL, "NULL argument");
  if (!(rtol > 0.0) || restart < 1 || restart > 1000 || maxit < 1)
    return lsp::set_error(LSP_EINVAL, "invalid rtol, restart or maxit");
  if (!p->have_setup) return lsp::set_error(LSP_ESTATE, "precond_solve needs a completed setup");
  const int64_t N = p->N;
  const int64_t N2 = 2 * N;
  int rc = check_setup_status(p);
  if (rc) return rc;
  rc = check_finite_device(p, f_dev, N2, "f");
  if (rc) return rc;
  // workspace: V (restart+1), Z (restart), w, tmp; coefficient buffer
  const size_t need = (size_t)N2 * (2 * (size_t)restart + 3) + 2 * (size_t)(restart + 2);
  if (need > p->kry_doubles) {
    (void)hipStreamSynchronize(p->stream);
    dfree(p->kry);
    if ((rc = dalloc((void**)&p->kry, sizeof(double) * need, "Krylov basis"))) return rc;
    p->kry_doubles = need;
    dfree(p->red);
    if (p->red_host) (void)hipHostFree(p->red_host);
    p->red_host = nullptr;
  }
  const int nblk = lsp::dot_blocks(N);
  const size_t red_doubles = 2 * (size_t)(restart + 2) * nblk;
  if (!p->red) {
    if ((rc = dalloc((void**)&p->red, sizeof(double) * red_doubles, "reduction"))) return rc;
    if (hipHostMalloc((void**)&p->red_host, sizeof(double) * (red_doubles + 4 * (size_t)N),
                      hipHostMallocDefault) != hipSuccess)
      return lsp::set_error(LSP_ENOMEM, "pinned host allocation failed");
  }
  double* V = p->kry;
  double* Z = V + (size_t)N2 * (restart + 1);
  double* w = Z + (size_t)N2 * restart;
  double* tmp = w + N2;
  double* coef = tmp + N2;
  double* hbuf = p->red_host;                  // reduction results
  double* rhs_h = p->red_host + red_doubles;   // P-solve right-hand side
  double* x_h = rhs_h + N2;                    // P-solve solution
  hipStream_t s = p->stream;

#define LSP_HIP(call, what)                                     \
  do {                                                          \
    hipError_t e_ = (call);                                     \
    if (e_ != hipSuccess) return lsp::hip_check(e_, what);      \
  } while (0)

  // dots: out[i] = <V_i, x> for i < nv, summed in block order on the host
  auto dots = [&](const double* Vb, int nv, const double* x, cplx* out) -> int {
    LSP_HIP(lsp::launch_multi_dot(Vb, N, nv, x, N, p->red, s), "dot");
    LSP_HIP(hipMemcpyAsync(hbuf, p->red, sizeof(double) * 2 * nv * nblk, hipMemcpyDeviceToHost,
                           s),
            "dot readback");
    LSP_HIP(hipStreamSynchronize(s), "dot sync");
    for (int i = 0; i < nv; ++i) {
      double re = 0.0, im = 0.0;
      for (int b = 0; b < nblk; ++b) {
        re += hbuf[2 * ((size_t)i * nblk + b)];
        im += hbuf[2 * ((size_t)i * nblk + b) + 1];
      }
      out[i] = cplx(re, im);
    }
    return LSP_OK;
  };
  auto axpy = [&](const double* Vb, int nv, const cplx* c, double sign, double* x) -> int {
    LSP_HIP(hipMemcpyAsync(coef, c, sizeof(double) * 2 * nv, hipMemcpyHostToDevice, s),
            "coefficient upload");
    LSP_HIP(lsp::launch_multi_axpy(Vb, N, nv, coef, sign, x, N, s), "axpy");
    LSP_HIP(hipStreamSynchronize(s), "axpy sync");  // coef is host memory read by the copy
    return LSP_OK;
  };

  cplx fn2;
  if ((rc = dots(f_dev, 1, f_dev, &fn2))) return rc;
  const double fnorm = sqrt(fn2.real());
  LSP_HIP(hipMemsetAsync(u_dev, 0, sizeof(double) * N2, s), "zero u");
  int it = 0;
  double est = 1.0;
  if (fnorm == 0.0) {
    if (iters) *iters = 0;
    if (relres) *relres = 0.0;
    return LSP_OK;
  }
  std::vector<cplx> H((size_t)(restart + 1) * restart), cs(restart), sn(restart), g(restart + 1),
      h(restart + 1), h2(restart + 1), y(restart);
  bool first = true;
  while (it < maxit) {
    // r = f - A u
    if (first) {
      LSP_HIP(hipMemcpyAsync(V, f_dev, sizeof(double) * N2, hipMemcpyDeviceToDevice, s), "copy f");
    } else {
      LSP_HIP(lsp::launch_ps_apply(p, u_dev, tmp), "apply");
      LSP_HIP(lsp::launch_sub(f_dev, tmp, V, N, s), "residual");
    }
    first = false;
    cplx b2;
    if ((rc = dots(V, 1, V, &b2))) return rc;
    const double beta = sqrt(b2.real());
    est = beta / fnorm;
    if (est <= rtol) break;
    LSP_HIP(lsp::launch_scale(V, 1.0 / beta, V, N, s), "normalise");
    std::fill(H.begin(), H.end(), cplx(0.0));
    std::fill(g.begin(), g.end(), cplx(0.0));
    g[0] = beta;
    int k_used = 0;
    for (int k = 0; k < restart; ++k) {
      double* vk = V + (size_t)N2 * k;
      double* zk = Z + (size_t)N2 * k;
      // z_k = P^-1 (C v_k): C on the device, the P-solve on the host
      LSP_HIP(lsp::launch_c_apply(p, vk, tmp), "c_apply");
      LSP_HIP(hipMemcpyAsync(rhs_h, tmp, sizeof(double) * N2, hipMemcpyDeviceToHost, s), "D2H");
      LSP_HIP(hipStreamSynchronize(s), "D2H sync");
      if (solveP(user, rhs_h, x_h, N) != 0)
        return lsp::set_error(LSP_ESOLVER, "host P-solve callback returned an error");
      LSP_HIP(hipMemcpyAsync(zk, x_h, sizeof(double) * N2, hipMemcpyHostToDevice, s), "H2D");
      // w = A z_k
      LSP_HIP(lsp::launch_ps_apply(p, zk, w), "apply");
      // classical Gram-Schmidt, twice
      if ((rc = dots(V, k + 1, w, h.data()))) return rc;
      if ((rc = axpy(V, k + 1, h.data(), -1.0, w))) return rc;
      if ((rc = dots(V, k + 1, w, h2.data()))) return rc;
      if ((rc = axpy(V, k + 1, h2.data(), -1.0, w))) return rc;
      for (int i = 0; i <= k; ++i) h[i] += h2[i];
      cplx wn2;
      if ((rc = dots(w, 1, w, &wn2))) return rc;
      const double hk1 = sqrt(wn2.real());
      if (hk1 > 0.0) {
        LSP_HIP(lsp::launch_scale(w, 1.0 / hk1, V + (size_t)N2 * (k + 1), N, s), "normalise");
      }
      // apply previous rotations to column k
      for (int i = 0; i < k; ++i) {
        const cplx t0 = std::conj(cs[i]) * h[i] + std::conj(sn[i]) * h[i + 1];
        h[i + 1] = -sn[i] * h[i] + cs[i] * h[i + 1];
        h[i] = t0;
      }
      const cplx a = h[k];
      const double bb = hk1;
      const double rho = hypot(std::abs(a), bb);
      cs[k] = rho > 0.0 ? a / rho : cplx(1.0);
      sn[k] = rho > 0.0 ? cplx(bb / rho) : cplx(0.0);
      h[k] = rho;
      for (int i = 0; i <= k; ++i) H[(size_t)i * restart + k] = h[i];
      g[k + 1] = -sn[k] * g[k];
      g[k] = std::conj(cs[k]) * g[k];
      ++it;
      k_used = k + 1;
      est = std::abs(g[k + 1]) / fnorm;
      if (est <= rtol || it >= maxit || hk1 == 0.0) break;
    }
    // y = H^-1 g (upper triangular), u += Z y
    for (int i = k_used - 1; i >= 0; --i) {
      cplx acc = g[i];
      for (int j = i + 1; j < k_used; ++j) acc -= H[(size_t)i * restart + j] * y[j];
      y[i] = acc / H[(size_t)i * restart + i];
    }
    if ((rc = axpy(Z, k_used, y.data(), 1.0, u_dev))) return rc;
    if (est <= rtol) break;
  }
  // true residual
  LSP_HIP(lsp::launch_ps_apply(p, u_dev, tmp), "apply");
  LSP_HIP(lsp::launch_sub(f_dev, tmp, w, N, s), "residual");
  cplx r2;
  if ((rc = dots(w, 1, w, &r2))) return rc;
  if (iters) *iters = it;
  if (relres) *relres = sqrt(r2.real()) / fnorm;
#undef LSP_HIP
  return (est <= rtol) ? LSP_OK : LSP_NOT_CONVERGED;
}

int lsp_precond_solve_device(lsp_problem* p, const double* f_dev, double* u_dev, double rtol,
                             int restart, int maxit, int* iters, double* relres) {
  if (!p || !f_dev || !u_dev) return lsp::set_error(LSP_EINVAL, "NULL argument");
  if (f_dev == u_dev) return lsp::set_error(LSP_EINVAL, "f and u must not alias");
  if (!(rtol > 0.0) || restart < 1 || restart > 1000 || maxit < 1)
    return lsp::set_error(LSP_EINVAL, "invalid rtol, restart or maxit");
  if (!p->have_setup) return lsp::set_error(LSP_ESTATE, "precond_solve needs a completed setup");
  if (!p->nd.ready) return lsp::set_error(LSP_ESTATE, "no P factors uploaded (lsp_psolve_upload)");
  const int64_t N = p->N;
  const int64_t N2 = 2 * N;
  int rc = check_setup_status(p);
  if (rc) return rc;
  rc = check_finite_device(p, f_dev, N2, "f");
  if (rc) return rc;
  const int nblk = lsp::dot_blocks(N);
  const size_t R = (size_t)restart;
  const size_t need = (size_t)N2 * (2 * R + 3) + 2 * (R + 1) * nblk + 2 * (R + 1) * 2 +
                      2 * R * R + 2 * R * 2 + 2 * (R + 1) + 2 * R + lsp::kScCount;
  hipStream_t s = p->stream;
  if (need > p->dk_doubles) {
    (void)hipStreamSynchronize(s);
    lsp::free_device_gmres(p);
    if ((rc = dalloc((void**)&p->dk, sizeof(double) * need, "device GMRES workspace"))) return rc;
    p->dk_doubles = need;
  }
  if (!p->dk_host &&
      hipHostMalloc((void**)&p->dk_host, sizeof(double) * lsp::kScCount, hipHostMallocDefault) !=
          hipSuccess) {
    p->dk_host = nullptr;
    return lsp::set_error(LSP_ENOMEM, "pinned host allocation failed");
  }
  double* V = p->dk;
  double* Z = V + (size_t)N2 * (R + 1);
  double* w = Z + (size_t)N2 * R;
  double* tmp = w + N2;
  double* part = tmp + N2;
  double* hA = part + 2 * (R + 1) * nblk;
  double* hB = hA + 2 * (R + 1);
  double* H = hB + 2 * (R + 1);
  double* cs = H + 2 * R * R;
  double* sn = cs + 2 * R;
  double* g = sn + 2 * R;
  double* y = g + 2 * (R + 1);
  double* sc = y + 2 * R;
  double* sc_h = p->dk_host;

#define LSP_HIP(call, what)                                \
  do {                                                     \
    hipError_t e_ = (call);                                \
    if (e_ != hipSuccess) return lsp::hip_check(e_, what); \
  } while (0)

  // the scalars of the last step, read back on the host
  auto read_scalars = [&]() -> int {
    LSP_HIP(hipMemcpyAsync(sc_h, sc, sizeof(double) * lsp::kScCount, hipMemcpyDeviceToHost, s),
            "scalar readback");
    LSP_HIP(hipStreamSynchronize(s), "scalar sync");
    return LSP_OK;
  };
  // one Arnoldi step at column k: z_k = P^-1 C v_k, w = A z_k, two passes of
  // classical Gram-Schmidt against v_0..v_k, the Givens update of column k
  // and v_{k+1} = w / ||w||
  auto step = [&](int k) -> hipError_t {
    double* vk = V + (size_t)N2 * k;
    double* zk = Z + (size_t)N2 * k;
    hipError_t e = lsp::launch_c_apply(p, vk, tmp);
    if (e == hipSuccess) e = lsp::launch_psolve(p, tmp, zk, s);
    if (e == hipSuccess) e = lsp::launch_ps_apply(p, zk, w, s);
    if (e == hipSuccess) e = lsp::launch_multi_dot(V, N, k + 1, w, N, part, s);
    if (e == hipSuccess) e = lsp::launch_reduce_parts(part, nblk, k + 1, hA, s);
    if (e == hipSuccess) e = lsp::launch_multi_axpy(V, N, k + 1, hA, -1.0, w, N, s);
    if (e == hipSuccess) e = lsp::launch_multi_dot(V, N, k + 1, w, N, part, s);
    if (e == hipSuccess) e = lsp::launch_reduce_parts(part, nblk, k + 1, hB, s);
    if (e == hipSuccess) e = lsp::launch_multi_axpy(V, N, k + 1, hB, -1.0, w, N, s);
    if (e == hipSuccess) e = lsp::launch_multi_dot(w, N, 1, w, N, part, s);
    if (e == hipSuccess)
      e = lsp::launch_givens(part, nblk, hA, hB, H, cs, sn, g, sc, k, restart, s);
    if (e == hipSuccess) e = lsp::launch_scale_dev(w, sc + lsp::kScInv, V + (size_t)N2 * (k + 1), N, s);
    return e;
  };
  // the step through a graph captured once per column (kept while the
  // workspaces, the setup's radius and kind and the factors are unchanged)
  const bool graphs = p->krylov_graphs && s != nullptr;
  if ((int)p->g_arnoldi.size() < restart) p->g_arnoldi.resize(restart);
  auto run_step = [&](int k) -> hipError_t {
    if (!graphs) return step(k);
    lsp_problem::GraphCache& gc = p->g_arnoldi[k];
    const uint64_t key[6] = {(uint64_t)(uintptr_t)p->dk, p->ws_gen,
                             (uint64_t)restart | ((uint64_t)k << 20),
                             (uint64_t)p->t | ((uint64_t)p->learned << 8) |
                                 ((uint64_t)p->nd_leaf << 9),
                             (uint64_t)(uintptr_t)p->c_rows ^ (uint64_t)(uintptr_t)p->nd1.C,
                             (uint64_t)(uintptr_t)p->nd.data};
    bool same = gc.valid;
    for (int i = 0; i < 6 && same; ++i) same = (gc.key[i] == key[i]);
    if (!same) {
      if (gc.exec) (void)hipGraphExecDestroy(gc.exec);
      gc.exec = nullptr;
      gc.valid = false;
      hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) return e;
      const hipError_t le = step(k);
      hipGraph_t graph = nullptr;
      e = hipStreamEndCapture(s, &graph);
      if (le != hipSuccess || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return le != hipSuccess ? le : e;
      }
      e = hipGraphInstantiate(&gc.exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (e != hipSuccess) {
        gc.exec = nullptr;
        return e;
      }
      for (int i = 0; i < 6; ++i) gc.key[i] = key[i];
      gc.valid = true;
    }
    return hipGraphLaunch(gc.exec, s);
  };

  // ||f||
  LSP_HIP(lsp::launch_multi_dot(f_dev, N, 1, f_dev, N, part, s), "dot");
  LSP_HIP(lsp::launch_krylov_norm(part, nblk, 0, restart, sc, g, s), "norm");
  LSP_HIP(hipMemsetAsync(u_dev, 0, sizeof(double) * N2, s), "zero u");
  if ((rc = read_scalars())) return rc;
  const double fnorm = sc_h[lsp::kScFnorm];
  if (fnorm == 0.0) {
    if (iters) *iters = 0;
    if (relres) *relres = 0.0;
    return LSP_OK;
  }
  int it = 0;
  double est = 1.0;
  bool first = true;
  while (it < maxit) {
    // r = f - A u, beta = ||r||, v_0 = r / beta
    if (first) {
      LSP_HIP(hipMemcpyAsync(tmp, f_dev, sizeof(double) * N2, hipMemcpyDeviceToDevice, s), "copy f");
    } else {
      LSP_HIP(lsp::launch_ps_apply(p, u_dev, w, s), "apply");
      LSP_HIP(lsp::launch_sub(f_dev, w, tmp, N, s), "residual");
    }
    first = false;
    LSP_HIP(lsp::launch_multi_dot(tmp, N, 1, tmp, N, part, s), "dot");
    LSP_HIP(lsp::launch_krylov_norm(part, nblk, 1, restart, sc, g, s), "cycle start");
    LSP_HIP(lsp::launch_scale_dev(tmp, sc + lsp::kScInv, V, N, s), "normalise");
    if ((rc = read_scalars())) return rc;
    est = sc_h[lsp::kScEst];
    if (est <= rtol) break;
    int k_used = 0;
    for (int k = 0; k < restart; ++k) {
      const int tk = lsp::stage_begin(p, LSP_STAGE_ARNOLDI);
      LSP_HIP(run_step(k), "Arnoldi step");
      lsp::stage_end(p, tk);
      if ((rc = read_scalars())) return rc;
      ++it;
      k_used = k + 1;
      est = sc_h[lsp::kScEst];
      if (est <= rtol || it >= maxit || sc_h[lsp::kScBreak] != 0.0) break;
    }
    // u += Z y with y = H^-1 g
    LSP_HIP(lsp::launch_trisolve(H, g, k_used, restart, y, s), "triangular solve");
    LSP_HIP(lsp::launch_multi_axpy(Z, N, k_used, y, 1.0, u_dev, N, s), "update");
    if (est <= rtol) break;
  }
  // true residual
  LSP_HIP(lsp::launch_ps_apply(p, u_dev, tmp, s), "apply");
  LSP_HIP(lsp::launch_sub(f_dev, tmp, w, N, s), "residual");
  LSP_HIP(lsp::launch_multi_dot(w, N, 1, w, N, part, s), "dot");
  LSP_HIP(lsp::launch_krylov_norm(part, nblk, 1, restart, sc, g, s), "residual norm");
  if ((rc = read_scalars())) return rc;
  if (iters) *iters = it;
  if (relres) *relres = sc_h[lsp::kScBeta] / fnorm;
#undef LSP_HIP
  return (est <= rtol) ? LSP_OK : LSP_NOT_CONVERGED;
}

}  // extern "C"
