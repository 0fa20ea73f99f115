// Batched form: many independent problems of uneven n set up and applied
// together. Each setup stage (min/max partials, Green's sums, Gram matrices
// and null vectors, per-point rows) is ONE launch over the (problem, block)
// work items of all problems, so small problems share the GPU instead of
// each taking a launch sequence of its own. The four launches are captured
// once into a HIP graph and replayed while the arguments are unchanged, and
// the batched pseudospectral apply is one graph over every problem's apply,
// the problems as parallel branches (LSP_GRAPHS=0 launches directly, one
// problem after another). The tables and rows each problem receives are those of its own
// single-problem setup (same kernels, same arithmetic), so every per-problem
// entry point (C-apply, GMRES, table export) works on them afterwards.
//
// The assembly tile width is chosen per batch by timing the candidate widths
// that divide every n of the batch, and in 2D the LDS-table form (8 x 64
// tiles, the shift tables copied into LDS; "width" 1) where every problem's
// tables fit (the first setup of a batch, and again whenever its sizes or
// shift counts change).
#include "lsp_internal.h"

#include <algorithm>
#include <functional>
#include <vector>

struct lsp_batch {
  std::vector<lsp_problem*> probs;
  int d = 0;
  hipStream_t stream = nullptr;
  // device records and block maps of the current arguments
  lsp::BatchRec* recs = nullptr;
  size_t recs_cap = 0;
  int4* maps = nullptr;
  size_t maps_cap = 0;
  int off_mm = 0, n_mm = 0, off_green = 0, n_green = 0, off_null = 0, n_null = 0;
  int off_asm = 0, n_asm = 0;
  std::vector<uint64_t> rec_key;  // arguments the records were built for
  // assembly tile width chosen by the tuner, for the sizes (and t, precision)
  // it was tuned on
  int tw = 0;
  std::vector<int> tuned_key;
  int forced_tw = 0;       // lsp_batch_set_tile: 0 = tune, else this width
  bool tw_forced = false;  // the current tw came from forced_tw
  int tw_candidates[4] = {0, 0, 0, 0};
  float tw_ms[4] = {0, 0, 0, 0};
  // graphs
  hipGraphExec_t g_setup = nullptr;
  std::vector<uint64_t> setup_key;
  hipGraphExec_t g_apply = nullptr;
  std::vector<uint64_t> apply_key;
  bool use_graphs = true;
  // the captured apply forks onto these streams, so that independent
  // problems become parallel branches of its graph (default priority)
  static constexpr int kBranches = 8;
  hipStream_t aux[kBranches] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t join[kBranches] = {};
  bool branches = false;
};

namespace {

constexpr int kTileWidths[4] = {16, 32, 64, 128};

void drop(hipGraphExec_t& g) {
  if (g) (void)hipGraphExecDestroy(g);
  g = nullptr;
}

template <typename T>
int grow(T** ptr, size_t* cap, size_t need, const char* what) {
  if (*cap >= need) return LSP_OK;
  if (*ptr) (void)hipFree(*ptr);
  *ptr = nullptr;
  *cap = 0;
  if (hipMalloc((void**)ptr, sizeof(T) * need) != hipSuccess)
    return lsp::set_error(LSP_ENOMEM, std::string("device allocation failed: ") + what);
  *cap = need;
  return LSP_OK;
}

// Replay the graph of `launch` when key matches, else capture it anew; launch
// directly on the legacy default stream or when capture is unavailable.
hipError_t run_batch_graph(lsp_batch* b, hipGraphExec_t& g, std::vector<uint64_t>& gkey,
                           const std::vector<uint64_t>& key,
                           const std::function<hipError_t()>& launch) {
  if (!b->use_graphs || b->stream == nullptr) return launch();
  if (!(g && gkey == key)) {
    drop(g);
    hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      b->use_graphs = false;
      return launch();
    }
    const hipError_t le = launch();
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(b->stream, &graph);
    if (le != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return le;
    }
    if (e != hipSuccess) return e;
    e = hipGraphInstantiate(&g, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      g = nullptr;
      return e;
    }
    gkey = key;
  }
  return hipGraphLaunch(g, b->stream);
}

// Block maps of the four stages for assembly tile width tw.
void build_maps(const lsp_batch* b, const std::vector<int>& nreq, int tw,
                std::vector<int4>& mm, std::vector<int4>& green, std::vector<int4>& null,
                std::vector<int4>& asmb) {
  mm.clear();
  green.clear();
  null.clear();
  asmb.clear();
  for (int i = 0; i < (int)b->probs.size(); ++i) {
    const lsp_problem* p = b->probs[i];
    for (int bx = 0; bx < lsp::kMinMaxBlocks; ++bx) mm.push_back(make_int4(i, bx, 0, 0));
    if (b->d == 2) {
      // the balanced Green's launch of the problem: its waves in blocks of 4
      const int blocks = lsp::green2d_waves(p->n, nreq[i]) / 4;
      for (int bx = 0; bx < blocks; ++bx) green.push_back(make_int4(i, bx, 0, 0));
    } else {
      const int groups = lsp::green_shift_groups(nreq[i]);
      for (int by = 0; by < groups; ++by)
        for (int bx = 0; bx < p->green_nunits; ++bx) green.push_back(make_int4(i, bx, by, 0));
    }
    for (int si = 0; si < nreq[i]; ++si) null.push_back(make_int4(i, si, 0, 0));
    if (tw == lsp::kBatchLdsTile) {
      // 2D tiles of 8 rows x 64 points (the LDS-table form)
      for (int by = 0; by < p->n / 8; ++by)
        for (int bx = 0; bx < p->n / 64; ++bx) asmb.push_back(make_int4(i, bx, by, 0));
      continue;
    }
    const int planes = (b->d == 3) ? p->n : 1;
    for (int bz = 0; bz < planes; ++bz)
      for (int by = 0; by < p->n; ++by)
        for (int bx = 0; bx < p->n / tw; ++bx) asmb.push_back(make_int4(i, bx, by, bz));
  }
}

int upload_maps(lsp_batch* b, const std::vector<int>& nreq, int tw) {
  std::vector<int4> mm, green, null, asmb;
  build_maps(b, nreq, tw, mm, green, null, asmb);
  b->off_mm = 0;
  b->n_mm = (int)mm.size();
  b->off_green = b->off_mm + b->n_mm;
  b->n_green = (int)green.size();
  b->off_null = b->off_green + b->n_green;
  b->n_null = (int)null.size();
  b->off_asm = b->off_null + b->n_null;
  b->n_asm = (int)asmb.size();
  std::vector<int4> all;
  all.reserve(b->off_asm + b->n_asm);
  all.insert(all.end(), mm.begin(), mm.end());
  all.insert(all.end(), green.begin(), green.end());
  all.insert(all.end(), null.begin(), null.end());
  all.insert(all.end(), asmb.begin(), asmb.end());
  int rc = grow(&b->maps, &b->maps_cap, all.size(), "batch block maps");
  if (rc) return rc;
  (void)hipStreamSynchronize(b->stream);
  if (hipMemcpy(b->maps, all.data(), sizeof(int4) * all.size(), hipMemcpyHostToDevice) !=
      hipSuccess)
    return lsp::set_error(LSP_EHIP, "upload of the batch block maps failed");
  return LSP_OK;
}

hipError_t launch_stages(const lsp_batch* b, int t, bool fp32, int tw) {
  hipError_t e = lsp::launch_minmax_batched(b->recs, b->maps + b->off_mm, b->n_mm,
                                            (int)b->probs.size(), b->stream);
  if (e == hipSuccess)
    e = lsp::launch_green_batched(b->d, t, b->recs, b->maps + b->off_green, b->n_green,
                                  b->stream);
  if (e == hipSuccess)
    e = lsp::launch_null_batched(b->d, t, b->recs, b->maps + b->off_null, b->n_null, b->stream);
  if (e == hipSuccess)
    e = lsp::launch_assemble_batched(b->d, t, tw, fp32, b->recs, b->maps + b->off_asm, b->n_asm,
                                     b->stream);
  return e;
}

}  // namespace

extern "C" {

int lsp_batch_create(int count, lsp_problem* const* problems, lsp_batch** out) {
  if (!out) return lsp::set_error(LSP_EINVAL, "out is NULL");
  *out = nullptr;
  if (count < 1 || !problems) return lsp::set_error(LSP_EINVAL, "count >= 1 problems needed");
  lsp_batch* b = new lsp_batch();
  for (int i = 0; i < count; ++i) {
    lsp_problem* p = problems[i];
    if (!p) {
      delete b;
      return lsp::set_error(LSP_EINVAL, "problem " + std::to_string(i) + " is NULL");
    }
    if (i > 0 && (p->d != b->d || p->stream != b->stream || p->device != b->probs[0]->device)) {
      delete b;
      return lsp::set_error(LSP_EINVAL,
                            "the problems of a batch share d, the HIP stream and the device");
    }
    if (p->n < 16) {
      delete b;
      return lsp::set_error(LSP_EINVAL, "batched problems need n >= 16");
    }
    b->d = p->d;
    b->stream = p->stream;
    b->probs.push_back(p);
  }
  // graph replay on by default here: the four batched launches take 0.33-0.35 ms
  // as a graph replay against 0.43 ms launched directly (64-problem workload)
  b->use_graphs = lsp::graphs_enabled(true);
  if (b->use_graphs && b->stream) {
    // on the problems' device, whichever device is current
    int cur = -1;
    bool ok = hipGetDevice(&cur) == hipSuccess;
    const int dev = b->probs[0]->device;
    if (ok && cur != dev) ok = hipSetDevice(dev) == hipSuccess;
    if (ok) ok = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) == hipSuccess;
    for (int k = 0; ok && k < lsp_batch::kBranches; ++k)
      ok = hipStreamCreateWithFlags(&b->aux[k], hipStreamNonBlocking) == hipSuccess &&
           hipEventCreateWithFlags(&b->join[k], hipEventDisableTiming) == hipSuccess;
    if (cur >= 0 && cur != dev) (void)hipSetDevice(cur);
    b->branches = ok;  // without them the captured apply stays one chain
    if (!ok) (void)hipGetLastError();
  }
  *out = b;
  return LSP_OK;
}

void lsp_batch_destroy(lsp_batch* b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->stream);
  drop(b->g_setup);
  drop(b->g_apply);
  for (int k = 0; k < lsp_batch::kBranches; ++k) {
    if (b->aux[k]) (void)hipStreamDestroy(b->aux[k]);
    if (b->join[k]) (void)hipEventDestroy(b->join[k]);
  }
  if (b->fork) (void)hipEventDestroy(b->fork);
  if (b->recs) (void)hipFree(b->recs);
  if (b->maps) (void)hipFree(b->maps);
  delete b;
}

int lsp_batch_stencil_setup(lsp_batch* b, int t, const int* num_shifts, int precision,
                            void* const* P_dev, int32_t* const* idx_dev) {
  if (!b || !P_dev) return lsp::set_error(LSP_EINVAL, "NULL argument");
  if (precision != LSP_FP64 && precision != LSP_FP32_REFINE)
    return lsp::set_error(LSP_EINVAL, "unsupported precision");
  const int count = (int)b->probs.size();
  std::vector<int> nreq(count);
  for (int i = 0; i < count; ++i) {
    if (!P_dev[i]) return lsp::set_error(LSP_EINVAL, "P_dev[" + std::to_string(i) + "] is NULL");
    nreq[i] = num_shifts ? num_shifts[i] : 0;
    if (b->probs[i]->d == 3 && t != 1)
      return lsp::set_error(LSP_EINVAL, "batched setups support d = 3 with t = 1");
    const int rc = lsp::prepare_setup(b->probs[i], t, &nreq[i]);
    if (rc) return rc;
  }
  const bool fp32 = precision == LSP_FP32_REFINE;
  // records of the current arguments
  std::vector<uint64_t> key = {(uint64_t)t, (uint64_t)precision};
  std::vector<int> sizes = {t, precision};
  for (int i = 0; i < count; ++i) {
    const lsp_problem* p = b->probs[i];
    key.push_back((uint64_t)(uintptr_t)P_dev[i]);
    key.push_back((uint64_t)(uintptr_t)(idx_dev ? idx_dev[i] : nullptr));
    key.push_back(p->ws_gen);
    key.push_back((uint64_t)nreq[i]);
    sizes.push_back(p->n);
    sizes.push_back(nreq[i]);
  }
  int rc = LSP_OK;
  if (key != b->rec_key) {
    std::vector<lsp::BatchRec> recs(count);
    for (int i = 0; i < count; ++i) {
      const lsp_problem* p = b->probs[i];
      lsp::BatchRec& r = recs[i];
      r.v = p->v;
      r.n = p->n;
      r.nreq = nreq[i];
      r.N = p->N;
      r.invN = 1.0 / (double)p->N;
      r.mm_part = p->ws.minmax_part;
      r.S = p->ws.S;
      r.nS = p->ws.nS;
      r.vrange = p->ws.vrange;
      r.cw = p->cosT;
      r.units = p->green_units;
      r.nunits = p->green_nunits;
      r.gwaves = (p->d == 2) ? lsp::green2d_waves(p->n, nreq[i]) : 0;
      r.sps = (p->d == 2) ? lsp::green2d_sps(p->n) : 0;
      r.part = p->ws.green_part;
      r.gtab = p->ws.gtab;
      r.gamtab = p->ws.gamtab;
      r.Mtab = p->ws.Mtab;
      r.alpha = p->ws.alpha;
      r.Ctab = p->ws.Ctab;
      r.sigma = p->ws.sigma;
      r.rho = p->ws.rho;
      r.actab = p->ws.actab;
      r.status = p->ws.status;
      r.P = P_dev[i];
      r.idx = idx_dev ? idx_dev[i] : nullptr;
    }
    if ((rc = grow(&b->recs, &b->recs_cap, (size_t)count, "batch records"))) return rc;
    (void)hipStreamSynchronize(b->stream);
    if (hipMemcpy(b->recs, recs.data(), sizeof(lsp::BatchRec) * count, hipMemcpyHostToDevice) !=
        hipSuccess)
      return lsp::set_error(LSP_EHIP, "upload of the batch records failed");
    b->rec_key = key;
    drop(b->g_setup);
  }
  hipError_t e = hipSuccess;
  const int64_t m_rows = (int64_t)(2 * t + 1) * (2 * t + 1);
  // the LDS-table form (2D, 8 x 64 tiles) where every problem's shift tables fit
  bool lds_ok = b->d == 2;
  for (int i = 0; i < count; ++i)
    lds_ok = lds_ok && b->probs[i]->n % 64 == 0 && (int64_t)nreq[i] * m_rows <= lsp::kBatchActLds;
  if (b->forced_tw) {
    // a width set by the caller: checked against this batch, no tuning
    const int w = b->forced_tw;
    bool ok = (w == lsp::kBatchLdsTile) ? lds_ok : true;
    if (w != lsp::kBatchLdsTile)
      for (const lsp_problem* p : b->probs) ok = ok && (p->n % w == 0);
    if (!ok)
      return lsp::set_error(LSP_EINVAL, "the assembly tile width set for this batch does not "
                                        "fit its sizes or shift tables");
    if (!b->tw_forced || b->tw != w || sizes != b->tuned_key || b->n_asm == 0 ||
        b->setup_key.empty() || key != b->setup_key) {
      b->tw = w;
      b->tw_forced = true;
      b->tuned_key = sizes;
      for (int c = 0; c < 4; ++c) {
        b->tw_candidates[c] = (c == 0) ? w : 0;
        b->tw_ms[c] = 0.f;
      }
      if ((rc = upload_maps(b, nreq, w))) return rc;
      drop(b->g_setup);
    }
  } else if (b->tw == 0 || b->tw_forced || sizes != b->tuned_key) {
    b->tw_forced = false;
    // tune the assembly tile width: one full setup, then each candidate width
    // that divides every n (the rows it writes are the same for every width)
    int ncand = 0;
    int cand[5] = {0, 0, 0, 0, 0};
    for (int w : kTileWidths) {
      bool ok = true;
      for (const lsp_problem* p : b->probs) ok = ok && (p->n % w == 0);
      if (ok) cand[ncand++] = w;
    }
    // the LDS-table form where it fits; with four widths as well, the
    // smallest width gives way
    if (lds_ok) {
      if (ncand == 4) {
        for (int c = 0; c < 3; ++c) cand[c] = cand[c + 1];
        ncand = 3;
      }
      cand[ncand++] = lsp::kBatchLdsTile;
    }
    for (int c = 0; c < 4; ++c) b->tw_candidates[c] = cand[c];
    if (ncand == 0) return lsp::set_error(LSP_EINVAL, "no assembly tile width divides every n");
    if ((rc = upload_maps(b, nreq, b->tw_candidates[ncand - 1]))) return rc;
    e = launch_stages(b, t, fp32, b->tw_candidates[ncand - 1]);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    int best = -1;
    for (int c = 0; c < ncand && e == hipSuccess; ++c) {
      const int w = b->tw_candidates[c];
      if ((rc = upload_maps(b, nreq, w))) break;
      constexpr int kReps = 3;
      e = lsp::launch_assemble_batched(b->d, t, w, fp32, b->recs, b->maps + b->off_asm,
                                       b->n_asm, b->stream);  // warm-up
      if (e == hipSuccess) e = hipEventRecord(e0, b->stream);
      for (int r = 0; r < kReps && e == hipSuccess; ++r)
        e = lsp::launch_assemble_batched(b->d, t, w, fp32, b->recs, b->maps + b->off_asm,
                                         b->n_asm, b->stream);
      if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      b->tw_ms[c] = ms / kReps;
      if (e == hipSuccess && (best < 0 || b->tw_ms[c] < b->tw_ms[best])) best = c;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (rc) return rc;
    if (e != hipSuccess) return lsp::hip_check(e, "assembly tile tuning");
    b->tw = b->tw_candidates[best];
    b->tuned_key = sizes;
    if ((rc = upload_maps(b, nreq, b->tw))) return rc;
    drop(b->g_setup);
  } else if (b->n_asm == 0 || b->setup_key.empty() || key != b->setup_key) {
    // new arguments: the block counts may change, so the graph is rebuilt
    if ((rc = upload_maps(b, nreq, b->tw))) return rc;
    drop(b->g_setup);
  }
  const int tw = b->tw;
  e = run_batch_graph(b, b->g_setup, b->setup_key, key,
                      [&]() { return launch_stages(b, t, fp32, tw); });
  if (e != hipSuccess) return lsp::hip_check(e, "batched setup launch");
  for (lsp_problem* p : b->probs) p->have_setup = true;
  return LSP_OK;
}

int lsp_batch_ps_apply(lsp_batch* b, const double* const* u_dev, double* const* y_dev) {
  if (!b || !u_dev || !y_dev) return lsp::set_error(LSP_EINVAL, "NULL argument");
  const int count = (int)b->probs.size();
  std::vector<uint64_t> key;
  for (int i = 0; i < count; ++i) {
    if (!u_dev[i] || !y_dev[i] || u_dev[i] == y_dev[i])
      return lsp::set_error(LSP_EINVAL, "apply " + std::to_string(i) +
                                            ": u and y must be non-NULL and distinct");
    key.push_back((uint64_t)(uintptr_t)u_dev[i]);
    key.push_back((uint64_t)(uintptr_t)y_dev[i]);
    key.push_back(b->probs[i]->ws_gen);
  }
  // the problems may run concurrently: an output may not be another's buffer
  for (int i = 0; i < count; ++i)
    for (int k = 0; k < count; ++k)
      if (k != i && (y_dev[i] == y_dev[k] || y_dev[i] == u_dev[k]))
        return lsp::set_error(LSP_EINVAL, "apply " + std::to_string(i) +
                                              ": y aliases a buffer of problem " +
                                              std::to_string(k));
  const hipError_t e = run_batch_graph(b, b->g_apply, b->apply_key, key, [&]() -> hipError_t {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    const bool capturing = b->branches && hipStreamIsCapturing(b->stream, &st) == hipSuccess &&
                           st == hipStreamCaptureStatusActive;
    if (!capturing) {  // direct launches: one chain on the batch's stream
      for (int i = 0; i < count; ++i) {
        const hipError_t le = lsp::launch_ps_apply(b->probs[i], u_dev[i], y_dev[i]);
        if (le != hipSuccess) return le;
      }
      return hipSuccess;
    }
    // fork: problem i on branch i mod kBranches (each problem has its own
    // workspace, so the branches share nothing); join every branch, also
    // after a failed launch, so that the capture ends cleanly
    hipError_t fe = hipEventRecord(b->fork, b->stream);
    for (int k = 0; fe == hipSuccess && k < lsp_batch::kBranches; ++k)
      fe = hipStreamWaitEvent(b->aux[k], b->fork, 0);
    hipError_t le = hipSuccess;
    for (int i = 0; fe == hipSuccess && le == hipSuccess && i < count; ++i)
      le = lsp::launch_ps_apply(b->probs[i], u_dev[i], y_dev[i],
                                b->aux[i % lsp_batch::kBranches]);
    for (int k = 0; k < lsp_batch::kBranches; ++k) {
      hipError_t je = hipEventRecord(b->join[k], b->aux[k]);
      if (je == hipSuccess) je = hipStreamWaitEvent(b->stream, b->join[k], 0);
      if (fe == hipSuccess) fe = je;
    }
    return fe != hipSuccess ? fe : le;
  });
  return lsp::hip_check(e, "batched ps_apply launch");
}

int lsp_batch_set_tile(lsp_batch* b, int tile_width) {
  if (!b) return lsp::set_error(LSP_EINVAL, "NULL argument");
  bool known = tile_width == 0 || tile_width == lsp::kBatchLdsTile;
  for (int w : kTileWidths) known = known || tile_width == w;
  if (!known) return lsp::set_error(LSP_EINVAL, "tile width must be 0, 1, 16, 32, 64 or 128");
  b->forced_tw = tile_width;
  return LSP_OK;
}

int lsp_batch_tile(const lsp_batch* b, int* tile_width, int* candidates, float* ms) {
  if (!b || !tile_width) return lsp::set_error(LSP_EINVAL, "NULL argument");
  *tile_width = b->tw;
  for (int c = 0; c < 4; ++c) {
    if (candidates) candidates[c] = b->tw_candidates[c];
    if (ms) ms[c] = b->tw_ms[c];
  }
  return LSP_OK;
}

}  // extern "C"
