// Internal declarations shared by the liblsp translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>
#include <string>
#include <vector>

#include "lsp.h"

namespace lsp {

// 4 pi^2: the symbol of -d^2/dx^2 on [0,1) is 4 pi^2 k^2 (Sec. 2).
constexpr double kFourPi2 = 39.47841760435743;
constexpr double kPi2 = 9.869604401089358;

// Upper bounds of the build.
constexpr int kMaxStencil = 125;    // m = (2t+1)^d
constexpr int kMaxShifts = 1024;    // requested |S|
constexpr int kMinMaxBlocks = 256;  // blocks (= partials) of the min/max reduction
constexpr int kActLds = 2048;       // (alpha, C) pairs the LDS-table assembly stages (32 KB)
constexpr int kBatchLdsTile = 1;    // batched assembly "tile width" of the LDS-table form
                                    // (8 rows x 64 points, 2D, nS m <= kBatchActLds)
constexpr int kBatchActLds = 1024;  // its table capacity in pairs (16 KB: more blocks per CU)

struct Workspace {
  // shift list (Sec. 4.1)
  double* minmax_part = nullptr;  // [2 * kMinMaxBlocks] (min, max), then [kMinMaxBlocks] sums
  double* S = nullptr;            // [kMaxShifts]
  int* nS = nullptr;              // effective |S|, device resident
  double* vrange = nullptr;       // [2] v_min, v_max
  // Green's kernel sums (Sec. 4.2)
  double* green_part = nullptr;   // [shifts][chunks][2 * W^d]
  size_t green_part_cap = 0;      // doubles
  // per-shift tables
  double* gtab = nullptr;         // [shifts][W^d]   W = 2t+1, offsets [0,2t]^d
  double* gamtab = nullptr;       // [shifts][W^d]
  double* Mtab = nullptr;         // [shifts][m*m]: packed parity blocks of M, then of A1, then of G
  double* alpha = nullptr;        // [shifts][m]
  double* Ctab = nullptr;         // [shifts][m]
  double* sigma = nullptr;        // [shifts]
  double* rho = nullptr;          // [shifts] rho*(s) of alpha_s (eq. A; the learned check)
  double* actab = nullptr;        // [shifts][m][2] interleaved (alpha, C)
  int* status = nullptr;          // [shifts] eigen-solver status
  int cap_shifts = 0;
  int cap_m = 0;
  int cap_w = 0;                  // W^d capacity
};

// One problem of a batched launch (device memory, plain pointers into the
// problem's own workspace): what the setup kernels of the problem take as
// arguments in a single-problem launch.
struct BatchRec {
  const double* v;
  int n;
  int nreq;          // requested |S|
  int64_t N;
  double invN;
  double* mm_part;   // min/max partials
  double* S;
  int* nS;
  double* vrange;
  const double* cw;  // folded cosine weights
  const int* units;  // Green's-sum work units (3D)
  int nunits;
  int gwaves;        // waves of the balanced 2D Green's launch (green2d_waves)
  int sps;           // its steps per shift (green2d_sps), 0 in 3D
  double* part;      // Green's partial sums
  double* gtab;
  double* gamtab;
  double* Mtab;
  double* alpha;
  double* Ctab;
  double* sigma;
  double* rho;
  double* actab;
  int* status;
  void* P;           // rows (float64 or float32)
  int32_t* idx;      // may be null
};

// per-point-radius setup: radius-1 tables (nS shifts, m1 = 3^d) formed from
// the radius-2 Green's pass
struct NdTables1 {
  double *gtab, *gamtab, *Mtab, *alpha, *C, *sigma, *rho;
  double2* actab;  // [nS][5^d] (alpha, C) pairs in the radius-2 layout, (0, 0) outside mu_0^1
  int* status;
};

// Device P-solve: nested-dissection factors of P uploaded by
// lsp_psolve_upload (front sizes, offsets, index lists, dense blocks), the
// product tasks of each level and the solve's buffers.
struct NDSolve {
  struct Level {
    int64_t row0 = 0, row1 = 0;   // rows of the level's fronts in the F lists
    int64_t front0 = 0;           // its fronts: front0 .. front0 + nfronts - 1
    int nfronts = 0;
    bool fused = false;           // one block per front, else split products
    bool staged = false;          // split: each block gathers r_F into LDS (else a gather launch)
    int64_t fmax = 0, umax = 0;   // largest f and u of the level
    int lanes_f = 8, lanes_b = 8; // lanes per row: forward (f columns), backward (f and u)
    // split levels: row tasks of the forward (f + u rows) and backward (f rows)
    int64_t fwd_task0 = 0, bwd_task0 = 0;
    int fwd_tasks = 0, bwd_tasks = 0;
  };
  int64_t *f = nullptr, *u = nullptr, *off_F = nullptr, *off_U = nullptr;
  int64_t *idx_F = nullptr, *idx_Fp = nullptr, *idx_U = nullptr, *off_blk = nullptr;
  int64_t *upd_ptr = nullptr, *slot = nullptr;  // updates of a point: slots upd_ptr[i]..upd_ptr[i+1]
  double* data = nullptr;
  int2* tasks = nullptr;           // (front, first row) of the split products
  double2 *R = nullptr, *Yc = nullptr, *W = nullptr;
  std::vector<Level> levels;
  bool ready = false;
};

}  // namespace lsp

struct lsp_problem {
  int d = 0;
  int n = 0;
  int64_t N = 0;
  hipStream_t stream = nullptr;
  int device = 0;
  int cus = 0;                // compute units of the device
  double* v = nullptr;        // [N] potential
  double* tw = nullptr;       // [2n] exp(-2 pi i j / n), interleaved
  double* cosT = nullptr;     // [cos_table_doubles(n, 2t+1)] folded cosine weights of the current t
  double* cos_by_t[4] = {nullptr, nullptr, nullptr, nullptr};  // tables kept per t = 1..3
  int* green_units = nullptr; // [green_nunits] Green's-sum work units
  int green_nunits = 0;
  double* z = nullptr;        // [2N] ps_apply partial sums
  int* flag = nullptr;        // [1] device scratch flag
  // setup state
  int t = 0;
  int m = 0;
  int num_shifts = 0;         // requested |S| of the last setup
  bool have_setup = false;
  // learned setup: per-point C rows [N][m] (the exact setup uses the per-shift
  // table instead); c_apply reads them while `learned` is set
  bool learned = false;
  // setup with per-point radius (Sec. 4.2): C rows are per point too
  int nd_leaf = 0;            // leaf box of a per-point-radius setup (0: none)
  double* c_rows = nullptr;
  size_t c_rows_cap = 0;      // doubles
  // radius-1 tables of that setup (one allocation, nd_t1_bytes, carved into nd1)
  char* nd_t1 = nullptr;
  size_t nd_t1_bytes = 0;
  lsp::NdTables1 nd1{};
  int nd1_shifts = 0;
  char* learn_buf = nullptr;  // rho*(s) per shift, fallback count, network in/out chunks
  size_t learn_cap = 0;       // bytes
  lsp::Workspace ws;
  // HIP graphs of the setup and apply launch sequences, replayed while the
  // arguments and workspaces they captured are unchanged
  struct GraphCache {
    hipGraphExec_t exec = nullptr;
    uint64_t key[6] = {0, 0, 0, 0, 0, 0};
    bool valid = false;
  };
  GraphCache g_setup, g_apply;
  uint64_t ws_gen = 1;        // bumped whenever a workspace pointer changes
  bool use_graphs = true;
  bool krylov_graphs = true;   // capture the Arnoldi step of the device GMRES
  // launch shapes chosen by lsp_autotune / lsp_set_tuning (0: the default)
  int tune[LSP_TUNE_COUNT] = {0, 0, 0};
  // per-stage event timing (lsp_profile)
  bool profiling = false;
  std::vector<hipEvent_t> ev_pool;                 // created events, reused
  std::vector<std::pair<int, int>> ev_pending;     // (stage, index of start event)
  size_t ev_used = 0;
  double prof_ms[LSP_NUM_STAGES] = {0};
  int prof_count[LSP_NUM_STAGES] = {0};
  // Krylov workspace (allocated on first precond_solve)
  double* kry = nullptr;      // basis and temporaries
  size_t kry_doubles = 0;
  double* red = nullptr;      // reduction partials
  double* red_host = nullptr; // pinned host mirror
  // device P-solve and device GMRES
  lsp::NDSolve nd;
  double* dk = nullptr;       // device GMRES: basis, Hessenberg state, partials
  size_t dk_doubles = 0;
  double* dk_host = nullptr;  // pinned: residual estimate and flags of the last step
  std::vector<GraphCache> g_arnoldi;  // one captured Arnoldi step per column k
};

namespace lsp {

int set_error(int code, const std::string& msg);
// Record a timing event pair around a stage when profiling is on:
// stage_begin returns a token passed to stage_end (-1 when off).
int stage_begin(lsp_problem* p, int stage);
void stage_end(lsp_problem* p, int token);
int hip_check(hipError_t e, const char* what);
// HIP-graph replay of launch sequences: LSP_GRAPHS=1 turns it on, 0 off,
// unset gives by_default (read at problem and batch creation)
bool graphs_enabled(bool by_default);
// validation, workspaces and cosine table before a setup of radius t;
// num_shifts (0 = default) is replaced by the effective request
int prepare_setup(lsp_problem* p, int t, int* num_shifts);

// ---- kernel launchers (asynchronous, on p->stream) ----
// ps_apply: y = (L + diag v) u
hipError_t launch_ps_apply(const lsp_problem* p, const double* u, double* y);
// the same on stream s (the problem's own workspace; s only orders the launches)
hipError_t launch_ps_apply(const lsp_problem* p, const double* u, double* y, hipStream_t s);
// count of non-finite entries of x[0..count) written to *flag (flag zeroed first)
hipError_t launch_count_nonfinite(const double* x, int64_t count, int* flag, hipStream_t s);
// stencil setup stages
// min/max partials of v for the shift list S (Sec. 4.1; global: also the
// per-block sums for the one shift of the non-localized method of Sec. 3)
// into ws.minmax_part; the Green's-sum launch that follows forms S from them.
// With cw non-null the same launch also writes the folded cosine table of
// (cos_n, cos_w).
hipError_t launch_minmax_parts(const double* v, int64_t N, const Workspace& ws, bool global,
                               hipStream_t s, int cos_n, int cos_w, double* cw);
hipError_t launch_minmax(lsp_problem* p, bool global = false);
// folded cosine table cw[k][dl] = w(k) cos(2 pi k dl / n), k in [0, n/2], dl in [0, W),
// followed by the same values halved and by k^2 (as doubles) for k in [0, n/2]
hipError_t launch_cos_table(int n, int W, double* cw, hipStream_t s);
__host__ __device__ inline int cos_table_doubles(int n, int W) { return (n / 2 + 1) * (2 * W + 1); }
// rows of per-point radius (Sec. 4.2, leaf box `leaf`, radius <= 2) from the
// radius-1 (alpha, C) pairs act1 (in the radius-2 layout, (0, 0) outside
// mu_0^1) and the radius-2 pairs of the workspace; writes P and idx
hipError_t launch_assemble_nd(lsp_problem* p, const double2* act1, int leaf, double* P,
                              int32_t* idx);
// Green's sums (num_shifts = requested |S|); every block of the launch forms
// the shift list from the min/max partials that launch_minmax left in the
// workspace and block 0 publishes it (ws.S, ws.nS, ws.vrange). global: the
// one shift of the non-localized method.
hipError_t launch_green_sums(lsp_problem* p, int num_shifts, bool global = false);
// waves of the balanced 2D Green's launch for (n, requested |S|) and its steps
// per shift; a function of the arguments only, shared by single and batched launches
// waves of the balanced 2D Green's launch; max_waves (a multiple of 4,
// <= 2048) caps the count, 0 = the default cap of 2048
int green2d_waves(int n, int num_shifts, int max_waves = 0);
int green2d_sps(int n);
// work units of the 3D Green's-sum launch for (d, n), packed (outer tile << 16) | k tile
void green_units(int d, int n, std::vector<int>& units);
// doubles of partial sums the Green's-sum launch writes for (d, n, t, shifts)
size_t green_partial_doubles(int d, int n, int t, int shifts);
// full m x m Gram matrix from the packed parity blocks (host)
int expand_gram_host(int d, int t, const double* packed, double* full);
// also clears *clear_counter (a kernel store, not a memset) when it is non-null
hipError_t launch_null_vectors(lsp_problem* p, int num_shifts, int* clear_counter = nullptr);
// one launch: the radius-2 tables into the workspace and the radius-1 tables
// into t1 (its (alpha, C) pairs in the radius-2 layout), both from the
// radius-2 Green's partial sums (p->t must be 2)
hipError_t launch_null_nd(lsp_problem* p, int num_shifts, const NdTables1& t1);
// P: float64 rows, or float32 rows when fp32
hipError_t launch_assemble(lsp_problem* p, void* P, bool fp32, int32_t* idx);
// batched launches: one launch per stage over the problems of a batch; map
// holds (problem, block coordinates) per block
// min/max partials of every problem of a batch (map: (problem, block) of
// each problem's kMinMaxBlocks blocks), then each problem's shift list
// (count problems, one block each)
hipError_t launch_minmax_batched(const BatchRec* recs, const int4* map, int blocks, int count,
                                 hipStream_t s);
hipError_t launch_green_batched(int d, int t, const BatchRec* recs, const int4* map, int blocks,
                                hipStream_t s);
int green_shift_groups(int num_shifts);  // shift groups (blocks) per work unit
hipError_t launch_null_batched(int d, int t, const BatchRec* recs, const int4* map, int blocks,
                               hipStream_t s);
hipError_t launch_assemble_batched(int d, int t, int tw, bool fp32, const BatchRec* recs,
                                   const int4* map, int blocks, hipStream_t s);
// preconditioner halves and Krylov helpers
hipError_t launch_c_apply(const lsp_problem* p, const double* r, double* z);
// ---- GMRES (krylov.hip); vectors complex128 ----
// part[i * dot_blocks(N) + b] = block b's share of <V_i, w>, i < nv
hipError_t launch_multi_dot(const double* V, int64_t ldv, int nv, const double* w, int64_t N,
                            double* part, hipStream_t s);
// w += sign * sum_i coef[i] V_i (coef: nv complex, device)
hipError_t launch_multi_axpy(const double* V, int64_t ldv, int nv, const double* coef,
                             double sign, double* w, int64_t N, hipStream_t s);
hipError_t launch_scale(const double* x, double a, double* y, int64_t N, hipStream_t s);
hipError_t launch_sub(const double* b, const double* x, double* y, int64_t N, hipStream_t s);
int dot_blocks(int64_t N);  // <= 256
// out[i] = sum_b part[i * nblk + b] for i < nv, in a fixed order
hipError_t launch_reduce_parts(const double* part, int nblk, int nv, double* out, hipStream_t s);
// slots of the device GMRES scalars
enum { kScFnorm = 0, kScEst = 1, kScInv = 2, kScBreak = 3, kScBeta = 4, kScCount = 8 };
// ||x|| from the partials of <x, x>: mode 0 stores ||f||; mode 1 starts a
// restart cycle (beta, g = beta e_1, estimate, scale 1/beta)
hipError_t launch_krylov_norm(const double* part, int nblk, int mode, int restart, double* sc,
                              double* g, hipStream_t s);
// Hessenberg column k from the two Gram-Schmidt passes and ||w||, rotated
hipError_t launch_givens(const double* part, int nblk, const double* hA, const double* hB,
                         double* H, double* cs, double* sn, double* g, double* sc, int k,
                         int restart, hipStream_t s);
hipError_t launch_trisolve(const double* H, const double* g, int k_used, int restart, double* y,
                           hipStream_t s);
hipError_t launch_scale_dev(const double* x, const double* a, double* y, int64_t N,
                            hipStream_t s);
// device P-solve z = P^-1 r from the uploaded factors (r, z: N complex)
hipError_t launch_psolve(const lsp_problem* p, const double* r, double* z, hipStream_t s);
void free_psolve(lsp_problem* p);
void free_device_gmres(lsp_problem* p);
// surrogate (mlp.hip)
// device pointers of a network's BF16 weights (padded layout: W1 [H][round16(n_in)],
// W2 [H][H], W3 [round16(n_out)][H]), FP32 biases and standardisation
// (mu_x, sd_x, mu_y, sd_y)
struct MlpView {
  int n_in, n_hidden, n_out;
  const unsigned short* W1;
  const unsigned short* W2;
  const unsigned short* W3;
  const float* b1;
  const float* b2;
  const float* b3;
  const float* norm;
};
MlpView mlp_view(const lsp_mlp* q);
hipError_t mlp_forward_raw(lsp_mlp* q, const float* X, int rows, float* Y, hipStream_t s);
hipStream_t mlp_stream(const lsp_mlp* q);
int mlp_batch_rows(const lsp_mlp* q);
int mlp_inputs(const lsp_mlp* q);
int mlp_outputs(const lsp_mlp* q);
hipError_t launch_features(const lsp_problem* p, const int64_t* points, int64_t j0, int rows,
                           float* X);
hipError_t launch_targets(const lsp_problem* p, const double* P, const int64_t* points, int rows,
                          float* T);
// fused learned setup (learned.hip): network, check and rows in one pass
bool learned_fused_supported(const lsp_problem* p, const MlpView& mv);
hipError_t launch_learned_fused(const lsp_problem* p, const MlpView& mv, double thr,
                                const double* rho_star, double* P, double* Crows,
                                int32_t* fallback, int* nfall);
hipError_t launch_learned_rows(const lsp_problem* p, const double* rho_star, const float* Y,
                               int64_t j0, int rows, double thr, double* P, double* Crows,
                               int32_t* fallback, int* nfall);

}  // namespace lsp
