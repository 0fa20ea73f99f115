// The P-solve of the preconditioner P^-1 C (eq. PC) on the device, from the
// nested-dissection factors of P computed on the host (Sec. 3, Fig. 1; the
// factorisation itself is the plain host step, see nd.py).
//
// The factors come per front (the points eliminated together: a box interior
// or a separator piece): its F and U index lists, the inverses of its
// triangular blocks L^-1 and U^-1 and its off-diagonal blocks L_UF and U_FU,
// all dense and row-major. With Pi the row permutation of F,
//   forward  (levels in order):   y_F = L^-1 Pi r_F,   r_U -= L_UF y_F
//   backward (levels reversed):   x_F = U^-1 (y_F - U_FU x_U)
// Fronts of one level (one merge step of the boxes) do not depend on each
// other, so a level is three launches forward (gather, two products) and two
// backward. The updates r_U -= L_UF y_F are not scattered: each front stores
// its products L_UF y_F in the slots of its U list, and a point gathers the
// slots that name it, in front order, when its own front is reached; every
// sum is in a fixed order, so the solve is deterministic.
//
// Row products: a block of 256 threads computes 32 rows of one front, 8 lanes
// per row striding over the columns (complex right-hand side, real factors),
// then a butterfly over the 8 lanes.
#include <vector>

#include "lsp_internal.h"

namespace {

constexpr int kThreads = 256;
constexpr int kLanesPerRow = 8;
constexpr int kRowsPerTask = kThreads / kLanesPerRow;  // 32

enum { kFwdL = 0, kFwdLUF = 1, kBwdUFU = 2, kBwdU = 3 };

struct Fac {
  const int64_t* f;
  const int64_t* u;
  const int64_t* off_F;
  const int64_t* off_U;
  const int64_t* idx_F;
  const int64_t* idx_U;
  const int64_t* off_blk;
  const double* data;
};

// R[row] = r[idx_Fp[row]] - sum of the update slots naming that point, for
// the rows [r0, r1) of one level (its fronts are consecutive)
__global__ __launch_bounds__(kThreads) void nd_gather_kernel(
    const double2* __restrict__ r, const int64_t* __restrict__ idx_Fp,
    const int64_t* __restrict__ upd_ptr, const int64_t* __restrict__ upd_pos,
    const double2* __restrict__ Wslots, int64_t r0, int64_t r1, double2* __restrict__ R) {
  const int64_t row = r0 + (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (row >= r1) return;
  const int64_t pt = idx_Fp[row];
  double2 v = r[pt];
  for (int64_t q = upd_ptr[pt]; q < upd_ptr[pt + 1]; ++q) {
    const double2 w = Wslots[upd_pos[q]];
    v.x -= w.x;
    v.y -= w.y;
  }
  R[row] = v;
}

// One task = 32 rows of one front's product (see MODE):
//   kFwdL    Yc[oF + i] = sum_j Linv[i][j] R[oF + j]            i < f
//   kFwdLUF  W[oU + i]  = sum_j LUF[i][j] Yc[oF + j]            i < u
//   kBwdUFU  T[oF + i]  = Yc[oF + i] - sum_j UFU[i][j] X[U[j]]  i < f
//   kBwdU    X[F[i]]    = sum_j Uinv[i][j] T[oF + j]            i < f
template <int MODE>
__global__ __launch_bounds__(kThreads) void nd_product_kernel(Fac fc, const int2* __restrict__ tasks,
                                                              const double2* __restrict__ in,
                                                              const double2* __restrict__ Yc,
                                                              double2* __restrict__ out) {
  const int2 tk = tasks[blockIdx.x];
  const int k = tk.x;
  const int64_t fk = fc.f[k], uk = fc.u[k];
  const int64_t oF = fc.off_F[k], oU = fc.off_U[k];
  const int64_t rows = (MODE == kFwdLUF) ? uk : fk;
  const int64_t cols = (MODE == kFwdLUF) ? fk : (MODE == kBwdUFU ? uk : fk);
  const int blk = (MODE == kFwdL) ? 0 : (MODE == kFwdLUF) ? 1 : (MODE == kBwdU) ? 2 : 3;
  const double* mat = fc.data + fc.off_blk[4 * k + blk];
  const int sub = threadIdx.x % kLanesPerRow;
  const int64_t i = tk.y + threadIdx.x / kLanesPerRow;
  double ar = 0.0, ai = 0.0;
  if (i < rows) {
    const double* mrow = mat + i * cols;
    for (int64_t j = sub; j < cols; j += kLanesPerRow) {
      const double m = mrow[j];
      double2 x;
      if constexpr (MODE == kBwdUFU) x = in[fc.idx_U[oU + j]];
      else x = in[oF + j];
      ar = fma(m, x.x, ar);
      ai = fma(m, x.y, ai);
    }
  }
#pragma unroll
  for (int o = 1; o < kLanesPerRow; o <<= 1) {
    ar += __shfl_xor(ar, o);
    ai += __shfl_xor(ai, o);
  }
  if (sub != 0 || i >= rows) return;
  if constexpr (MODE == kFwdL) {
    out[oF + i] = make_double2(ar, ai);
  } else if constexpr (MODE == kFwdLUF) {
    out[oU + i] = make_double2(ar, ai);
  } else if constexpr (MODE == kBwdUFU) {
    const double2 y = Yc[oF + i];
    out[oF + i] = make_double2(y.x - ar, y.y - ai);
  } else {
    out[fc.idx_F[oF + i]] = make_double2(ar, ai);
  }
}

// device copy of count host entries (src NULL: allocation only)
template <typename T>
int up(T** dst, const T* src, size_t count, const char* what) {
  if (hipMalloc((void**)dst, sizeof(T) * (count ? count : 1)) != hipSuccess) {
    *dst = nullptr;
    (void)hipGetLastError();
    return lsp::set_error(LSP_ENOMEM, std::string("device allocation failed: ") + what);
  }
  if (src && count && hipMemcpy(*dst, src, sizeof(T) * count, hipMemcpyHostToDevice) != hipSuccess)
    return lsp::set_error(LSP_EHIP, std::string("upload failed: ") + what);
  return LSP_OK;
}

}  // namespace

namespace lsp {

void free_psolve(lsp_problem* p) {
  NDSolve& s = p->nd;
  for (void* ptr : {(void*)s.f, (void*)s.u, (void*)s.off_F, (void*)s.off_U, (void*)s.idx_F,
                    (void*)s.idx_Fp, (void*)s.idx_U, (void*)s.off_blk, (void*)s.data,
                    (void*)s.upd_ptr, (void*)s.upd_pos, (void*)s.tasks, (void*)s.R,
                    (void*)s.Yc, (void*)s.T, (void*)s.W})
    if (ptr) (void)hipFree(ptr);
  s = NDSolve();
}

hipError_t launch_psolve(const lsp_problem* p, const double* r_dev, double* z_dev, hipStream_t st) {
  const NDSolve& s = p->nd;
  const Fac fc{s.f, s.u, s.off_F, s.off_U, s.idx_F, s.idx_U, s.off_blk, s.data};
  const double2* r = reinterpret_cast<const double2*>(r_dev);
  double2* X = reinterpret_cast<double2*>(z_dev);
  const int L = (int)s.levels.size();
  for (int l = 0; l < L; ++l) {
    const NDSolve::Level& lv = s.levels[l];
    const int64_t nrow = lv.row1 - lv.row0;
    hipLaunchKernelGGL(nd_gather_kernel, dim3((unsigned)((nrow + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, st, r, s.idx_Fp, s.upd_ptr, s.upd_pos, s.W, lv.row0,
                       lv.row1, s.R);
    hipLaunchKernelGGL(nd_product_kernel<kFwdL>, dim3(lv.nf_tasks), dim3(kThreads), 0, st, fc,
                       s.tasks + lv.f_task0, s.R, s.Yc, s.Yc);
    if (lv.nu_tasks)
      hipLaunchKernelGGL(nd_product_kernel<kFwdLUF>, dim3(lv.nu_tasks), dim3(kThreads), 0, st,
                         fc, s.tasks + lv.u_task0, s.Yc, s.Yc, s.W);
  }
  for (int l = L - 1; l >= 0; --l) {
    const NDSolve::Level& lv = s.levels[l];
    hipLaunchKernelGGL(nd_product_kernel<kBwdUFU>, dim3(lv.nf_tasks), dim3(kThreads), 0, st, fc,
                       s.tasks + lv.f_task0, X, s.Yc, s.T);
    hipLaunchKernelGGL(nd_product_kernel<kBwdU>, dim3(lv.nf_tasks), dim3(kThreads), 0, st, fc,
                       s.tasks + lv.f_task0, s.T, s.Yc, X);
  }
  return hipGetLastError();
}

}  // namespace lsp

extern "C" {

int lsp_psolve_upload(lsp_problem* p, const lsp_nd_factors* fac) {
  if (!p || !fac) return lsp::set_error(LSP_EINVAL, "NULL argument");
  const int64_t N = p->N, nf = fac->nfronts, nl = fac->nlevels, nU = fac->nidx_U;
  if (nf < 1 || nl < 1 || nl > nf || nU < 0 || fac->ndata < 0)
    return lsp::set_error(LSP_EINVAL, "invalid front, level or size counts");
  if (!fac->f || !fac->u || !fac->off_F || !fac->off_U || !fac->idx_F || !fac->idx_Fp ||
      (nU && (!fac->idx_U || !fac->upd_pos)) || !fac->off_blk || (fac->ndata && !fac->data) ||
      !fac->upd_ptr || !fac->lev_ptr || !fac->lev_fronts)
    return lsp::set_error(LSP_EINVAL, "NULL array in the factors");
  // consistency of the structure (host): offsets, index ranges, block extents
  if (fac->off_F[0] != 0 || fac->off_U[0] != 0 || fac->off_F[nf] != N || fac->off_U[nf] != nU ||
      fac->upd_ptr[0] != 0 || fac->upd_ptr[N] != nU || fac->lev_ptr[0] != 0 ||
      fac->lev_ptr[nl] != nf)
    return lsp::set_error(LSP_EINVAL, "factor offsets do not match N or the list sizes");
  for (int64_t k = 0; k < nf; ++k) {
    const int64_t f = fac->f[k], u = fac->u[k];
    if (f < 1 || u < 0 || fac->off_F[k + 1] - fac->off_F[k] != f ||
        fac->off_U[k + 1] - fac->off_U[k] != u)
      return lsp::set_error(LSP_EINVAL, "front sizes do not match their offsets");
    const int64_t need[4] = {f * f, u * f, f * f, f * u};
    for (int j = 0; j < 4; ++j) {
      const int64_t o = fac->off_blk[4 * k + j];
      if (o < 0 || o + need[j] > fac->ndata)
        return lsp::set_error(LSP_EINVAL, "a dense block lies outside the data array");
    }
  }
  for (int64_t i = 0; i < N; ++i) {
    if (fac->idx_F[i] < 0 || fac->idx_F[i] >= N || fac->idx_Fp[i] < 0 || fac->idx_Fp[i] >= N ||
        fac->upd_ptr[i + 1] < fac->upd_ptr[i])
      return lsp::set_error(LSP_EINVAL, "index list entry out of range");
  }
  for (int64_t i = 0; i < nU; ++i)
    if (fac->idx_U[i] < 0 || fac->idx_U[i] >= N || fac->upd_pos[i] < 0 || fac->upd_pos[i] >= nU)
      return lsp::set_error(LSP_EINVAL, "update list entry out of range");
  // levels: consecutive fronts, and the tasks of their products
  std::vector<lsp::NDSolve::Level> levels;
  std::vector<int2> tasks;
  for (int64_t l = 0; l < nl; ++l) {
    const int64_t a = fac->lev_ptr[l], b = fac->lev_ptr[l + 1];
    if (b <= a) return lsp::set_error(LSP_EINVAL, "empty level");
    for (int64_t q = a; q < b; ++q)
      if (fac->lev_fronts[q] != q) return lsp::set_error(LSP_EINVAL, "levels must list fronts in order");
    lsp::NDSolve::Level lv;
    lv.row0 = fac->off_F[a];
    lv.row1 = fac->off_F[b];
    lv.f_task0 = (int64_t)tasks.size();
    for (int64_t k = a; k < b; ++k)
      for (int64_t r0 = 0; r0 < fac->f[k]; r0 += kRowsPerTask) tasks.push_back(make_int2((int)k, (int)r0));
    lv.nf_tasks = (int)(tasks.size() - lv.f_task0);
    lv.u_task0 = (int64_t)tasks.size();
    for (int64_t k = a; k < b; ++k)
      for (int64_t r0 = 0; r0 < fac->u[k]; r0 += kRowsPerTask) tasks.push_back(make_int2((int)k, (int)r0));
    lv.nu_tasks = (int)(tasks.size() - lv.u_task0);
    levels.push_back(lv);
  }
  (void)hipStreamSynchronize(p->stream);
  lsp::free_psolve(p);
  lsp::NDSolve& s = p->nd;
  int rc = LSP_OK;
  if ((rc = up(&s.f, fac->f, nf, "front sizes")) || (rc = up(&s.u, fac->u, nf, "update sizes")) ||
      (rc = up(&s.off_F, fac->off_F, nf + 1, "F offsets")) ||
      (rc = up(&s.off_U, fac->off_U, nf + 1, "U offsets")) ||
      (rc = up(&s.idx_F, fac->idx_F, N, "F lists")) ||
      (rc = up(&s.idx_Fp, fac->idx_Fp, N, "pivoted F lists")) ||
      (rc = up(&s.idx_U, fac->idx_U, nU, "U lists")) ||
      (rc = up(&s.off_blk, fac->off_blk, 4 * nf, "block offsets")) ||
      (rc = up(&s.data, fac->data, fac->ndata, "dense blocks")) ||
      (rc = up(&s.upd_ptr, fac->upd_ptr, N + 1, "update pointers")) ||
      (rc = up(&s.upd_pos, fac->upd_pos, nU, "update positions")) ||
      (rc = up(&s.tasks, tasks.data(), tasks.size(), "tasks")) ||
      (rc = up<double2>(&s.R, nullptr, N, "solve buffer")) ||
      (rc = up<double2>(&s.Yc, nullptr, N, "solve buffer")) ||
      (rc = up<double2>(&s.T, nullptr, N, "solve buffer")) ||
      (rc = up<double2>(&s.W, nullptr, nU, "update slots"))) {
    lsp::free_psolve(p);
    return rc;
  }
  s.levels = levels;
  s.ready = true;
  ++p->ws_gen;
  return LSP_OK;
}

int lsp_psolve_apply(lsp_problem* p, const double* r_dev, double* z_dev) {
  if (!p || !r_dev || !z_dev) return lsp::set_error(LSP_EINVAL, "NULL argument");
  if (r_dev == z_dev) return lsp::set_error(LSP_EINVAL, "r and z must not alias");
  if (!p->nd.ready) return lsp::set_error(LSP_ESTATE, "no factors uploaded (lsp_psolve_upload)");
  const int tk = lsp::stage_begin(p, LSP_STAGE_PSOLVE);
  const int rc = lsp::hip_check(lsp::launch_psolve(p, r_dev, z_dev, p->stream), "P-solve launch");
  lsp::stage_end(p, tk);
  return rc;
}

}  // extern "C"
