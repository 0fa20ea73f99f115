// The P-solve of the preconditioner P^-1 C (eq. PC) on the device, from the
// nested-dissection factors of P computed on the host (Sec. 3, Fig. 1; the
// factorisation itself is the plain host step, see nd.py).
//
// The factors come per front (the points eliminated together: a box interior
// or a separator piece): its F and U index lists and four dense row-major
// blocks, L_FF^-1, L_UF L_FF^-1, U_FF^-1 and U_FF^-1 U_FU (formed on the
// host). With Pi the row permutation of F and r_F the front's right-hand side
// after the updates of earlier fronts,
//   forward  (levels in order):   y_F = L_FF^-1 Pi r_F,
//                                 updates (L_UF L_FF^-1) Pi r_F for the U points
//   backward (levels reversed):   x_F = U_FF^-1 y_F - (U_FF^-1 U_FU) x_U
// so each pass is a set of independent row products per level: one launch
// per level and pass. Fronts of one level (one merge step of the boxes) do
// not depend on each other. The updates are not scattered: each front stores
// them in the slots of its U list, numbered so that the updates a point
// receives are consecutive (in front order), and a point gathers them when
// its own front is reached; every sum is in a fixed order, so the solve is
// deterministic.
//
// Levels with many small fronts run one block per front (the block gathers
// r_F, or y_F and x_U, into LDS first); levels with few large fronts split
// the rows over blocks, each block gathering the front's r_F into LDS itself
// (backward, the blocks read y_F and x_U directly).
//
// Row products: LANES lanes share a row (8 to 64, by the row length), each
// striding over the columns with four independent loads in flight (the last
// up to three chunks as predicated loads issued together), then a butterfly
// over the LANES lanes. Real factors, complex vectors.
#include <algorithm>
#include <vector>

#include "lsp_internal.h"

namespace {

constexpr int kThreads = 256;
constexpr int kFusedMinFronts = 64;   // a level runs fused with at least this many fronts
constexpr int kFusedMaxFU = 2048;     // and f + u <= this (LDS: (f + u) complex entries)
constexpr int kSplitGatherMax = 4096; // split levels gather inside the first product up to this f
constexpr int kStagedMaxTasks = 4;    // ... and while a front spans at most this many blocks
                                      // (each block gathers the whole r_F again)

struct Fac {
  const int64_t* f;
  const int64_t* u;
  const int64_t* off_F;
  const int64_t* off_U;
  const int64_t* idx_F;
  const int64_t* idx_Fp;
  const int64_t* idx_U;
  const int64_t* off_blk;
  const double* data;
  const int64_t* upd_ptr;
  const int64_t* slot;  // U-list position -> its update slot (slots grouped by point)
};

// lanes per row for rows of c columns: split products (few rows per block)
// and one-block-per-front products (many rows per block, so fewer lanes per
// row keep more rows in flight)
int lanes_for(int64_t c) { return c >= 192 ? 64 : c >= 96 ? 32 : c >= 40 ? 16 : 8; }
int lanes_for_fused(int64_t c) { return c >= 384 ? 64 : c >= 192 ? 32 : c >= 80 ? 16 : 8; }

// r_eff = r[pt] - the updates sent to pt, which sit in the consecutive slots
// upd_ptr[pt] .. upd_ptr[pt+1] in front order
__device__ inline double2 gather_point(const Fac& fc, const double2* __restrict__ r,
                                       const double2* __restrict__ Wslots, int64_t pt) {
  double2 v = r[pt];
  int64_t q = fc.upd_ptr[pt];
  const int64_t qe = fc.upd_ptr[pt + 1];
  for (; q + 3 < qe; q += 4) {  // four loads in flight, subtracted in order
    const double2 w0 = Wslots[q], w1 = Wslots[q + 1], w2 = Wslots[q + 2], w3 = Wslots[q + 3];
    v.x = (((v.x - w0.x) - w1.x) - w2.x) - w3.x;
    v.y = (((v.y - w0.y) - w1.y) - w2.y) - w3.y;
  }
  for (; q < qe; ++q) {
    const double2 w = Wslots[q];
    v.x -= w.x;
    v.y -= w.y;
  }
  return v;
}

// sum_j mrow[j] x(j) over this lane's columns j = sub, sub + LANES, ...,
// reduced over the LANES lanes of the row (every lane gets the sum)
template <int LANES, typename X>
__device__ inline double2 row_dot(const double* __restrict__ mrow, int64_t cols, int sub,
                                  bool active, X x) {
  double ar0 = 0.0, ai0 = 0.0, ar1 = 0.0, ai1 = 0.0;
  if (active) {
    int64_t j = sub;
    for (; j + 3 * LANES < cols; j += 4 * LANES) {
      const double m0 = mrow[j], m1 = mrow[j + LANES], m2 = mrow[j + 2 * LANES],
                   m3 = mrow[j + 3 * LANES];
      const double2 x0 = x(j), x1 = x(j + LANES), x2 = x(j + 2 * LANES), x3 = x(j + 3 * LANES);
      ar0 = fma(m0, x0.x, ar0);
      ai0 = fma(m0, x0.y, ai0);
      ar1 = fma(m1, x1.x, ar1);
      ai1 = fma(m1, x1.y, ai1);
      ar0 = fma(m2, x2.x, ar0);
      ai0 = fma(m2, x2.y, ai0);
      ar1 = fma(m3, x3.x, ar1);
      ai1 = fma(m3, x3.y, ai1);
    }
    // the last (up to three) chunks: predicated loads issued together
    const bool t0 = j < cols, t1 = j + LANES < cols, t2 = j + 2 * LANES < cols;
    const double m0 = t0 ? mrow[j] : 0.0, m1 = t1 ? mrow[j + LANES] : 0.0,
                 m2 = t2 ? mrow[j + 2 * LANES] : 0.0;
    const double2 z = make_double2(0.0, 0.0);
    const double2 x0 = t0 ? x(j) : z, x1 = t1 ? x(j + LANES) : z, x2 = t2 ? x(j + 2 * LANES) : z;
    if (t0) {
      ar0 = fma(m0, x0.x, ar0);
      ai0 = fma(m0, x0.y, ai0);
    }
    if (t1) {
      ar1 = fma(m1, x1.x, ar1);
      ai1 = fma(m1, x1.y, ai1);
    }
    if (t2) {
      ar0 = fma(m2, x2.x, ar0);
      ai0 = fma(m2, x2.y, ai0);
    }
  }
  double ar = ar0 + ar1, ai = ai0 + ai1;
#pragma unroll
  for (int o = 1; o < LANES; o <<= 1) {
    ar += __shfl_xor(ar, o);
    ai += __shfl_xor(ai, o);
  }
  return make_double2(ar, ai);
}

// forward, one block per front of the level: rows i < f give y_F (stored in
// Yc), rows f <= i < f + u the updates (stored in their slots)
template <int LANES>
__global__ __launch_bounds__(kThreads) void nd_fwd_fused_kernel(Fac fc, int64_t front0,
                                                                const double2* __restrict__ r,
                                                                double2* __restrict__ Yc,
                                                                double2* __restrict__ Wslots) {
  extern __shared__ double2 lds[];
  const int64_t k = front0 + blockIdx.x;
  const int64_t f = fc.f[k], u = fc.u[k], oF = fc.off_F[k], oU = fc.off_U[k];
  for (int64_t i = threadIdx.x; i < f; i += kThreads)
    lds[i] = gather_point(fc, r, Wslots, fc.idx_Fp[oF + i]);
  __syncthreads();
  constexpr int G = kThreads / LANES;
  const int g = threadIdx.x / LANES, sub = threadIdx.x % LANES;
  const double* Linv = fc.data + fc.off_blk[4 * k];
  const double* LUFL = fc.data + fc.off_blk[4 * k + 1];
  for (int64_t i0 = 0; i0 < f + u; i0 += G) {
    const int64_t i = i0 + g;
    const double* row = (i < f) ? Linv + i * f : LUFL + (i - f) * f;
    const double2 y =
        row_dot<LANES>(row, f, sub, i < f + u, [&](int64_t j) { return lds[j]; });
    if (sub == 0 && i < f + u) {
      if (i < f) Yc[oF + i] = y;
      else Wslots[fc.slot[oU + i - f]] = y;
    }
  }
}

// backward, one block per front: x_F = U_FF^-1 y_F - (U_FF^-1 U_FU) x_U with
// y_F and x_U gathered into LDS
template <int LANES>
__global__ __launch_bounds__(kThreads) void nd_bwd_fused_kernel(Fac fc, int64_t front0,
                                                                const double2* __restrict__ Yc,
                                                                double2* __restrict__ X) {
  extern __shared__ double2 lds[];
  const int64_t k = front0 + blockIdx.x;
  const int64_t f = fc.f[k], u = fc.u[k], oF = fc.off_F[k], oU = fc.off_U[k];
  double2* YF = lds;
  double2* XU = lds + f;
  for (int64_t j = threadIdx.x; j < f; j += kThreads) YF[j] = Yc[oF + j];
  for (int64_t j = threadIdx.x; j < u; j += kThreads) XU[j] = X[fc.idx_U[oU + j]];
  __syncthreads();
  constexpr int G = kThreads / LANES;
  const int g = threadIdx.x / LANES, sub = threadIdx.x % LANES;
  const double* Uinv = fc.data + fc.off_blk[4 * k + 2];
  const double* UU = fc.data + fc.off_blk[4 * k + 3];
  for (int64_t i0 = 0; i0 < f; i0 += G) {
    const int64_t i = i0 + g;
    const bool act = i < f;
    const double2 a = row_dot<LANES>(Uinv + i * f, f, sub, act, [&](int64_t j) { return YF[j]; });
    const double2 b = row_dot<LANES>(UU + i * u, u, sub, act, [&](int64_t j) { return XU[j]; });
    if (sub == 0 && act) X[fc.idx_F[oF + i]] = make_double2(a.x - b.x, a.y - b.y);
  }
}

// split levels, gather: R[row] = r_eff of the point of F-list row `row`,
// rows [r0, r1) (only for fronts too large to stage r_F in LDS)
__global__ __launch_bounds__(kThreads) void nd_gather_kernel(Fac fc, const double2* __restrict__ r,
                                                             const double2* __restrict__ Wslots,
                                                             int64_t r0, int64_t r1,
                                                             double2* __restrict__ R) {
  const int64_t row = r0 + (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (row >= r1) return;
  R[row] = gather_point(fc, r, Wslots, fc.idx_Fp[row]);
}

// split levels, forward: one task = kThreads / LANES rows (of the f + u rows
// of a front) of y_F and the updates. STAGED: each block gathers the front's
// r_F into LDS; otherwise r_F is read from R (filled by nd_gather_kernel).
template <int LANES, bool STAGED>
__global__ __launch_bounds__(kThreads) void nd_fwd_split_kernel(Fac fc,
                                                                const int2* __restrict__ tasks,
                                                                const double2* __restrict__ r,
                                                                const double2* __restrict__ R,
                                                                double2* __restrict__ Yc,
                                                                double2* __restrict__ Wslots) {
  extern __shared__ double2 lds[];
  const int2 tk = tasks[blockIdx.x];
  const int64_t k = tk.x;
  const int64_t f = fc.f[k], u = fc.u[k], oF = fc.off_F[k], oU = fc.off_U[k];
  if constexpr (STAGED) {
    for (int64_t i = threadIdx.x; i < f; i += kThreads)
      lds[i] = gather_point(fc, r, Wslots, fc.idx_Fp[oF + i]);
    __syncthreads();
  }
  const int sub = threadIdx.x % LANES;
  const int64_t i = tk.y + threadIdx.x / LANES;
  const bool act = i < f + u;
  const double* row = (i < f) ? fc.data + fc.off_blk[4 * k] + i * f
                              : fc.data + fc.off_blk[4 * k + 1] + (i - f) * f;
  double2 y;
  if constexpr (STAGED) {
    y = row_dot<LANES>(row, f, sub, act, [&](int64_t j) { return lds[j]; });
  } else {
    y = row_dot<LANES>(row, f, sub, act, [&](int64_t j) { return R[oF + j]; });
  }
  if (sub != 0 || !act) return;
  if (i < f) Yc[oF + i] = y;
  else Wslots[fc.slot[oU + i - f]] = y;
}

// split levels, backward: one task = kThreads / LANES rows of x_F
template <int LANES>
__global__ __launch_bounds__(kThreads) void nd_bwd_split_kernel(Fac fc,
                                                                const int2* __restrict__ tasks,
                                                                const double2* __restrict__ Yc,
                                                                double2* __restrict__ X) {
  const int2 tk = tasks[blockIdx.x];
  const int64_t k = tk.x;
  const int64_t f = fc.f[k], u = fc.u[k], oF = fc.off_F[k], oU = fc.off_U[k];
  const int sub = threadIdx.x % LANES;
  const int64_t i = tk.y + threadIdx.x / LANES;
  const bool act = i < f;
  const double* Uinv = fc.data + fc.off_blk[4 * k + 2];
  const double* UU = fc.data + fc.off_blk[4 * k + 3];
  const int64_t* U = fc.idx_U + oU;
  const double2 a = row_dot<LANES>(Uinv + i * f, f, sub, act, [&](int64_t j) { return Yc[oF + j]; });
  const double2 b = row_dot<LANES>(UU + i * u, u, sub, act, [&](int64_t j) { return X[U[j]]; });
  if (sub == 0 && act) X[fc.idx_F[oF + i]] = make_double2(a.x - b.x, a.y - b.y);
}

#define LSP_LANES_SWITCH(lanes, CALL8, CALL16, CALL32, CALL64) \
  switch (lanes) {                                             \
    case 8: CALL8; break;                                      \
    case 16: CALL16; break;                                    \
    case 32: CALL32; break;                                    \
    default: CALL64; break;                                    \
  }

void launch_fwd_fused(int lanes, int nfronts, size_t lds, hipStream_t st, const Fac& fc,
                      int64_t front0, const double2* r, double2* Yc, double2* W) {
  const dim3 grid(nfronts), block(kThreads);
  LSP_LANES_SWITCH(lanes,
      hipLaunchKernelGGL(nd_fwd_fused_kernel<8>, grid, block, lds, st, fc, front0, r, Yc, W),
      hipLaunchKernelGGL(nd_fwd_fused_kernel<16>, grid, block, lds, st, fc, front0, r, Yc, W),
      hipLaunchKernelGGL(nd_fwd_fused_kernel<32>, grid, block, lds, st, fc, front0, r, Yc, W),
      hipLaunchKernelGGL(nd_fwd_fused_kernel<64>, grid, block, lds, st, fc, front0, r, Yc, W))
}

void launch_bwd_fused(int lanes, int nfronts, size_t lds, hipStream_t st, const Fac& fc,
                      int64_t front0, const double2* Yc, double2* X) {
  const dim3 grid(nfronts), block(kThreads);
  LSP_LANES_SWITCH(lanes,
      hipLaunchKernelGGL(nd_bwd_fused_kernel<8>, grid, block, lds, st, fc, front0, Yc, X),
      hipLaunchKernelGGL(nd_bwd_fused_kernel<16>, grid, block, lds, st, fc, front0, Yc, X),
      hipLaunchKernelGGL(nd_bwd_fused_kernel<32>, grid, block, lds, st, fc, front0, Yc, X),
      hipLaunchKernelGGL(nd_bwd_fused_kernel<64>, grid, block, lds, st, fc, front0, Yc, X))
}

template <bool STAGED>
void launch_fwd_split(int lanes, int ntasks, size_t lds, hipStream_t st, const Fac& fc,
                      const int2* tasks, const double2* r, const double2* R, double2* Yc,
                      double2* W) {
  const dim3 grid(ntasks), block(kThreads);
  LSP_LANES_SWITCH(lanes,
      hipLaunchKernelGGL((nd_fwd_split_kernel<8, STAGED>), grid, block, lds, st, fc, tasks, r, R, Yc, W),
      hipLaunchKernelGGL((nd_fwd_split_kernel<16, STAGED>), grid, block, lds, st, fc, tasks, r, R, Yc, W),
      hipLaunchKernelGGL((nd_fwd_split_kernel<32, STAGED>), grid, block, lds, st, fc, tasks, r, R, Yc, W),
      hipLaunchKernelGGL((nd_fwd_split_kernel<64, STAGED>), grid, block, lds, st, fc, tasks, r, R, Yc, W))
}

void launch_bwd_split(int lanes, int ntasks, hipStream_t st, const Fac& fc, const int2* tasks,
                      const double2* Yc, double2* X) {
  const dim3 grid(ntasks), block(kThreads);
  LSP_LANES_SWITCH(lanes,
      hipLaunchKernelGGL(nd_bwd_split_kernel<8>, grid, block, 0, st, fc, tasks, Yc, X),
      hipLaunchKernelGGL(nd_bwd_split_kernel<16>, grid, block, 0, st, fc, tasks, Yc, X),
      hipLaunchKernelGGL(nd_bwd_split_kernel<32>, grid, block, 0, st, fc, tasks, Yc, X),
      hipLaunchKernelGGL(nd_bwd_split_kernel<64>, grid, block, 0, st, fc, tasks, Yc, X))
}
#undef LSP_LANES_SWITCH

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
                    (void*)s.upd_ptr, (void*)s.slot, (void*)s.tasks, (void*)s.R,
                    (void*)s.Yc, (void*)s.W})
    if (ptr) (void)hipFree(ptr);
  s = NDSolve();
}

hipError_t launch_psolve(const lsp_problem* p, const double* r_dev, double* z_dev, hipStream_t st) {
  const NDSolve& s = p->nd;
  const Fac fc{s.f,    s.u,    s.off_F,   s.off_U, s.idx_F, s.idx_Fp,
               s.idx_U, s.off_blk, s.data, s.upd_ptr, s.slot};
  const double2* r = reinterpret_cast<const double2*>(r_dev);
  double2* X = reinterpret_cast<double2*>(z_dev);
  const int L = (int)s.levels.size();
  for (int l = 0; l < L; ++l) {
    const NDSolve::Level& lv = s.levels[l];
    if (lv.fused) {
      launch_fwd_fused(lv.lanes_f, lv.nfronts, sizeof(double2) * lv.fmax, st, fc, lv.front0, r,
                       s.Yc, s.W);
    } else if (lv.staged) {
      launch_fwd_split<true>(lv.lanes_f, lv.fwd_tasks, sizeof(double2) * lv.fmax, st, fc,
                             s.tasks + lv.fwd_task0, r, s.R, s.Yc, s.W);
    } else {
      const int64_t nrow = lv.row1 - lv.row0;
      hipLaunchKernelGGL(nd_gather_kernel, dim3((unsigned)((nrow + kThreads - 1) / kThreads)),
                         dim3(kThreads), 0, st, fc, r, s.W, lv.row0, lv.row1, s.R);
      launch_fwd_split<false>(lv.lanes_f, lv.fwd_tasks, 0, st, fc, s.tasks + lv.fwd_task0, r,
                              s.R, s.Yc, s.W);
    }
  }
  for (int l = L - 1; l >= 0; --l) {
    const NDSolve::Level& lv = s.levels[l];
    if (lv.fused)
      launch_bwd_fused(lv.lanes_b, lv.nfronts, sizeof(double2) * (lv.fmax + lv.umax), st, fc,
                       lv.front0, s.Yc, X);
    else
      launch_bwd_split(lv.lanes_b, lv.bwd_tasks, st, fc, s.tasks + lv.bwd_task0, s.Yc, X);
  }
  return hipGetLastError();
}

}  // namespace lsp

extern "C" {

int lsp_psolve_upload(lsp_problem* p, const lsp_nd_factors* fac) {
  if (!p || !fac) return lsp::set_error(LSP_EINVAL, "NULL argument");
  const int64_t N = p->N, nf = fac->nfronts, nl = fac->nlevels, nU = fac->nidx_U;
  if (nf < 1 || nf > INT32_MAX || nl < 1 || nl > nf || nU < 0 || fac->ndata < 0)
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
  // the forward pass writes the update of U-list position q into slot[q], so
  // that a point's updates are consecutive; upd_pos must be a permutation
  std::vector<int64_t> slot((size_t)nU, -1);
  for (int64_t q = 0; q < nU; ++q) {
    int64_t& sl = slot[(size_t)fac->upd_pos[q]];
    if (sl >= 0) return lsp::set_error(LSP_EINVAL, "upd_pos names a U-list position twice");
    sl = q;
  }
  for (int64_t pt = 0; pt < N; ++pt)
    for (int64_t q = fac->upd_ptr[pt]; q < fac->upd_ptr[pt + 1]; ++q)
      if (fac->idx_U[fac->upd_pos[q]] != pt)
        return lsp::set_error(LSP_EINVAL, "upd_pos lists a U-list position of another point");
  // levels: consecutive fronts; fused (one block per front) or split, and
  // the row tasks of the split products
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
    lv.front0 = a;
    lv.nfronts = (int)(b - a);
    for (int64_t k = a; k < b; ++k) {
      lv.fmax = std::max(lv.fmax, fac->f[k]);
      lv.umax = std::max(lv.umax, fac->u[k]);
    }
    lv.fused = lv.nfronts >= kFusedMinFronts && lv.fmax + lv.umax <= kFusedMaxFU;
    lv.lanes_f = lv.fused ? lanes_for_fused(lv.fmax) : lanes_for(lv.fmax);
    lv.lanes_b = lv.fused ? lanes_for_fused(std::max(lv.fmax, lv.umax))
                          : lanes_for(std::max(lv.fmax, lv.umax));
    lv.staged = lv.fmax <= kSplitGatherMax &&
                (lv.fmax + lv.umax + kThreads / lv.lanes_f - 1) / (kThreads / lv.lanes_f) <=
                    kStagedMaxTasks;
    if (!lv.fused) {
      auto add = [&](int lanes, bool with_u) {
        const int per = kThreads / lanes;
        for (int64_t k = a; k < b; ++k) {
          const int64_t rows = fac->f[k] + (with_u ? fac->u[k] : 0);
          for (int64_t r0 = 0; r0 < rows; r0 += per) tasks.push_back(make_int2((int)k, (int)r0));
        }
      };
      lv.fwd_task0 = (int64_t)tasks.size();
      add(lv.lanes_f, true);
      lv.fwd_tasks = (int)(tasks.size() - lv.fwd_task0);
      lv.bwd_task0 = (int64_t)tasks.size();
      add(lv.lanes_b, false);
      lv.bwd_tasks = (int)(tasks.size() - lv.bwd_task0);
    }
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
      (rc = up(&s.slot, slot.data(), nU, "update slots of the U lists")) ||
      (rc = up(&s.tasks, tasks.data(), tasks.size(), "tasks")) ||
      (rc = up<double2>(&s.R, nullptr, N, "solve buffer")) ||
      (rc = up<double2>(&s.Yc, nullptr, N, "solve buffer")) ||
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
