// The shift list S of Sec. 4.1 (and the one shift of the non-localized
// method of Sec. 3): a grid of blocks writes per-block (min, max) partials of
// the potential v (and, for the one shift, per-block sums) with plain
// stores; then the partials are reduced, the bin centres formed, snapped and
// deduplicated (lsp::shift_list_block; the kernel boundary orders the
// partials, no atomics). Every problem takes kMinMaxBlocks blocks. For a
// single problem every block of its Green's-sum launch forms the list (block
// 0 publishes S, |S| and (v_min, v_max)); a batch forms each problem's list
// in a one-block-per-problem launch. No value goes through the host.
//
// The same launch can also write the folded cosine weights of the Green's
// sums, cw[k][dl] = w(k) cos(2 pi k dl / n) for k in [0, n/2], dl in [0, W)
// (w = 1 at k = 0 and k = n/2, else 2), one entry per thread of the grid.
#include "setup_common.h"

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kUnroll = 8;

// Block b reduces a grid-strided share of v; blocks with no element write
// (+inf, -inf). N is a power of two >= 64, so v is read as double2.
// SUM also writes the block's sum of v to part[2 * kMinMaxBlocks + b] (for
// the mean of the non-localized shift), summed in a fixed order: each thread
// in its own element order, then a butterfly over the lanes (both partners
// add the same two values, so every lane holds the same sum), then the waves
// in index order.
template <bool SUM>
__device__ __forceinline__ void minmax_body(int bx, int gx, const double* __restrict__ v,
                                            int64_t N, double* part) {
  __shared__ double wmin[kWaves], wmax[kWaves], wsum[kWaves];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wid = tid >> 6;
  double lo = INFINITY, hi = -INFINITY, sum = 0.0;
  const int64_t half = N / 2;
  const double2* v2 = reinterpret_cast<const double2*>(v);
  const int64_t stride = (int64_t)gx * kThreads;
  int64_t i = (int64_t)bx * kThreads + tid;
  for (; i + (kUnroll - 1) * stride < half; i += kUnroll * stride) {
    double2 x[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) x[u] = v2[i + u * stride];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      lo = fmin(lo, fmin(x[u].x, x[u].y));
      hi = fmax(hi, fmax(x[u].x, x[u].y));
      if constexpr (SUM) sum = (sum + x[u].x) + x[u].y;
    }
  }
  for (; i < half; i += stride) {
    const double2 x = v2[i];
    lo = fmin(lo, fmin(x.x, x.y));
    hi = fmax(hi, fmax(x.x, x.y));
    if constexpr (SUM) sum = (sum + x.x) + x.y;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, o));
    hi = fmax(hi, __shfl_xor(hi, o));
    if constexpr (SUM) sum += __shfl_xor(sum, o);
  }
  if (lane == 0) {
    wmin[wid] = lo;
    wmax[wid] = hi;
    if constexpr (SUM) wsum[wid] = sum;
  }
  __syncthreads();
  if (tid == 0) {
    for (int w = 1; w < kWaves; ++w) {
      lo = fmin(lo, wmin[w]);
      hi = fmax(hi, wmax[w]);
      if constexpr (SUM) sum += wsum[w];
    }
    reinterpret_cast<double2*>(part)[bx] = make_double2(lo, hi);
    if constexpr (SUM) part[2 * lsp::kMinMaxBlocks + bx] = sum;
  }
}

// entry e of the cosine tables of (n, W), H = n/2 + 1 rows (lsp::cos_table_doubles):
// cw[k W + dl] for e < H W, then the same values halved (the weights of a
// diagonal tile pair of the 2D Green's sums), then the per-axis eigenvalues
// 4 pi^2 k^2 of the symbol of -Laplacian (Sec. 2)
__device__ __forceinline__ void cos_entry(int n, int W, int e, double* cw) {
  const int H = n / 2 + 1;
  if (e >= 2 * H * W) {
    const int k = e - 2 * H * W;
    cw[e] = lsp::kFourPi2 * (double)(k * k);
    return;
  }
  const bool halved = e >= H * W;
  const int eh = halved ? e - H * W : e;
  const int k = eh / W, dl = eh - k * W;
  const double wk = (k == 0 || k == n / 2) ? 1.0 : 2.0;
  const int j = (int)(((int64_t)k * dl) % n);
  const double c = wk * cospi(2.0 * (double)j / (double)n);
  cw[e] = halved ? 0.5 * c : c;
}

// the partials of a single problem (and, with cw, the cosine tables, one
// entry per thread of the grid)
template <bool SUM>
__global__ __launch_bounds__(kThreads) void minmax_part_kernel(const double* __restrict__ v,
                                                               int64_t N, double* part, int cos_n,
                                                               int cos_w, double* cw) {
  if (cw) {
    const int e = blockIdx.x * kThreads + threadIdx.x;
    if (e < lsp::cos_table_doubles(cos_n, cos_w)) cos_entry(cos_n, cos_w, e, cw);
  }
  minmax_body<SUM>(blockIdx.x, lsp::kMinMaxBlocks, v, N, part);
}

__global__ __launch_bounds__(kThreads) void cos_table_kernel(int n, int W, double* cw) {
  const int e = blockIdx.x * kThreads + threadIdx.x;
  if (e < lsp::cos_table_doubles(n, W)) cos_entry(n, W, e, cw);
}

// one launch for the problems of a batch: block b works for problem map[b].x
// as its block map[b].y of kMinMaxBlocks
__global__ __launch_bounds__(kThreads) void minmax_batched_kernel(const lsp::BatchRec* recs,
                                                                  const int4* map) {
  const int4 it = map[blockIdx.x];
  const lsp::BatchRec& r = recs[it.x];
  minmax_body<false>(it.y, lsp::kMinMaxBlocks, r.v, r.N, r.mm_part);
}

// block b forms the shift list of problem b of a batch from its partials
__global__ __launch_bounds__(kThreads) void shift_list_batched_kernel(const lsp::BatchRec* recs) {
  const lsp::BatchRec& r = recs[blockIdx.x];
  __shared__ double sS[lsp::kMaxShifts];
  __shared__ int sNS, sWave[kWaves];
  __shared__ double sRange[2], sRed[3 * kWaves];
  lsp::shift_list_block<kThreads>(r.mm_part, r.nreq, sS, &sNS, sRange, sWave, sRed);
  for (int i = threadIdx.x; i < sNS; i += kThreads) r.S[i] = sS[i];
  if (threadIdx.x == 0) {
    *r.nS = sNS;
    r.vrange[0] = sRange[0];
    r.vrange[1] = sRange[1];
  }
}

}  // namespace

namespace lsp {

hipError_t launch_minmax_batched(const BatchRec* recs, const int4* map, int blocks, int count,
                                 hipStream_t s) {
  hipLaunchKernelGGL(minmax_batched_kernel, dim3(blocks), dim3(kThreads), 0, s, recs, map);
  hipLaunchKernelGGL(shift_list_batched_kernel, dim3(count), dim3(kThreads), 0, s, recs);
  return hipGetLastError();
}


hipError_t launch_minmax_parts(const double* v, int64_t N, const Workspace& ws, bool global,
                               hipStream_t s, int cos_n, int cos_w, double* cw) {
  if (cw && cos_table_doubles(cos_n, cos_w) > kMinMaxBlocks * kThreads) return hipErrorInvalidValue;
  if (global)
    hipLaunchKernelGGL(minmax_part_kernel<true>, dim3(kMinMaxBlocks), dim3(kThreads), 0, s, v, N,
                       ws.minmax_part, cos_n, cos_w, cw);
  else
    hipLaunchKernelGGL(minmax_part_kernel<false>, dim3(kMinMaxBlocks), dim3(kThreads), 0, s, v, N,
                       ws.minmax_part, cos_n, cos_w, cw);
  return hipGetLastError();
}

hipError_t launch_minmax(lsp_problem* p, bool global) {
  return launch_minmax_parts(p->v, p->N, p->ws, global, p->stream, 0, 0, nullptr);
}

hipError_t launch_cos_table(int n, int W, double* cw, hipStream_t s) {
  const int cnt = cos_table_doubles(n, W);
  hipLaunchKernelGGL(cos_table_kernel, dim3((cnt + kThreads - 1) / kThreads), dim3(kThreads), 0,
                     s, n, W, cw);
  return hipGetLastError();
}

}  // namespace lsp
