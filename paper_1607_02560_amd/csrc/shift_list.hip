// First half of the shift list S of Sec. 4.1: per-block (min, max) of the
// potential v over a fixed grid of kMinMaxBlocks blocks (and, for the one
// shift of the non-localized method of Sec. 3, per-block sums of v). The Green's-sum
// kernel reduces these partials in its prologue and forms the bin centres
// (lsp::shift_list_block), so the list never takes a launch of its own and no
// value goes through the host.
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
    part[2 * bx] = lo;
    part[2 * bx + 1] = hi;
    if constexpr (SUM) part[2 * lsp::kMinMaxBlocks + bx] = sum;
  }
}

__global__ __launch_bounds__(kThreads) void minmax_partial_kernel(const double* __restrict__ v,
                                                                  int64_t N, double* part) {
  minmax_body<false>(blockIdx.x, gridDim.x, v, N, part);
}

__global__ __launch_bounds__(kThreads) void minmax_sum_partial_kernel(
    const double* __restrict__ v, int64_t N, double* part) {
  minmax_body<true>(blockIdx.x, gridDim.x, v, N, part);
}

// one launch for the problems of a batch: block b works for problem map[b].x
// as its block map[b].y of kMinMaxBlocks
__global__ __launch_bounds__(kThreads) void minmax_batched_kernel(const lsp::BatchRec* recs,
                                                                  const int4* map) {
  const int4 it = map[blockIdx.x];
  const lsp::BatchRec& r = recs[it.x];
  minmax_body<false>(it.y, lsp::kMinMaxBlocks, r.v, r.N, r.mm_part);
}

}  // namespace

namespace lsp {

hipError_t launch_minmax_batched(const BatchRec* recs, const int4* map, int blocks,
                                 hipStream_t s) {
  hipLaunchKernelGGL(minmax_batched_kernel, dim3(blocks), dim3(kThreads), 0, s, recs, map);
  return hipGetLastError();
}

hipError_t launch_minmax(lsp_problem* p, bool with_sum) {
  if (with_sum)
    hipLaunchKernelGGL(minmax_sum_partial_kernel, dim3(kMinMaxBlocks), dim3(kThreads), 0,
                       p->stream, p->v, p->N, p->ws.minmax_part);
  else
    hipLaunchKernelGGL(minmax_partial_kernel, dim3(kMinMaxBlocks), dim3(kThreads), 0, p->stream,
                       p->v, p->N, p->ws.minmax_part);
  return hipGetLastError();
}

}  // namespace lsp
