// First half of the shift list S of Sec. 4.1: per-block (min, max) of the
// potential v over a fixed grid of kMinMaxBlocks blocks. The Green's-sum
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
__device__ __forceinline__ void minmax_body(int bx, int gx, const double* __restrict__ v,
                                            int64_t N, double* part) {
  __shared__ double wmin[kWaves], wmax[kWaves];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wid = tid >> 6;
  double lo = INFINITY, hi = -INFINITY;
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
    }
  }
  for (; i < half; i += stride) {
    const double2 x = v2[i];
    lo = fmin(lo, fmin(x.x, x.y));
    hi = fmax(hi, fmax(x.x, x.y));
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, o));
    hi = fmax(hi, __shfl_xor(hi, o));
  }
  if (lane == 0) {
    wmin[wid] = lo;
    wmax[wid] = hi;
  }
  __syncthreads();
  if (tid == 0) {
    for (int w = 1; w < kWaves; ++w) {
      lo = fmin(lo, wmin[w]);
      hi = fmax(hi, wmax[w]);
    }
    part[2 * bx] = lo;
    part[2 * bx + 1] = hi;
  }
}

__global__ __launch_bounds__(kThreads) void minmax_partial_kernel(const double* __restrict__ v,
                                                                  int64_t N, double* part) {
  minmax_body(blockIdx.x, gridDim.x, v, N, part);
}

// one launch for the problems of a batch: block b works for problem map[b].x
// as its block map[b].y of kMinMaxBlocks
__global__ __launch_bounds__(kThreads) void minmax_batched_kernel(const lsp::BatchRec* recs,
                                                                  const int4* map) {
  const int4 it = map[blockIdx.x];
  const lsp::BatchRec& r = recs[it.x];
  minmax_body(it.y, lsp::kMinMaxBlocks, r.v, r.N, r.mm_part);
}

}  // namespace

namespace lsp {

hipError_t launch_minmax_batched(const BatchRec* recs, const int4* map, int blocks,
                                 hipStream_t s) {
  hipLaunchKernelGGL(minmax_batched_kernel, dim3(blocks), dim3(kThreads), 0, s, recs, map);
  return hipGetLastError();
}

hipError_t launch_minmax(lsp_problem* p) {
  hipLaunchKernelGGL(minmax_partial_kernel, dim3(kMinMaxBlocks), dim3(kThreads), 0, p->stream,
                     p->v, p->N, p->ws.minmax_part);
  return hipGetLastError();
}

}  // namespace lsp
