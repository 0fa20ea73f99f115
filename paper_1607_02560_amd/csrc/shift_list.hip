// First stage of the shift list of Sec. 4.1: per-block (min, max) of the
// potential v. The list itself (bin centres over [v_min, v_max] snapped to
// (4m+2) pi^2, duplicates removed) is derived from these partials at the
// start of the next kernel by lsp::shift_list_block, which every block of
// that kernel runs, so no cross-block synchronisation or host round trip is
// needed.
#include "setup_common.h"

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kUnroll = 8;

__global__ __launch_bounds__(kThreads) void minmax_partial_kernel(const double* __restrict__ v,
                                                                  int64_t N, double* part) {
  __shared__ double wmin[kWaves], wmax[kWaves];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wid = tid >> 6;
  double lo = INFINITY, hi = -INFINITY;
  const int64_t half = N / 2;  // N is a power of two >= 64
  const double2* v2 = reinterpret_cast<const double2*>(v);
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  int64_t i = (int64_t)blockIdx.x * kThreads + tid;
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
    part[2 * blockIdx.x] = lo;
    part[2 * blockIdx.x + 1] = hi;
  }
}

}  // namespace

namespace lsp {

int minmax_blocks(int64_t N) {
  int64_t blocks = (N / 2 + (int64_t)kThreads * kUnroll - 1) / ((int64_t)kThreads * kUnroll);
  if (blocks > kMinMaxBlocks) blocks = kMinMaxBlocks;
  if (blocks < 1) blocks = 1;
  return (int)blocks;
}

hipError_t launch_shift_list(lsp_problem* p, int num_shifts) {
  (void)num_shifts;
  hipLaunchKernelGGL(minmax_partial_kernel, dim3(minmax_blocks(p->N)), dim3(kThreads), 0,
                     p->stream, p->v, p->N, p->ws.minmax_part);
  return hipGetLastError();
}

}  // namespace lsp
