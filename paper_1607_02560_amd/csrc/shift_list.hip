// The shift list S of Sec. 4.1 (and the one shift of the non-localized
// method of Sec. 3): a fixed grid of kMinMaxBlocks blocks writes per-block
// (min, max) partials of the potential v (and, for the one shift, per-block
// sums); a block then reduces the partials, forms the bin centres, snaps
// them and removes duplicates (lsp::shift_list_block). No value goes through
// the host. For a single problem every block of the Green's-sum launch that
// follows forms the list itself from the partials (the kernel boundary orders
// them; no atomics), and its block 0 publishes S, |S| and (v_min, v_max).
// The batched form keeps one launch per batch here, where the block that
// finishes last (a ticket counter that is never reset: 256 tickets per
// problem and launch, so it stays a multiple of 256) forms the list.
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
// ATOMIC writes the partials with device-scope atomic swaps (for a reader in
// the same launch), else with plain stores (for a reader in a later launch).
template <bool SUM, bool ATOMIC>
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
    // device-scope atomic swaps: they take effect where the ticket's atomic
    // does, so the last block's atomic reads see them without writing back
    // this XCD's L2 (which a fence would); s_waitcnt below makes them
    // complete before the ticket is drawn
    if constexpr (ATOMIC) {
      using u64 = unsigned long long;
      u64* pu = reinterpret_cast<u64*>(part);
      (void)atomicExch(pu + 2 * bx, (u64)__double_as_longlong(lo));
      (void)atomicExch(pu + 2 * bx + 1, (u64)__double_as_longlong(hi));
      if constexpr (SUM)
        (void)atomicExch(pu + 2 * lsp::kMinMaxBlocks + bx, (u64)__double_as_longlong(sum));
    } else {
      reinterpret_cast<double2*>(part)[bx] = make_double2(lo, hi);
      if constexpr (SUM) part[2 * lsp::kMinMaxBlocks + bx] = sum;
    }
  }
}

// Block bx of kMinMaxBlocks: its partials, then a ticket; the block that draws
// the last ticket of the launch forms the shift list from all partials.
// GLOBAL: the one shift of the non-localized method (the mean of v), else the
// nreq bin centres of Sec. 4.1.
template <bool GLOBAL>
__device__ __forceinline__ void minmax_shift_body(int bx, const double* __restrict__ v, int64_t N,
                                                  double* part, unsigned* ticket, int nreq,
                                                  double* S_out, int* nS_out,
                                                  double* vrange_out) {
  minmax_body<GLOBAL, true>(bx, lsp::kMinMaxBlocks, v, N, part);
  __shared__ int last;
  if (threadIdx.x == 0) {
    __builtin_amdgcn_s_waitcnt(0);  // the partials' swaps have completed
    const unsigned tk = atomicAdd(ticket, 1u);
    last = ((tk + 1u) % (unsigned)lsp::kMinMaxBlocks) == 0u;
  }
  __syncthreads();
  if (!last) return;
  // every block's partials, read with device-scope atomics (see minmax_body)
  __shared__ double sPart[3 * lsp::kMinMaxBlocks];
  {
    using u64 = unsigned long long;
    u64* pu = reinterpret_cast<u64*>(part);
    constexpr int cnt = (GLOBAL ? 3 : 2) * lsp::kMinMaxBlocks;
    for (int e = threadIdx.x; e < cnt; e += kThreads)
      sPart[e] = __longlong_as_double((long long)atomicAdd(pu + e, 0ull));
  }
  __syncthreads();
  __shared__ double sS[lsp::kMaxShifts];
  __shared__ int sNS, sWave[kWaves];
  __shared__ double sRange[2], sRed[3 * kWaves];
  if constexpr (GLOBAL)
    lsp::global_shift_block<kThreads>(sPart, N, sS, &sNS, sRange, sRed);
  else
    lsp::shift_list_block<kThreads>(sPart, nreq, sS, &sNS, sRange, sWave, sRed);
  const int nS = sNS;
  for (int i = threadIdx.x; i < nS; i += kThreads) S_out[i] = sS[i];
  if (threadIdx.x == 0) {
    *nS_out = nS;
    vrange_out[0] = sRange[0];
    vrange_out[1] = sRange[1];
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
  minmax_body<SUM, false>(blockIdx.x, lsp::kMinMaxBlocks, v, N, part);
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
  minmax_shift_body<false>(it.y, r.v, r.N, r.mm_part, r.ticket, r.nreq, r.S, r.nS, r.vrange);
}

}  // namespace

namespace lsp {

hipError_t launch_minmax_batched(const BatchRec* recs, const int4* map, int blocks,
                                 hipStream_t s) {
  hipLaunchKernelGGL(minmax_batched_kernel, dim3(blocks), dim3(kThreads), 0, s, recs, map);
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
