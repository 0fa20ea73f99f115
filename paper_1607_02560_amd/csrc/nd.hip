// Rows of per-point radius (Sec. 4.2, Fig. 3): point j uses the stencil of
// radius t_j, the largest radius that keeps the sparsity nested dissection with
// leaf box b needs, capped at 2 (the radii Sec. 5 computes). The separators are
// the grid planes j_i = 0 mod b; a vertex (every coordinate on a separator)
// may reach t = b, any other point reaches up to the nearest separator plane
// across its coordinates off the separators.
//
// Rows keep the layout of radius 2 (the 5^d offsets of mu_0^2, lexicographic,
// last axis fastest); a row with t_j = 1 holds the radius-1 stencil on the
// offsets of mu_0^1 and zeros elsewhere. Entry a of row j is
//   alpha^{t_j}_{s_j}[a] + C^{t_j}_{s_j}[a] (v[j + a] - s_j),
// evaluated exactly as the uniform-radius assembly does, and the row of C is
// written beside it for the C-apply.
#include "setup_common.h"

#pragma clang fp contract(off)

namespace {

using lsp::nearest_shift;
using lsp::Pow;

template <int D>
__device__ __forceinline__ int nd_radius(const int* c, int b, int tmax) {
  int reach = b;
  bool off = false;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const int r = c[i] % b;
    if (r != 0) {
      off = true;
      reach = min(reach, min(r, b - r));
    }
  }
  return min(off ? reach : b, tmax);
}

// one thread per entry (j, a) of the radius-2 layout, so that consecutive
// threads store consecutive doubles; act1/act2 are the (alpha, C) tables of
// radius 1 and 2
template <int D>
__global__ __launch_bounds__(256) void assemble_nd_kernel(
    const double* __restrict__ v, int n, int64_t N, const double* __restrict__ S,
    const int* __restrict__ nS_ptr, const double2* __restrict__ act1,
    const double2* __restrict__ act2, int b, double* __restrict__ P,
    double* __restrict__ Crows, int32_t* __restrict__ idx_out) {
  constexpr int W2 = 5;
  constexpr int M2 = Pow<D, 5>::v;
  constexpr int M1 = Pow<D, 3>::v;
  // the shift list in LDS; then, once per point of the block's entry range
  // (at most 256 / M2 + 2 points), its shift, s_j and radius
  constexpr int PTS = 256 / M2 + 2;
  __shared__ double sS[lsp::kMaxShifts];
  __shared__ double sSj[PTS];
  __shared__ int sId[PTS], sT[PTS];
  const int nS = *nS_ptr;
  for (int i = threadIdx.x; i < nS; i += 256) sS[i] = S[i];
  __syncthreads();
  const int64_t e0 = (int64_t)blockIdx.x * 256;
  const int64_t j0 = e0 / M2;
  if (threadIdx.x < PTS) {
    const int64_t jp = j0 + threadIdx.x;
    if (jp < N) {
      int cp[D];
      int64_t rem = jp;
#pragma unroll
      for (int i = D - 1; i >= 0; --i) {
        cp[i] = (int)(rem % n);
        rem /= n;
      }
      const int id = nearest_shift(sS, nS, v[jp]);
      sId[threadIdx.x] = id;
      sSj[threadIdx.x] = sS[id];
      sT[threadIdx.x] = nd_radius<D>(cp, b, 2);
      if (idx_out) idx_out[jp] = id;
    }
  }
  __syncthreads();
  const int64_t e = e0 + threadIdx.x;
  if (e >= N * M2) return;
  const int64_t j = e / M2;
  const int a = (int)(e - j * M2);
  const int lp = (int)(j - j0);
  int c[D];
  {
    int64_t rem = j;
#pragma unroll
    for (int i = D - 1; i >= 0; --i) {
      c[i] = (int)(rem % n);
      rem /= n;
    }
  }
  const int id = sId[lp];
  const double s = sSj[lp];
  const int t = sT[lp];
  const int mask = n - 1;
  int o[D];
  {
    int rem = a;
#pragma unroll
    for (int i = D - 1; i >= 0; --i) {
      o[i] = rem % W2 - 2;
      rem /= W2;
    }
  }
  bool inner = true;
  int a1 = 0;
  int64_t g = 0;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    inner = inner && o[i] >= -1 && o[i] <= 1;
    a1 = a1 * 3 + o[i] + 1;
    g = g * n + ((c[i] + o[i]) & mask);
  }
  double pv = 0.0, cv = 0.0;
  if (t >= 2 || inner) {
    const double2 ac = (t >= 2) ? act2[(int64_t)id * M2 + a] : act1[(int64_t)id * M1 + a1];
    pv = ac.x + ac.y * (v[g] - s);
    cv = ac.y;
  }
  P[e] = pv;
  Crows[e] = cv;
}

}  // namespace

namespace lsp {

hipError_t launch_assemble_nd(lsp_problem* p, const double2* act1, int leaf, double* P,
                              int32_t* idx) {
  const int64_t N = p->N;
  const int64_t entries = N * (p->d == 2 ? 25 : 125);
  const dim3 grid((unsigned)((entries + 255) / 256)), blk(256);
  const double2* act2 = reinterpret_cast<const double2*>(p->ws.actab);
  if (p->d == 2)
    hipLaunchKernelGGL(assemble_nd_kernel<2>, grid, blk, 0, p->stream, p->v, p->n, N, p->ws.S,
                       p->ws.nS, act1, act2, leaf, P, p->c_rows, idx);
  else
    hipLaunchKernelGGL(assemble_nd_kernel<3>, grid, blk, 0, p->stream, p->v, p->n, N, p->ws.S,
                       p->ws.nS, act1, act2, leaf, P, p->c_rows, idx);
  return hipGetLastError();
}

}  // namespace lsp
