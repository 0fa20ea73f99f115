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
// evaluated exactly as the uniform-radius assembly does.
#include "setup_common.h"

#pragma clang fp contract(off)

namespace {

using lsp::nd_radius;
using lsp::nearest_shift;
using lsp::Pow;

// A block owns TW consecutive points of one grid row (as the uniform
// assembly tiles): the potential on the row segment plus a halo of 2 in
// every direction, the shift list and per point its shift and its row of
// the (alpha, C) table of its radius are staged in LDS (the radius-1 pairs
// are stored in the radius-2 layout, (0, 0) outside mu_0^1, so both radii
// read one layout). The tile's rows form one span of TW * 5^d entries,
// written in steps of a whole number of points by the first TACT = 256 -
// 256 % M2 threads; each thread's VEC = 2 entries per step keep their
// offsets, so the offset-dependent parts (table position, halo position,
// point increment) are worked out once. P is written with 16-byte stores;
// the C-apply reads C from the tables of the point's radius (no C rows are
// stored).
template <int D, int TW>
__global__ __launch_bounds__(256) void assemble_nd_kernel(
    const double* __restrict__ v, int n, int lg, const double* __restrict__ S,
    const int* __restrict__ nS_ptr, const double2* __restrict__ act1,
    const double2* __restrict__ act2, int b, double* __restrict__ P,
    int32_t* __restrict__ idx_out) {
  constexpr int W2 = 5;
  constexpr int t = 2;
  constexpr int M2 = Pow<D, 5>::v;
  constexpr int PL = (D == 3) ? W2 : 1;
  constexpr int HR = 1 + 2 * t;
  constexpr int HC = TW + 2 * t;
  __shared__ double halo[PL * HR * HC];
  __shared__ double sS[lsp::kMaxShifts];
  __shared__ double spS[TW];            // per point: s_j
  __shared__ const double2* spP[TW];    // per point: its (alpha, C) row (radius t_j)
  const int tid = threadIdx.x;
  const int nS = *nS_ptr;
  const int c0 = blockIdx.x * TW;
  const int r0 = blockIdx.y;
  const int p0 = (D == 3) ? (int)blockIdx.z : 0;
  const int mask = n - 1;
  for (int i = tid; i < nS; i += 256) sS[i] = S[i];
  for (int e = tid; e < PL * HR * HC; e += 256) {
    const int hc = e % HC;
    const int hr = (e / HC) % HR;
    const int hp = e / (HC * HR);
    const int gc = (c0 - t + hc) & mask;
    const int gr = (r0 - t + hr) & mask;
    int64_t g;
    if constexpr (D == 3) {
      const int gp = (p0 - t + hp) & mask;
      g = ((((int64_t)gp << lg) + gr) << lg) + gc;
    } else {
      g = ((int64_t)gr << lg) + gc;
    }
    halo[e] = v[g];
  }
  __syncthreads();
  const int64_t pbase = (D == 3) ? ((((int64_t)p0 << lg) + r0) << lg) + c0
                                 : ((int64_t)r0 << lg) + c0;
  for (int pt = tid; pt < TW; pt += 256) {
    const int id = nearest_shift(sS, nS, halo[((PL / 2) * HR + t) * HC + pt + t]);
    int cp[D];
    if constexpr (D == 3) {
      cp[0] = p0;
      cp[1] = r0;
      cp[2] = c0 + pt;
    } else {
      cp[0] = r0;
      cp[1] = c0 + pt;
    }
    const int tj = nd_radius<D>(cp, b, 2);
    spS[pt] = sS[id];
    spP[pt] = ((tj >= 2) ? act2 : act1) + (int64_t)id * M2;
    if (idx_out) idx_out[pbase + pt] = id;
  }
  __syncthreads();

  constexpr int VEC = 2;
  constexpr int SPAN = TW * M2;
  constexpr int TACT = 256 - 256 % M2;
  constexpr int STEP = VEC * TACT;
  constexpr int DP = STEP / M2;
  static_assert(SPAN % VEC == 0 && STEP % M2 == 0, "whole stores, whole points per step");
  if (tid >= TACT) return;
  const int e0 = VEC * tid;
  const int pt0 = e0 / M2;
  int a2[VEC], hoff[VEC], pinc[VEC];
#pragma unroll
  for (int h = 0; h < VEC; ++h) {
    const int e = e0 + h;
    pinc[h] = e / M2 - pt0;
    const int a = e % M2;
    a2[h] = a;
    int rem = a, ho = 0, hm = 1;
#pragma unroll
    for (int i = D - 1; i >= 0; --i) {
      ho += (rem % W2) * hm;
      rem /= W2;
      hm *= (i == D - 1) ? HC : HR;
    }
    hoff[h] = ho + pinc[h];  // halo index = point + hoff
  }
  const int64_t rowbase = pbase * M2;
  int pp = pt0;
  for (int e = e0; e < SPAN; e += STEP, pp += DP) {
    double pv[VEC];
#pragma unroll
    for (int h = 0; h < VEC; ++h) {
      // both radii in the radius-2 layout; a radius-1 row's entries outside
      // its window are (0, 0), giving 0 + 0 * (v - s) = +0
      const int q = pp + pinc[h];
      const double2 ac = spP[q][a2[h]];
      const double va = halo[pp + hoff[h]];
      pv[h] = ac.x + ac.y * (va - spS[q]);
    }
    reinterpret_cast<double2*>(P + rowbase)[e >> 1] = make_double2(pv[0], pv[1]);
  }
}

template <int D, int TW>
hipError_t run_assemble_nd(lsp_problem* p, const double2* act1, int leaf, double* P,
                           int32_t* idx) {
  const int n = p->n;
  if (n % TW != 0) return hipErrorInvalidValue;
  int lg = 0;
  while ((1 << lg) < n) ++lg;
  const dim3 grid(n / TW, n, (D == 3) ? n : 1), blk(256);
  const double2* act2 = reinterpret_cast<const double2*>(p->ws.actab);
  hipLaunchKernelGGL((assemble_nd_kernel<D, TW>), grid, blk, 0, p->stream, p->v, n, lg, p->ws.S,
                     p->ws.nS, act1, act2, leaf, P, idx);
  return hipGetLastError();
}

}  // namespace

namespace lsp {

hipError_t launch_assemble_nd(lsp_problem* p, const double2* act1, int leaf, double* P,
                              int32_t* idx) {
  const int n = p->n;
  if (p->d == 2) {
    switch (n) {
      case 8: return run_assemble_nd<2, 8>(p, act1, leaf, P, idx);
      case 16: return run_assemble_nd<2, 16>(p, act1, leaf, P, idx);
      case 32: return run_assemble_nd<2, 32>(p, act1, leaf, P, idx);
      case 64: return run_assemble_nd<2, 64>(p, act1, leaf, P, idx);
      default: return run_assemble_nd<2, 128>(p, act1, leaf, P, idx);
    }
  }
  switch (n) {
    case 8: return run_assemble_nd<3, 8>(p, act1, leaf, P, idx);
    case 16: return run_assemble_nd<3, 16>(p, act1, leaf, P, idx);
    case 32: return run_assemble_nd<3, 32>(p, act1, leaf, P, idx);
    default: return run_assemble_nd<3, 64>(p, act1, leaf, P, idx);
  }
}

}  // namespace lsp
