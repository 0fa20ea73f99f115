// Green's kernel sums (Sec. 3 and 4.2) at the offsets the Gram matrix needs.
//
// g_s[delta] = (1/N) sum_{k in K} cos(2 pi k.delta/n) / (lambda_k + s) is the
// first column of G_s = (L+s)^-1 and (g_s * g_s)[delta] is the same sum with
// (lambda_k + s)^2, i.e. the inverse DFTs of the symbols 1/(lambda+s) and
// 1/(lambda+s)^2. Eq. (A) only needs delta in [-2t, 2t]^d; both kernels are
// even in every coordinate, so delta in [0, 2t]^d suffices. Instead of the
// paper's full FFT per shift the sums are evaluated directly at those
// (2t+1)^d offsets (a pruned inverse DFT: same numbers, O(N) work per shift
// and no memory traffic):
//   * each axis folds onto k_i in [0, n/2] with weight 1 at 0 and n/2 and 2
//     elsewhere: cw[k][dl] = w(k) cos(2 pi k dl / n);
//   * the summand is symmetric in (k_{d-1}, k_d), so only k_d >= k_{d-1} is
//     visited (half weight on the diagonal) and the two offset axes are
//     symmetrised: g[.., da, db] = sum_kk cw[kk][da] T[db] + cw[kk][db] T[da],
//     with T[dl] = sum_{k_d} cw[k_d][dl] r the inner sum of the thread's row;
//     only the pairs da <= db are accumulated.
// A wave owns 64 consecutive outer indices o = (k_1..k_{d-1}) (one per lane)
// and 64 consecutive values of k_d, whose cw rows are staged in LDS (all loads
// in flight at once) and read as wave-wide broadcasts; work units are uniform,
// so the load is balanced.
// Units write their partial sums, unscaled:
// [g | g*g][leading offsets W^(d-2)][pairs W(W+1)/2].
#include "setup_common.h"

#pragma clang fp contract(off)

namespace {

using lsp::Pow;

template <int D, int W>
struct GreenLayout {
  static constexpr int NP = W * (W + 1) / 2;  // offset pairs da <= db
  static constexpr int WO2 = Pow<D - 2, W>::v;
  static constexpr int NV = 2 * WO2 * NP;     // values per partial
};

// One term of the sums: r = 1/(lambda_k + s) with lambda_k = 4 pi^2 |k|^2
// rounded as "4 pi^2 |k|^2, then + s"; K2 = |k|^2 < 2^31 for n <= 1024.
__device__ __forceinline__ double green_r(int K2, double s) {
  const double lam = lsp::kFourPi2 * (double)K2;
  return lsp::rcp_nr(lam + s);
}

constexpr int kTile = 64;   // outer indices per wave (one per lane)
constexpr int kKTile = 64;  // values of k_d per wave

// kd terms [kd0, kd0 + U) of the inner sums T. MASKED applies the triangle
// weights: 1 above, 1/2 on and 0 below the diagonal k_d = k_{d-1}, 0 for
// padding lanes.
template <int W, int U, bool MASKED>
__device__ __forceinline__ void green_terms(const double* __restrict__ cws, int kd0, int K2o,
                                            int kk, bool valid, double s, double* tg,
                                            double* tq) {
  double r[U], r2[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int kd = kd0 + u;
    const double r0 = green_r(K2o + kd * kd, s);
    if (MASKED) {
      const double wgt = valid ? ((kd > kk) ? 1.0 : ((kd == kk) ? 0.5 : 0.0)) : 0.0;
      r[u] = wgt * r0;
      r2[u] = r[u] * r0;
    } else {
      r[u] = r0;
      r2[u] = r0 * r0;
    }
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const double* c = cws + u * W;
#pragma unroll
    for (int j = 0; j < W; ++j) {
      tg[j] = fma(c[j], r[u], tg[j]);
      tq[j] = fma(c[j], r2[u], tq[j]);
    }
  }
}

// One wave per work unit (shift, 64 consecutive outer indices, KT consecutive
// values of k_d). The prologue forms the shift list from the min/max partials
// (Sec. 4.1); unit (0, 0) publishes it. Units below the diagonal (every
// k_d < k_{d-1}) write zeros.
template <int D, int W, int KT>
__global__ __launch_bounds__(kTile) void green_sums_kernel(
    const double* __restrict__ mm_part, int nreq, double* __restrict__ S_out,
    int* __restrict__ nS_out, double* __restrict__ vrange_out, const double* __restrict__ cw,
    int n, int ktiles, double* __restrict__ part) {
  using Lay = GreenLayout<D, W>;
  constexpr int NP = Lay::NP;
  constexpr int WO2 = Lay::WO2;
  constexpr int NV = Lay::NV;
  constexpr int RCH = 15;  // values reduced per round
  constexpr int SCR = (RCH * (kTile + 1) > lsp::kMaxShifts) ? RCH * (kTile + 1) : lsp::kMaxShifts;
  constexpr int PER = (KT * W + kTile - 1) / kTile;  // staged table values per lane
  __shared__ double cws[KT * W];
  __shared__ double scratch[SCR];  // shift list first, then the reduction buffer
  __shared__ int sNS, sWave[1];
  __shared__ double sRange[2], sRed[2];
  const int lane = threadIdx.x;
  const int si = blockIdx.y;

  const int H = n / 2 + 1;
  const int ot = blockIdx.x / ktiles;
  const int q = blockIdx.x % ktiles;
  int O = 1;
#pragma unroll
  for (int i = 0; i < D - 1; ++i) O *= H;
  const int o = ot * kTile + lane;
  const bool valid = o < O;
  int ko[D - 1];
  {
    int rem = valid ? o : 0;
#pragma unroll
    for (int i = D - 2; i >= 0; --i) {
      ko[i] = rem % H;
      rem /= H;
    }
  }
  int K2o = 0;
#pragma unroll
  for (int i = 0; i < D - 1; ++i) K2o += ko[i] * ko[i];
  const int kk = ko[D - 2];
  const int k_begin = q * KT;
  const int k_end = min(H, k_begin + KT);

  // every table load of the unit is issued before the shift list is formed
  const int cnt = (k_end - k_begin) * W;
  double stage[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) stage[i] = cw[k_begin * W + min(lane + i * kTile, cnt - 1)];
  double ck[W];
#pragma unroll
  for (int j = 0; j < W; ++j) ck[j] = cw[kk * W + j];
  double lead[WO2];
  if constexpr (D == 3) {
#pragma unroll
    for (int x = 0; x < WO2; ++x) lead[x] = cw[ko[0] * W + x];
  } else {
    lead[0] = 1.0;
  }

  lsp::shift_list_block<kTile>(mm_part, nreq, scratch, &sNS, sRange, sWave, sRed);
  const int nS = sNS;
  if (blockIdx.x == 0 && blockIdx.y == 0) {
    for (int i = lane; i < nS; i += kTile) S_out[i] = scratch[i];
    if (lane == 0) {
      *nS_out = nS;
      vrange_out[0] = sRange[0];
      vrange_out[1] = sRange[1];
    }
  }
  if (si >= nS) return;
  const double s = scratch[si];
  double* out = part + ((int64_t)si * gridDim.x + blockIdx.x) * NV;
  if (!__any(valid && kk < k_end)) {
    // the whole tile lies below the diagonal: no contribution
    static_assert(NV <= kTile, "one lane per partial value");
    if (lane < NV) out[lane] = 0.0;
    return;
  }
#pragma unroll
  for (int i = 0; i < PER; ++i)
    if (lane + i * kTile < cnt) cws[lane + i * kTile] = stage[i];
  __syncthreads();  // also orders every read of the shift list before scratch is reused

  double tg[W], tq[W];
#pragma unroll
  for (int j = 0; j < W; ++j) tg[j] = tq[j] = 0.0;
  constexpr int U = 4;
  int kd = k_begin;
  if (__all(valid && kk < k_begin)) {
    // every term of the tile lies above the diagonal: weight 1
    for (; kd + U <= k_end; kd += U)
      green_terms<W, U, false>(cws + (kd - k_begin) * W, kd, K2o, kk, valid, s, tg, tq);
    for (; kd < k_end; ++kd)
      green_terms<W, 1, false>(cws + (kd - k_begin) * W, kd, K2o, kk, valid, s, tg, tq);
  } else {
    for (; kd + U <= k_end; kd += U)
      green_terms<W, U, true>(cws + (kd - k_begin) * W, kd, K2o, kk, valid, s, tg, tq);
    for (; kd < k_end; ++kd)
      green_terms<W, 1, true>(cws + (kd - k_begin) * W, kd, K2o, kk, valid, s, tg, tq);
  }

  // symmetrised accumulation of the offset pairs (da <= db)
  double acc[NV];
#pragma unroll
  for (int x = 0; x < WO2; ++x) {
    int pi = 0;
#pragma unroll
    for (int da = 0; da < W; ++da) {
#pragma unroll
      for (int db = da; db < W; ++db) {
        acc[x * NP + pi] = lead[x] * (ck[da] * tg[db] + ck[db] * tg[da]);
        acc[WO2 * NP + x * NP + pi] = lead[x] * (ck[da] * tq[db] + ck[db] * tq[da]);
        ++pi;
      }
    }
  }

  // wave reduction through LDS in a fixed order, RCH values per round
#pragma unroll
  for (int v0 = 0; v0 < NV; v0 += RCH) {
    if (v0 > 0) __syncthreads();
#pragma unroll
    for (int vv = 0; vv < RCH; ++vv)
      if (v0 + vv < NV) scratch[vv * (kTile + 1) + lane] = acc[v0 + vv];
    __syncthreads();
    if (lane < RCH && v0 + lane < NV) {
      const double* rr = scratch + lane * (kTile + 1);
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
      for (int l = 0; l < kTile; l += 4) {
        s0 += rr[l];
        s1 += rr[l + 1];
        s2 += rr[l + 2];
        s3 += rr[l + 3];
      }
      out[v0 + lane] = (s0 + s1) + (s2 + s3);
    }
  }
}

template <int D, int W>
hipError_t run_green(lsp_problem* p, int num_shifts, int* blocks_out) {
  const int H = p->n / 2 + 1;
  int64_t O = 1;
  for (int i = 0; i < D - 1; ++i) O *= H;
  const int otiles = (int)((O + kTile - 1) / kTile);
  const int ktiles = (H + kKTile - 1) / kKTile;
  const int blocks = otiles * ktiles;
  const size_t need = (size_t)num_shifts * blocks * GreenLayout<D, W>::NV;
  if (need > p->ws.green_part_cap) return hipErrorOutOfMemory;
  *blocks_out = blocks;
  hipLaunchKernelGGL((green_sums_kernel<D, W, kKTile>), dim3(blocks, num_shifts), dim3(kTile), 0,
                     p->stream, p->ws.minmax_part, num_shifts, p->ws.S, p->ws.nS, p->ws.vrange,
                     p->cosT, p->n, ktiles, p->ws.green_part);
  return hipGetLastError();
}

template <int D, int W>
size_t green_need(int n, int shifts) {
  const int H = n / 2 + 1;
  int64_t O = 1;
  for (int i = 0; i < D - 1; ++i) O *= H;
  const int64_t blocks = ((O + kTile - 1) / kTile) * ((H + kKTile - 1) / kKTile);
  return (size_t)shifts * blocks * GreenLayout<D, W>::NV;
}

}  // namespace

namespace lsp {

hipError_t launch_green_sums(lsp_problem* p, int num_shifts, int* blocks) {
  const int W = 2 * p->t + 1;
  if (p->d == 2 && W == 3) return run_green<2, 3>(p, num_shifts, blocks);
  if (p->d == 2 && W == 5) return run_green<2, 5>(p, num_shifts, blocks);
  if (p->d == 2 && W == 7) return run_green<2, 7>(p, num_shifts, blocks);
  if (p->d == 3 && W == 3) return run_green<3, 3>(p, num_shifts, blocks);
  return hipErrorInvalidValue;
}

size_t green_partial_doubles(int d, int n, int t, int shifts) {
  const int W = 2 * t + 1;
  if (d == 2 && W == 3) return green_need<2, 3>(n, shifts);
  if (d == 2 && W == 5) return green_need<2, 5>(n, shifts);
  if (d == 2 && W == 7) return green_need<2, 7>(n, shifts);
  if (d == 3 && W == 3) return green_need<3, 3>(n, shifts);
  return 0;
}

}  // namespace lsp
