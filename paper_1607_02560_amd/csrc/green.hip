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
// A work unit is 64 consecutive outer indices o = (k_1..k_{d-1}) (one per
// lane) and 64 consecutive values of k_d, whose cw rows are staged in LDS (all
// loads in flight at once) and read as wave-wide broadcasts. A block of four
// waves takes one unit for four shifts, so the shift list and the staging are
// shared; units entirely below the diagonal are never launched. Each wave
// reduces its sums over the lanes by recursive halving and writes one
// partial per (shift, unit), unscaled:
// [g | g*g][leading offsets W^(d-2)][pairs W(W+1)/2].
#include <algorithm>
#include <vector>

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

constexpr int kTile = 64;     // outer indices per unit (one per lane)
constexpr int kKTile = 64;    // values of k_d per unit
constexpr int kWaves = 4;     // shifts per block (one wave each)
constexpr int kThreads = 64 * kWaves;
constexpr size_t kResidencyLds = 40 * 1024;  // dynamic LDS per block (unused)

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

// Sum of the P2 values a[] over the 64 lanes by recursive halving: at each
// step a lane keeps one half of its vector and adds the partner's copy of
// that half (partner = lane ^ o). After log2(P2) steps lane l holds value
// l >> (6 - log2 P2) summed over its group of 2^(6 - log2 P2) lanes; the
// remaining steps add across that group. The order is fixed, so the result
// is deterministic.
template <int P2, int O = 32>
__device__ __forceinline__ void halving_sum(double* a, int lane) {
  if constexpr (O >= 1) {
    if constexpr (P2 > 1) {
      constexpr int h = P2 / 2;
      const bool up = (lane & O) != 0;
#pragma unroll
      for (int i = 0; i < h; ++i) {
        const double send = up ? a[i] : a[h + i];
        const double keep = up ? a[h + i] : a[i];
        a[i] = keep + __shfl_xor(send, O);
      }
      halving_sum<h, O / 2>(a, lane);
    } else {
      a[0] += __shfl_xor(a[0], O);
      halving_sum<1, O / 2>(a, lane);
    }
  }
}

constexpr int pow2_at_least(int x) {
  int p = 1;
  while (p < x) p *= 2;
  return p;
}
constexpr int log2_exact(int x) {
  int l = 0;
  while ((1 << l) < x) ++l;
  return l;
}

// One block per (work unit, group of kWaves shifts); wave w handles shift
// kWaves * blockIdx.y + w. A work unit is 64 consecutive outer indices
// o = (k_1..k_{d-1}) (one per lane) and KT consecutive values of k_d; only
// units with a term on or above the diagonal k_d >= k_{d-1} are launched
// (their (outer tile, k tile) pairs come from `units`, built on the host).
// The prologue forms the shift list from the min/max partials (Sec. 4.1) once
// per block and stages the unit's cosine rows in LDS; unit 0 of shift group 0
// publishes S, |S| and (v_min, v_max).
template <int D, int W, int KT>
__global__ __launch_bounds__(kThreads) void green_sums_kernel(
    const double* __restrict__ mm_part, int nreq, double* __restrict__ S_out,
    int* __restrict__ nS_out, double* __restrict__ vrange_out, const double* __restrict__ cw,
    const int* __restrict__ units, int n, double* __restrict__ part) {
  using Lay = GreenLayout<D, W>;
  constexpr int NP = Lay::NP;
  constexpr int WO2 = Lay::WO2;
  constexpr int NV = Lay::NV;
  static_assert(NV <= 64, "one lane per partial value");
  constexpr int P2 = pow2_at_least(NV);
  constexpr int PER = (KT * W + kThreads - 1) / kThreads;  // staged table values per thread
  __shared__ double cws[KT * W];
  __shared__ double sS[lsp::kMaxShifts];
  __shared__ int sNS, sWave[kWaves];
  __shared__ double sRange[2], sRed[2 * kWaves];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wid = tid >> 6;

  const int H = n / 2 + 1;
  const int unit = units[blockIdx.x];
  const int ot = unit >> 16;
  const int q = unit & 0xffff;
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

  // every table load of the block is issued before the shift list is formed
  const int cnt = (k_end - k_begin) * W;
  double stage[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) stage[i] = cw[k_begin * W + min(tid + i * kThreads, cnt - 1)];
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

  lsp::shift_list_block<kThreads>(mm_part, nreq, sS, &sNS, sRange, sWave, sRed);
  const int nS = sNS;
  if (blockIdx.x == 0 && blockIdx.y == 0) {
    for (int i = tid; i < nS; i += kThreads) S_out[i] = sS[i];
    if (tid == 0) {
      *nS_out = nS;
      vrange_out[0] = sRange[0];
      vrange_out[1] = sRange[1];
    }
  }
#pragma unroll
  for (int i = 0; i < PER; ++i)
    if (tid + i * kThreads < cnt) cws[tid + i * kThreads] = stage[i];
  __syncthreads();  // the last barrier of the block: waves are independent below

  const int si = blockIdx.y * kWaves + wid;
  if (si >= nS) return;
  const double s = sS[si];
  double tg[W], tq[W];
#pragma unroll
  for (int j = 0; j < W; ++j) tg[j] = tq[j] = 0.0;
  constexpr int U = 4;
  int kd = k_begin;
  if (__all(valid && kk < k_begin)) {
    // every term of the unit lies above the diagonal: weight 1
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

  // symmetrised accumulation of the offset pairs (da <= db), padded to P2
  double a[P2];
#pragma unroll
  for (int x = 0; x < WO2; ++x) {
    int pi = 0;
#pragma unroll
    for (int da = 0; da < W; ++da) {
#pragma unroll
      for (int db = da; db < W; ++db) {
        a[x * NP + pi] = lead[x] * (ck[da] * tg[db] + ck[db] * tg[da]);
        a[WO2 * NP + x * NP + pi] = lead[x] * (ck[da] * tq[db] + ck[db] * tq[da]);
        ++pi;
      }
    }
  }
#pragma unroll
  for (int i = NV; i < P2; ++i) a[i] = 0.0;
  halving_sum<P2>(a, lane);
  constexpr int G = 6 - log2_exact(P2);  // lanes per value: 2^G
  const int vi = lane >> G;
  if ((lane & ((1 << G) - 1)) == 0 && vi < NV)
    part[((int64_t)si * gridDim.x + blockIdx.x) * NV + vi] = a[0];
}

// Work units with at least one term on or above the diagonal, in
// (outer tile, k tile) order, packed as (ot << 16) | q.
template <int D>
void build_units(int n, std::vector<int>& units) {
  const int H = n / 2 + 1;
  int64_t O = 1;
  for (int i = 0; i < D - 1; ++i) O *= H;
  const int otiles = (int)((O + kTile - 1) / kTile);
  const int ktiles = (H + kKTile - 1) / kKTile;
  units.clear();
  for (int ot = 0; ot < otiles; ++ot) {
    for (int q = 0; q < ktiles; ++q) {
      const int k_end = std::min(H, (q + 1) * kKTile);
      bool any = false;
      for (int l = 0; l < kTile && !any; ++l) {
        const int64_t o = (int64_t)ot * kTile + l;
        if (o < O && (int)(o % H) < k_end) any = true;
      }
      if (any) units.push_back((ot << 16) | q);
    }
  }
}

template <int D, int W>
hipError_t run_green(lsp_problem* p, int num_shifts, int* units_out) {
  const int nunits = p->green_nunits;
  const size_t need = (size_t)num_shifts * nunits * GreenLayout<D, W>::NV;
  if (need > p->ws.green_part_cap || nunits < 1) return hipErrorInvalidValue;
  *units_out = nunits;
  const int groups = (num_shifts + kWaves - 1) / kWaves;
  // The blocks are uniform and all resident at once, so the time is set by
  // the most loaded SIMD. Reserving kResidencyLds bytes of LDS per block (on
  // top of its ~10-12 KB of static LDS) lets at most three blocks share a
  // CU's 160 KB, so no SIMD takes more than three waves.
  hipLaunchKernelGGL((green_sums_kernel<D, W, kKTile>), dim3(nunits, groups), dim3(kThreads),
                     kResidencyLds, p->stream, p->ws.minmax_part, num_shifts, p->ws.S, p->ws.nS, p->ws.vrange,
                     p->cosT, p->green_units, p->n, p->ws.green_part);
  return hipGetLastError();
}

}  // namespace

namespace lsp {

hipError_t launch_green_sums(lsp_problem* p, int num_shifts, int* units) {
  const int W = 2 * p->t + 1;
  if (p->d == 2 && W == 3) return run_green<2, 3>(p, num_shifts, units);
  if (p->d == 2 && W == 5) return run_green<2, 5>(p, num_shifts, units);
  if (p->d == 2 && W == 7) return run_green<2, 7>(p, num_shifts, units);
  if (p->d == 3 && W == 3) return run_green<3, 3>(p, num_shifts, units);
  return hipErrorInvalidValue;
}

void green_units(int d, int n, std::vector<int>& units) {
  if (d == 2) build_units<2>(n, units);
  else build_units<3>(n, units);
}

size_t green_partial_doubles(int d, int n, int t, int shifts) {
  const int W = 2 * t + 1;
  std::vector<int> units;
  green_units(d, n, units);
  const size_t nu = units.size();
  if (d == 2 && W == 3) return shifts * nu * GreenLayout<2, 3>::NV;
  if (d == 2 && W == 5) return shifts * nu * GreenLayout<2, 5>::NV;
  if (d == 2 && W == 7) return shifts * nu * GreenLayout<2, 7>::NV;
  if (d == 3 && W == 3) return shifts * nu * GreenLayout<3, 3>::NV;
  return 0;
}

}  // namespace lsp
