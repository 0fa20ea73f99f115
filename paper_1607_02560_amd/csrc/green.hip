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
constexpr size_t kResidencyLds = 40 * 1024;  // reserved, never accessed: caps residency (run_green)

// kd terms [kd0, kd0 + U) of the inner sums T. MASKED applies the triangle
// weights: 1 above, 1/2 on and 0 below the diagonal k_d = k_{d-1}, 0 for
// padding lanes.
template <int W, int U, bool MASKED>
__device__ __forceinline__ void green_terms(const double* __restrict__ cws, int kd0, int K2o,
                                            int kk, bool valid, double s, double* tg,
                                            double* tq) {
  // all cosine values of the U terms are read before any arithmetic, so the
  // LDS reads overlap each other and the reciprocals
  double c[U][W];
#pragma unroll
  for (int u = 0; u < U; ++u) {
#pragma unroll
    for (int j = 0; j < W; ++j) c[u][j] = cws[u * W + j];
  }
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
#pragma unroll
    for (int j = 0; j < W; ++j) {
      tg[j] = fma(c[u][j], r[u], tg[j]);
      tq[j] = fma(c[u][j], r2[u], tq[j]);
    }
  }
}

// One step of recursive halving on lane bit BIT: of the P2 values a[], the
// lanes with the bit clear keep the lower half and those with it set the
// upper half, each adding the partner's copy of the half it keeps. The
// partner agrees with the lane on every bit used by earlier steps.
template <int P2, int BIT, int SRC>
__device__ __forceinline__ void halving_step(double* a, int lane) {
  constexpr int h = P2 / 2;
  const bool up = (lane >> BIT) & 1;
#pragma unroll
  for (int i = 0; i < h; ++i) {
    const double send = up ? a[i] : a[h + i];
    const double keep = up ? a[h + i] : a[i];
    double recv;
    if constexpr (SRC == 0) recv = lsp::dpp_move<lsp::kDppRowRor8>(send);
    else if constexpr (SRC == 1) recv = lsp::dpp_move<lsp::kDppHalfMirror>(send);
    else if constexpr (SRC == 2) recv = lsp::dpp_move<lsp::kDppQuadXor2>(send);
    else if constexpr (SRC == 3) recv = lsp::dpp_move<lsp::kDppQuadXor1>(send);
    else recv = __shfl_xor(send, 1 << BIT);
    a[i] = keep + recv;
  }
}

// Sum of the P2 (a power of two, 2..64) values a[] over the 64 lanes by
// recursive halving. The in-row steps (bits 3, 2, 1, 0, through DPP) halve
// the largest vectors; the cross-row bits 4 and 5 go last, through LDS
// permutes, when one or two values are left. The order is fixed, so the
// result is deterministic. Returns the index of the value the lane holds
// (the sum over all 64 lanes); lanes that agree on the returned index hold
// the same value.
template <int P2>
__device__ __forceinline__ int halving_sum(double* a, int lane) {
  static_assert(P2 >= 2 && P2 <= 64 && (P2 & (P2 - 1)) == 0, "power of two");
  int idx = 0;
  // bits in step order with their halvings; once one value is left the
  // remaining bits add across lanes
  if constexpr (P2 >= 2) halving_step<P2, 3, 0>(a, lane);
  if constexpr (P2 >= 4) halving_step<P2 / 2, 2, 1>(a, lane);
  if constexpr (P2 >= 8) halving_step<P2 / 4, 1, 2>(a, lane);
  if constexpr (P2 >= 16) halving_step<P2 / 8, 0, 3>(a, lane);
  if constexpr (P2 >= 32) halving_step<P2 / 16, 4, 4>(a, lane);
  if constexpr (P2 >= 64) halving_step<P2 / 32, 5, 4>(a, lane);
  // index: each step's bit selects the upper half, weights P2/2, P2/4, ...
  {
    constexpr int order[6] = {3, 2, 1, 0, 4, 5};
    int w = P2 / 2;
#pragma unroll
    for (int st = 0; st < 6; ++st) {
      if (w >= 1) idx += ((lane >> order[st]) & 1) * w;
      w /= 2;
    }
  }
  // bits not used for halving: plain sums across the lanes that differ in them
  if constexpr (P2 < 2) a[0] += lsp::dpp_move<lsp::kDppRowRor8>(a[0]);
  if constexpr (P2 < 4) a[0] += lsp::dpp_move<lsp::kDppHalfMirror>(a[0]);
  if constexpr (P2 < 8) a[0] += lsp::dpp_move<lsp::kDppQuadXor2>(a[0]);
  if constexpr (P2 < 16) a[0] += lsp::dpp_move<lsp::kDppQuadXor1>(a[0]);
  if constexpr (P2 < 32) a[0] += __shfl_xor(a[0], 16);
  if constexpr (P2 < 64) a[0] += __shfl_xor(a[0], 32);
  return idx;
}

constexpr int pow2_at_least(int x) {
  int p = 1;
  while (p < x) p *= 2;
  return p;
}

// Wavenumbers per axis covered by the tiles: in 2D the Nyquist value
// k = n/2 is left out of the tiling and added as single terms (see below),
// so that every unit holds the same amount of work; in 3D all of [0, n/2].
template <int D>
__host__ __device__ inline int tiled_wavenumbers(int n) {
  return D == 2 ? n / 2 : n / 2 + 1;
}

// One block per (work unit, group of kWaves shifts); wave w handles shift
// kWaves * blockIdx.y + w. A work unit is 64 consecutive outer indices
// o = (k_1..k_{d-1}) (one per lane) and KT consecutive values of k_d; only
// units with a term on or above the diagonal k_d >= k_{d-1} are launched
// (their (outer tile, k tile) pairs come from `units`, built on the host).
// The prologue stages the unit's cosine rows in LDS; the shift list comes
// from the min/max launch before this one.
//
// 2D: with Ht = n/2 tiled wavenumbers, a unit is either wholly above the
// diagonal or a square tile on it. A square tile is summed in full, which
// gives twice the symmetrised triangle sum (the summand is symmetric in
// (k_1, k_2)); a factor 1/2 on its pair sums undoes that. Units in the last
// k tile add the Nyquist column k_2 = n/2 as one more term (weight 1 above
// the diagonal, hence 2 inside a square tile before the 1/2), and the waves
// of unit 0 add the corner (n/2, n/2), whose cosine weights are (-1)^delta.
template <int D, int W, int KT>
__device__ __forceinline__ void green_body(
    int bx, int by, int gx, const double* __restrict__ S, const int* __restrict__ nS_ptr,
    const double* __restrict__ cw, const int* __restrict__ units, int n,
    double* __restrict__ part) {
  using Lay = GreenLayout<D, W>;
  constexpr int NP = Lay::NP;
  constexpr int WO2 = Lay::WO2;
  constexpr int NV = Lay::NV;
  static_assert(NV <= 64 || D == 3, "one lane per partial value (2D)");
  static_assert(D == 3 || KT == kTile, "2D diagonal units must be square tiles");
  constexpr int P2 = pow2_at_least(NV <= 64 ? NV : 64);
  constexpr int PER = (KT * W + kThreads - 1) / kThreads;  // staged table values per thread
  __shared__ double cws[KT * W];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wid = tid >> 6;

  const int Ht = tiled_wavenumbers<D>(n);
  const int nyq = n / 2;
  const int unit = units[bx];
  const int ot = unit >> 16;
  const int q = unit & 0xffff;
  int O = 1;
#pragma unroll
  for (int i = 0; i < D - 1; ++i) O *= Ht;
  const int o = ot * kTile + lane;
  const bool valid = o < O;
  int ko[D - 1];
  {
    int rem = valid ? o : 0;
#pragma unroll
    for (int i = D - 2; i >= 0; --i) {
      ko[i] = rem % Ht;
      rem /= Ht;
    }
  }
  int K2o = 0;
#pragma unroll
  for (int i = 0; i < D - 1; ++i) K2o += ko[i] * ko[i];
  const int kk = ko[D - 2];
  const int k_begin = q * KT;
  const int k_end = min(Ht, k_begin + KT);
  const bool nyq_col = (D == 2) && (k_end == Ht);

  // every table load of the block is issued before any is used
  const int cnt = (k_end - k_begin) * W;
  double stage[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) stage[i] = cw[k_begin * W + min(tid + i * kThreads, cnt - 1)];
  double ck[W], cn[W];
#pragma unroll
  for (int j = 0; j < W; ++j) {
    ck[j] = cw[kk * W + j];
    cn[j] = cw[nyq * W + j];
  }
  double lead[WO2];
  if constexpr (D == 3) {
#pragma unroll
    for (int x = 0; x < WO2; ++x) lead[x] = cw[ko[0] * W + x];
  } else {
    lead[0] = 1.0;
  }

  const int nS = *nS_ptr;
#pragma unroll
  for (int i = 0; i < PER; ++i)
    if (tid + i * kThreads < cnt) cws[tid + i * kThreads] = stage[i];
  __syncthreads();  // the last barrier of the block: waves are independent below

  const int si = by * kWaves + wid;
  if (si >= nS) return;
  const double s = S[si];
  double tg[W], tq[W];
#pragma unroll
  for (int j = 0; j < W; ++j) tg[j] = tq[j] = 0.0;
  constexpr int U = 4;
  int kd = k_begin;
  if (D == 2 || __all(valid && kk < k_begin)) {
    // weight 1 on every term
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
  if constexpr (D == 2) {
    const bool square = (q == ot);
    if (nyq_col) {
      const double wn = square ? 2.0 : 1.0;
      const double r0 = green_r(K2o + nyq * nyq, s);
      const double r1 = wn * r0;
      const double r2 = r1 * r0;
#pragma unroll
      for (int j = 0; j < W; ++j) {
        tg[j] = fma(cn[j], r1, tg[j]);
        tq[j] = fma(cn[j], r2, tq[j]);
      }
    }
    const double half = !valid ? 0.0 : (square ? 0.5 : 1.0);
#pragma unroll
    for (int j = 0; j < W; ++j) ck[j] *= half;
  }

  if constexpr (NV > 64) {
    // 3D with more than 64 values per partial (W = 5: 150): the leading
    // offsets x go in chunks of XC, each chunk one halving sum of its
    // 2 XC NP <= 64 values, laid out [g | g*g][x in chunk][pairs]; the lane
    // holding local value lv writes the global value it stands for.
    constexpr int XC = 64 / (2 * NP);
    constexpr int NCH = (WO2 + XC - 1) / XC;
    static_assert(XC >= 1 && D == 3, "chunked partials");
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
      double a[64];
#pragma unroll
      for (int i = 0; i < 64; ++i) a[i] = 0.0;
#pragma unroll
      for (int xx = 0; xx < XC; ++xx) {
        const int x = ch * XC + xx;
        if (x < WO2) {
          int pi = 0;
#pragma unroll
          for (int da = 0; da < W; ++da) {
#pragma unroll
            for (int db = da; db < W; ++db) {
              a[xx * NP + pi] = lead[x] * (ck[da] * tg[db] + ck[db] * tg[da]);
              a[XC * NP + xx * NP + pi] = lead[x] * (ck[da] * tq[db] + ck[db] * tq[da]);
              ++pi;
            }
          }
        }
      }
      const int lv = halving_sum<64>(a, lane);
      const bool gpart = lv < XC * NP;
      const int loc = gpart ? lv : lv - XC * NP;
      const int x = ch * XC + loc / NP;
      if (loc < XC * NP && x < WO2) {
        const int vi = (gpart ? 0 : WO2 * NP) + x * NP + loc % NP;
        part[((int64_t)si * gx + bx) * NV + vi] = a[0];
      }
    }
    return;
  } else {
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
  const int vi = halving_sum<P2>(a, lane);
  // one writer per value: the lanes holding value vi differ only in the bits
  // not used for halving, the highest log2(64 / P2) of the step order
  constexpr int kUnusedMask = (P2 >= 64) ? 0 : (P2 >= 32) ? 0x20 : (P2 >= 16) ? 0x30
                              : (P2 >= 8) ? 0x31 : (P2 >= 4) ? 0x33 : 0x37;
  if ((lane & kUnusedMask) == 0 && vi < NV) {
    double val = a[0];
    if (D == 2 && bx == 0) {
      // corner (n/2, n/2): pair (da, db) of value vi gets cn[da] cn[db] r
      // (r^2 for the g*g half)
      const int pi = vi % NP;
      int da = 0, rest = pi;
      while (rest >= W - da) {
        rest -= W - da;
        ++da;
      }
      const int db = da + rest;
      // select with constant indices so cn[] stays in registers
      double ca = 0.0, cb = 0.0;
#pragma unroll
      for (int j = 0; j < W; ++j) {
        if (j == da) ca = cn[j];
        if (j == db) cb = cn[j];
      }
      const double r = green_r(2 * nyq * nyq, s);
      const double rr = (vi < NP) ? r : r * r;
      val += (ca * cb) * rr;
    }
    part[((int64_t)si * gx + bx) * NV + vi] = val;
  }
  }
}

// Shift list of a single problem, formed by every block of its Green's-sum
// launch from the min/max partials of the launch before (the same list in
// every block: the same partials through the same fixed-order code); block
// (0, 0) (publish) also writes S, |S| and (v_min, v_max) for the launches
// after. global: the one shift of the non-localized method. (The batched
// launches read the list that the batched shift-list launch formed.)
struct ShiftShared {
  double S[lsp::kMaxShifts];
  double range[2];
  double red[3 * kWaves];
  int nS;
  int wave[kWaves];
};

__device__ __forceinline__ void shift_prologue(ShiftShared& sh, const double* __restrict__ mm_part,
                                               int64_t N, int nreq, int global, bool publish,
                                               double* __restrict__ S_out,
                                               int* __restrict__ nS_out,
                                               double* __restrict__ vrange_out) {
  if (global)
    lsp::global_shift_block<kThreads>(mm_part, N, sh.S, &sh.nS, sh.range, sh.red);
  else
    lsp::shift_list_block<kThreads>(mm_part, nreq, sh.S, &sh.nS, sh.range, sh.wave, sh.red);
  if (publish) {
    for (int i = threadIdx.x; i < sh.nS; i += kThreads) S_out[i] = sh.S[i];
    if (threadIdx.x == 0) {
      *nS_out = sh.nS;
      vrange_out[0] = sh.range[0];
      vrange_out[1] = sh.range[1];
    }
  }
}

template <int D, int W, int KT>
__global__ __launch_bounds__(kThreads) void green_sums_kernel(
    const double* __restrict__ mm_part, int64_t N, int nreq, int global,
    const double* __restrict__ cw, const int* __restrict__ units, int n,
    double* __restrict__ part, double* __restrict__ S_out, int* __restrict__ nS_out,
    double* __restrict__ vrange_out) {
  __shared__ ShiftShared sh;
  shift_prologue(sh, mm_part, N, nreq, global, blockIdx.x == 0 && blockIdx.y == 0, S_out, nS_out,
                 vrange_out);
  green_body<D, W, KT>(blockIdx.x, blockIdx.y, gridDim.x, sh.S, &sh.nS, cw, units, n, part);
}

// one launch for the problems of a batch: block b is unit map[b].y of shift
// group map[b].z of problem map[b].x
template <int D, int W, int KT>
__global__ __launch_bounds__(kThreads) void green_batched_kernel(const lsp::BatchRec* recs,
                                                                 const int4* map) {
  const int4 it = map[blockIdx.x];
  const lsp::BatchRec& r = recs[it.x];
  green_body<D, W, KT>(it.y, it.z, r.nunits, r.S, r.nS, r.cw, r.units, r.n, r.part);
}

// --------------------------------------------------------------------------
// 2D with balanced waves. With Ht = n/2 tiled wavenumbers per axis, KT =
// min(64, Ht) and T = Ht / KT tiles, the work is the upper triangle of
// NU = T (T + 1) / 2 tile pairs (ot <= q, row-major) per shift; one "step" is
// one value of k_2 for the KT values k_1 = 64 ot + lane of a tile pair, so
// every shift holds SPS = NU KT steps and the whole launch nS SPS. The launch
// has a fixed number of waves NWV (a function of n and the requested |S|
// only, so a batched launch partitions a problem exactly as its own launch
// does); wave w takes the R = ceil(nS SPS / NWV) consecutive steps from w R.
// Along its range a lane accumulates the inner sums T[dl] of its k_1 over the
// steps of one row of tile pairs (all pairs of one ot share the lane's k_1;
// the diagonal pair ot = q is summed over its full square with halved
// cosine weights, the summand being symmetric in (k_1, k_2)) and, where the
// row ends, folds them into its pair sums. Where its range leaves a shift (or
// ends) the wave sums the pair sums over its lanes (recursive halving with
// DPP lane moves, a fixed order) and writes them as the partial of (wave w,
// shift s), at slot w + s.
// Slots of one shift are consecutive in w, and slot w + s is unique, since
// each step along the ranges advances w or s. The cosine values and 4 pi^2 k_2^2 of
// a step are wave-uniform (scalar loads). The Nyquist column k_2 = n/2 is one
// extra term of the piece that ends a row's last pair, and the corner
// (n/2, n/2) is added by the wave that holds a shift's first step.
// --------------------------------------------------------------------------

// One term r = 1/(lambda_k + s), lambda_k = 4 pi^2 |k|^2 with |k|^2 exact as a
// double: the roundings of green_r.
__device__ __forceinline__ double green_rd(double K2, double s) {
  const double lam = lsp::kFourPi2 * K2;
  return lsp::rcp_cubic(lam + s);
}

// steps kd0 .. kd0 + U - 1 of a lane's inner sums: weights cws, lam2 the
// per-axis eigenvalues 4 pi^2 k_2^2 of the steps (table), base = 4 pi^2 k_1^2
// + s of the lane (one rounding), so a term costs one add before its
// reciprocal: r = 1/(base + lam2)
template <int W, int U>
__device__ __forceinline__ void green2d_terms(const double* __restrict__ cws,
                                              const double* __restrict__ lam2, double base,
                                              double* tg, double* tq) {
  double c[U][W], r[U], r2[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
#pragma unroll
    for (int j = 0; j < W; ++j) c[u][j] = cws[u * W + j];
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    r[u] = lsp::rcp_cubic(base + lam2[u]);
    r2[u] = r[u] * r[u];
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
#pragma unroll
    for (int j = 0; j < W; ++j) {
      tg[j] = fma(c[u][j], r[u], tg[j]);
      tq[j] = fma(c[u][j], r2[u], tq[j]);
    }
  }
}

template <int W>
struct Green2d {
  static constexpr int NP = GreenLayout<2, W>::NP;
  static constexpr int NV = GreenLayout<2, W>::NV;
  static constexpr int P2 = pow2_at_least(NV);
};

template <int W>
__device__ __forceinline__ void green2d_body(int wave, int nwv, const double* __restrict__ S,
                                             const int* __restrict__ nS_ptr,
                                             const double* __restrict__ cw, int n,
                                             double* __restrict__ part) {
  using G = Green2d<W>;
  constexpr int NP = G::NP, NV = G::NV, P2 = G::P2;
  constexpr int U = 4;
  const int lane = threadIdx.x & 63;
  const int Ht = n / 2;
  const int H = Ht + 1;
  const double* cwh = cw + H * W;   // halved weights (diagonal tile pairs)
  const double* lam2 = cw + 2 * H * W;  // 4 pi^2 k^2, k in [0, n/2]
  const int KT = Ht < kTile ? Ht : kTile;
  const int T = Ht / KT;
  const int NU = T * (T + 1) / 2;
  const int SPS = NU * KT;
  const int nS = *nS_ptr;
  const int total = nS * SPS;
  const int R = (total + nwv - 1) / nwv;
  int g = wave * R;
  const int gend = min(g + R, total);
  if (g >= gend) return;
  const int nyq = n / 2;
  double cn[W];
#pragma unroll
  for (int j = 0; j < W; ++j) cn[j] = cw[nyq * W + j];
  const bool valid = lane < KT;
  // KT is a power of two (n is): the step's pair and position within it by
  // shifts; the shift index advances with g (each range after the first
  // starts at a shift boundary)
  const int kts = __builtin_ctz(KT);
  int si = g / SPS;
  for (; g < gend; ++si) {
    const int send = min(gend, (si + 1) * SPS);
    const double s = S[si];
    double a[P2];
#pragma unroll
    for (int i = 0; i < P2; ++i) a[i] = 0.0;
    const bool corner = (g == si * SPS);
    while (g < send) {
      // the row of tile pairs (ot, q >= ot) holding step g
      const int rem = g - si * SPS;
      const int u = rem >> kts;
      int ot = 0, base = 0;
      while (u >= base + (T - ot)) {
        base += T - ot;
        ++ot;
      }
      const int rstop = min(send, si * SPS + (base + T - ot) * KT);
      const int k1 = ot * KT + (valid ? lane : 0);
      const double lbase = fma(lsp::kFourPi2, (double)(k1 * k1), s);
      // the lane's cosine row for the fold, loaded before the row's terms so
      // that its latency overlaps them
      double ck[W];
#pragma unroll
      for (int j = 0; j < W; ++j) ck[j] = valid ? cw[k1 * W + j] : 0.0;
      double tg[W], tq[W];
#pragma unroll
      for (int j = 0; j < W; ++j) tg[j] = tq[j] = 0.0;
      while (g < rstop) {
        const int rr = g - si * SPS;
        const int uu = rr >> kts;
        const int kk = rr & (KT - 1);
        const int q = ot + (uu - base);
        const int ustop = min(rstop, g - kk + KT);
        const double* tab = (q == ot) ? cwh : cw;
        int kd = q * KT + kk;
        const int kd_end = kd + (ustop - g);
        for (; kd + U <= kd_end; kd += U)
          green2d_terms<W, U>(tab + kd * W, lam2 + kd, lbase, tg, tq);
        for (; kd < kd_end; ++kd) green2d_terms<W, 1>(tab + kd * W, lam2 + kd, lbase, tg, tq);
        if (q == T - 1 && ustop - g + kk == KT) {
          // the Nyquist column k_2 = n/2, weight 1 (a diagonal pair's full
          // square counts it twice, then halves)
          const double r0 = lsp::rcp_cubic(lbase + lam2[nyq]);
          const double r2 = r0 * r0;
#pragma unroll
          for (int j = 0; j < W; ++j) {
            tg[j] = fma(cn[j], r0, tg[j]);
            tq[j] = fma(cn[j], r2, tq[j]);
          }
        }
        g = ustop;
      }
      int pi = 0;
#pragma unroll
      for (int da = 0; da < W; ++da) {
#pragma unroll
        for (int db = da; db < W; ++db) {
          a[pi] = fma(ck[da], tg[db], fma(ck[db], tg[da], a[pi]));
          a[NP + pi] = fma(ck[da], tq[db], fma(ck[db], tq[da], a[NP + pi]));
          ++pi;
        }
      }
    }
    if (corner && lane == 0) {
      // the corner (n/2, n/2) once per shift: pair (da, db) gets cn[da] cn[db] r
      // (r^2 for the g*g half)
      const double r = green_rd((double)(2 * nyq * nyq), s);
      int pi = 0;
#pragma unroll
      for (int da = 0; da < W; ++da) {
#pragma unroll
        for (int db = da; db < W; ++db) {
          a[pi] += (cn[da] * cn[db]) * r;
          a[NP + pi] += (cn[da] * cn[db]) * (r * r);
          ++pi;
        }
      }
    }
    // sum over the lanes by recursive halving (a fixed order); one writer
    // per value: the lanes holding value vi differ only in the bits the
    // halving did not use
    const int vi = halving_sum<P2>(a, lane);
    constexpr int kUnusedMask = (P2 >= 64) ? 0 : (P2 >= 32) ? 0x20 : (P2 >= 16) ? 0x30
                                : (P2 >= 8) ? 0x31 : (P2 >= 4) ? 0x33 : 0x37;
    if ((lane & kUnusedMask) == 0 && vi < NV) part[((int64_t)wave + si) * NV + vi] = a[0];
  }
}

template <int W>
__global__ __launch_bounds__(kThreads) void green2d_kernel(
    int nwv, const double* __restrict__ mm_part, int64_t N, int nreq, int global,
    const double* __restrict__ cw, int n, double* __restrict__ part, double* __restrict__ S_out,
    int* __restrict__ nS_out, double* __restrict__ vrange_out) {
  __shared__ ShiftShared sh;
  shift_prologue(sh, mm_part, N, nreq, global, blockIdx.x == 0 && blockIdx.y == 0, S_out, nS_out,
                 vrange_out);
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wave = blockIdx.x * kWaves + wid;
  green2d_body<W>(wave, nwv, sh.S, &sh.nS, cw, n, part);
}

// one launch for the problems of a batch: block b holds waves 4 map[b].y ..
// 4 map[b].y + 3 of problem map[b].x
template <int W>
__global__ __launch_bounds__(kThreads) void green2d_batched_kernel(const lsp::BatchRec* recs,
                                                                   const int4* map) {
  const int4 it = map[blockIdx.x];
  const lsp::BatchRec& r = recs[it.x];
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wave = it.y * kWaves + wid;
  green2d_body<W>(wave, r.gwaves, r.S, r.nS, r.cw, r.n, r.part);
}

// Work units with at least one term on or above the diagonal, in
// (outer tile, k tile) order, packed as (ot << 16) | q.
template <int D>
void build_units(int n, std::vector<int>& units) {
  const int Ht = tiled_wavenumbers<D>(n);
  int64_t O = 1;
  for (int i = 0; i < D - 1; ++i) O *= Ht;
  const int otiles = (int)((O + kTile - 1) / kTile);
  const int ktiles = (Ht + kKTile - 1) / kKTile;
  units.clear();
  for (int ot = 0; ot < otiles; ++ot) {
    for (int q = 0; q < ktiles; ++q) {
      const int k_end = std::min(Ht, (q + 1) * kKTile);
      bool any = false;
      for (int l = 0; l < kTile && !any; ++l) {
        const int64_t o = (int64_t)ot * kTile + l;
        if (o < O && (int)(o % Ht) < k_end) any = true;
      }
      if (any) units.push_back((ot << 16) | q);
    }
  }
}

// LDS reserved (never accessed) per 2D block so that the blocks spread evenly
// over the CUs. The blocks are uniform and all resident at once, so the time
// is set by the most loaded SIMD. Their VGPRs let three blocks share a CU;
// where two per CU are wanted (CUs < blocks <= 2 CUs), a total of 64 KB of
// LDS per block (of a CU's 160 KB) lets no CU take a third.
size_t green2d_residency_lds(int blocks, int cus) {
  if (cus <= 0 || blocks <= cus || blocks > 2 * cus) return 0;
  return 64 * 1024 - sizeof(ShiftShared);
}

template <int D, int W>
hipError_t run_green(const lsp_problem* p, int num_shifts, bool global) {
  if constexpr (D == 2) {
    const int nwv = lsp::green2d_waves(p->n, num_shifts, p->tune[LSP_TUNE_GREEN_WAVES]);
    const size_t need = (size_t)(nwv + num_shifts) * GreenLayout<2, W>::NV;
    if (need > p->ws.green_part_cap) return hipErrorInvalidValue;
    const int blocks = nwv / kWaves;
    hipLaunchKernelGGL((green2d_kernel<W>), dim3(blocks), dim3(kThreads),
                       green2d_residency_lds(blocks, p->cus), p->stream, nwv, p->ws.minmax_part,
                       p->N, num_shifts, (int)global, p->cosT, p->n, p->ws.green_part, p->ws.S,
                       p->ws.nS, p->ws.vrange);
  } else {
    const int nunits = p->green_nunits;
    const size_t need = (size_t)num_shifts * nunits * GreenLayout<D, W>::NV;
    if (need > p->ws.green_part_cap || nunits < 1) return hipErrorInvalidValue;
    const int groups = (num_shifts + kWaves - 1) / kWaves;
    // The blocks are uniform and all resident at once, so the time is set by
    // the most loaded SIMD. Reserving kResidencyLds bytes of LDS per block (on
    // top of its ~10-12 KB of static LDS) lets at most three blocks share a
    // CU's 160 KB, so no SIMD takes more than three waves.
    hipLaunchKernelGGL((green_sums_kernel<D, W, kKTile>), dim3(nunits, groups), dim3(kThreads),
                       kResidencyLds, p->stream, p->ws.minmax_part, p->N, num_shifts,
                       (int)global, p->cosT, p->green_units, p->n, p->ws.green_part, p->ws.S,
                       p->ws.nS, p->ws.vrange);
  }
  return hipGetLastError();
}

}  // namespace

namespace lsp {

int green2d_waves(int n, int num_shifts, int max_waves) {
  const int Ht = n / 2;
  const int KT = Ht < kTile ? Ht : kTile;
  const int T = Ht / KT;
  const int64_t steps = (int64_t)num_shifts * (T * (T + 1) / 2) * KT;
  // at least 32 steps per wave (the per-piece reduction stays a small part
  // of a wave's work), by default at most 2048 waves (two per SIMD of a
  // 256-CU part; up to 3072 on request), a whole number of 4-wave blocks
  int64_t w = (steps + 31) / 32;
  const int64_t cap = (max_waves > 0 && max_waves <= 3072) ? max_waves : 2048;
  w = std::max<int64_t>(kWaves, std::min<int64_t>(cap, w));
  return (int)((w + kWaves - 1) / kWaves * kWaves);
}

int green2d_sps(int n) {
  const int Ht = n / 2;
  const int KT = Ht < kTile ? Ht : kTile;
  const int T = Ht / KT;
  return (T * (T + 1) / 2) * KT;
}

hipError_t launch_green_batched(int d, int t, const BatchRec* recs, const int4* map, int blocks,
                                hipStream_t s) {
  const int W = 2 * t + 1;
#define LSP_GREEN2_B(W_)                                                                  \
  if (d == 2 && W == W_) {                                                                \
    hipLaunchKernelGGL((green2d_batched_kernel<W_>), dim3(blocks), dim3(kThreads), 0, s,  \
                       recs, map);                                                        \
    return hipGetLastError();                                                             \
  }
  LSP_GREEN2_B(3)
  LSP_GREEN2_B(5)
  LSP_GREEN2_B(7)
#undef LSP_GREEN2_B
  if (d == 3 && W == 3) {
    hipLaunchKernelGGL((green_batched_kernel<3, 3, kKTile>), dim3(blocks), dim3(kThreads),
                       kResidencyLds, s, recs, map);
    return hipGetLastError();
  }
  return hipErrorInvalidValue;
}

int green_shift_groups(int num_shifts) { return (num_shifts + kWaves - 1) / kWaves; }

hipError_t launch_green_sums(lsp_problem* p, int num_shifts, bool global) {
  const int W = 2 * p->t + 1;
  if (p->d == 2 && W == 3) return run_green<2, 3>(p, num_shifts, global);
  if (p->d == 2 && W == 5) return run_green<2, 5>(p, num_shifts, global);
  if (p->d == 2 && W == 7) return run_green<2, 7>(p, num_shifts, global);
  if (p->d == 3 && W == 3) return run_green<3, 3>(p, num_shifts, global);
  if (p->d == 3 && W == 5) return run_green<3, 5>(p, num_shifts, global);
  return hipErrorInvalidValue;
}

void green_units(int d, int n, std::vector<int>& units) {
  if (d == 2) build_units<2>(n, units);
  else build_units<3>(n, units);
}

size_t green_partial_doubles(int d, int n, int t, int shifts) {
  const int W = 2 * t + 1;
  if (d == 2) {
    // room for the largest wave count a tuning may ask for
    const size_t slots = (size_t)green2d_waves(n, shifts, 3072) + shifts;
    if (W == 3) return slots * GreenLayout<2, 3>::NV;
    if (W == 5) return slots * GreenLayout<2, 5>::NV;
    if (W == 7) return slots * GreenLayout<2, 7>::NV;
    return 0;
  }
  std::vector<int> units;
  green_units(d, n, units);
  const size_t nu = units.size();
  if (W == 3) return shifts * nu * GreenLayout<3, 3>::NV;
  if (W == 5) return shifts * nu * GreenLayout<3, 5>::NV;
  return 0;
}

}  // namespace lsp
