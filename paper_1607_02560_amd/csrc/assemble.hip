// Per-point work of the localized sparsifying preconditioner (Sec. 4.1):
//   assemble_kernel  s_j and the row P[j, mu_j] = alpha_{s_j} + C_{s_j} (v[mu_j] - s_j)
//   c_apply_kernel   z = C r, the first half of the preconditioner P^-1 C of eq. (PC)
#include "setup_common.h"

// The P row formula is evaluated with one rounding per operation.
#pragma clang fp contract(off)

namespace {

using lsp::kBatchLdsTile;
using lsp::nearest_shift;
using lsp::Pow;

// --------------------------------------------------------------------------
// Per-point assignment and P rows.
// A block owns TR x TW points (TR rows of axis d-2, TW columns of axis d-1,
// one plane of axis 0 in 3D); small tiles keep many blocks in flight, which
// is what this store-bound kernel needs.
//   1. The potential on the tile plus a halo of t in every direction and the
//      shift list are staged in LDS.
//   2. Each point gets idx_j = argmin_i |S_i - v_j| (S is sorted: the two
//      neighbours of the insertion point are compared, ties to the lower index).
//   3. The tile's P rows are TR contiguous spans of TW*m entries, written in
//      steps of a whole number of points; thread k writes entries
//      VEC k .. VEC k + VEC-1 of each step with one 16-byte store (2 doubles,
//      or 4 floats for FP32 storage), evaluating
//      P[j, a] = alpha_{s_j}[a] + C_{s_j}[a] (v[j + a] - s_j) for each in
//      FP64 with one rounding per operation (then one rounding to FP32).
// --------------------------------------------------------------------------
template <int D, int W, int TR, int TW, typename PT>
__device__ __forceinline__ void assemble_body(
    int bx, int by, int bz, const double* __restrict__ v, int n, const double* __restrict__ S,
    const int* __restrict__ nS_ptr, const double2* __restrict__ actab, PT* __restrict__ P,
    int32_t* __restrict__ idx_out) {
  constexpr int t = (W - 1) / 2;
  constexpr int M = Pow<D, W>::v;
  constexpr int PL = (D == 3) ? W : 1;  // halo planes
  constexpr int HR = TR + 2 * t;
  constexpr int HC = TW + 2 * t;
  __shared__ double halo[PL * HR * HC];
  __shared__ double sS[lsp::kMaxShifts];
  __shared__ int spM[TR * TW];     // per point: M times its shift index
  __shared__ double spS[TR * TW];  // per point: its shift s_j
  __shared__ int soff[M];
  const int tid = threadIdx.x;
  const int nS = *nS_ptr;
  const int c0 = bx * TW;
  const int r0 = by * TR;
  const int p0 = (D == 3) ? bz : 0;
  const int mask = n - 1;

  for (int i = tid; i < nS; i += 256) sS[i] = S[i];
  for (int a = tid; a < M; a += 256) {
    if constexpr (D == 3) {
      soff[a] = ((a / (W * W)) * HR + (a / W) % W) * HC + a % W;
    } else {
      soff[a] = (a / W) * HC + a % W;
    }
  }
  for (int e = tid; e < PL * HR * HC; e += 256) {
    const int hc = e % HC;
    const int hr = (e / HC) % HR;
    const int hp = e / (HC * HR);
    const int gc = (c0 - t + hc) & mask;
    const int gr = (r0 - t + hr) & mask;
    int64_t g;
    if constexpr (D == 3) {
      const int gp = (p0 - t + hp) & mask;
      g = ((int64_t)gp * n + gr) * n + gc;
    } else {
      g = (int64_t)gr * n + gc;
    }
    halo[e] = v[g];
  }
  __syncthreads();

  for (int pt = tid; pt < TR * TW; pt += 256) {
    const int r = pt / TW, c = pt % TW;
    const int best = nearest_shift(sS, nS, halo[((PL / 2) * HR + r + t) * HC + c + t]);
    spM[pt] = best * M;
    spS[pt] = sS[best];
    if (idx_out) {
      const int64_t g = (D == 3) ? (((int64_t)p0 * n + r0 + r) * n + c0 + c)
                                 : ((int64_t)(r0 + r) * n + c0 + c);
      idx_out[g] = best;
    }
  }
  __syncthreads();

  // VEC entries per 16-byte store: 2 doubles or 4 floats (TW is a multiple of 4).
  // The span of TR * TW * M entries (TR > 1 only with TW = n, so that the
  // tile's rows follow each other in P) is written in steps of STEP entries
  // by the first TACT = 256 - 256 % M threads, so that a step is a whole
  // number DP of points: thread k's store always covers the same VEC offsets
  // (entries VEC k .. VEC k + VEC - 1 of a step, possibly reaching into the
  // next point), and their offsets, halo positions and point increments are
  // worked out once. Per entry the loop then reads the point's shift (row
  // base and value, both in LDS), one alpha/C pair and one halo value.
  static_assert(TR == 1 || D == 3, "multi-row tiles: 3D rows of n points");
  constexpr int VEC = 16 / (int)sizeof(PT);
  constexpr int SPAN = TR * TW * M;
  constexpr int TACT = 256 - 256 % M;
  constexpr int STEP = VEC * TACT;
  constexpr int DP = STEP / M;
  static_assert(SPAN % VEC == 0 && STEP % M == 0, "whole stores, whole points per step");
  if (tid >= TACT) return;
  const int e0 = VEC * tid;
  const int pt0 = e0 / M;
  int aoff[VEC], hoff[VEC], pinc[VEC];
#pragma unroll
  for (int h = 0; h < VEC; ++h) {
    const int e = e0 + h;
    pinc[h] = e / M - pt0;
    aoff[h] = e % M;
    hoff[h] = soff[aoff[h]] + pinc[h];  // halo index = point + hoff
  }
  const int64_t rowbase = (D == 3) ? ((((int64_t)p0 * n + r0) * n + c0) * M)
                                   : (((int64_t)r0 * n + c0) * M);
  int pp = pt0;
  for (int e = e0; e < SPAN; e += STEP, pp += DP) {
    double outv[VEC];
#pragma unroll
    for (int h = 0; h < VEC; ++h) {
      const int q = pp + pinc[h];
      const double s = spS[q];
      const double2 ac = actab[spM[q] + aoff[h]];
      // point q sits in halo row q / TW (TW is a power of two), whose start
      // is 2t further on per row than in a single-row tile
      const double va = halo[pp + hoff[h] + (TR > 1 ? (q / TW) * (2 * t) : 0)];
      outv[h] = ac.x + ac.y * (va - s);
    }
    if constexpr (VEC == 2) {
      reinterpret_cast<double2*>(P + rowbase)[e >> 1] = make_double2(outv[0], outv[1]);
    } else {
      // FP32 storage: each entry is the FP64 value rounded once to nearest
      reinterpret_cast<float4*>(P + rowbase)[e >> 2] =
          make_float4((float)outv[0], (float)outv[1], (float)outv[2], (float)outv[3]);
    }
  }
}

template <int D, int W, int TR, int TW, typename PT>
__global__ __launch_bounds__(256) void assemble_kernel(
    const double* __restrict__ v, int n, const double* __restrict__ S,
    const int* __restrict__ nS_ptr, const double2* __restrict__ actab, PT* __restrict__ P,
    int32_t* __restrict__ idx_out) {
  assemble_body<D, W, TR, TW, PT>(blockIdx.x, blockIdx.y, blockIdx.z, v, n, S, nS_ptr, actab, P,
                                  idx_out);
}

// 2D assembly with the shift tables in LDS. The (alpha, C) gathers of the
// kernel above go through L1 (16 B per entry, spread over the points' shift
// rows), which bounds it above its store floor in the FP32 form. Here a
// block owns TR rows of TW points and first copies the nS x M table into LDS
// (kActLds pairs at most), so the per-entry gathers read LDS; the copy is
// amortised over the TR rows. Same stores, same arithmetic, same rows.
using lsp::kActLds;

template <int W, int TR, int TW, typename PT, int ACT = kActLds>
__device__ __forceinline__ void assemble_lds_body(
    int bx, int by, const double* __restrict__ v, int n, const double* __restrict__ S,
    const int* __restrict__ nS_ptr, const double2* __restrict__ actab, PT* __restrict__ P,
    int32_t* __restrict__ idx_out) {
  constexpr int t = (W - 1) / 2;
  constexpr int M = W * W;
  constexpr int HR = TR + 2 * t;
  constexpr int HC = TW + 2 * t;
  __shared__ double halo[HR * HC];
  __shared__ double sS[ACT / M];  // nS <= ACT / M on this path
  __shared__ double2 sAct[ACT];
  __shared__ int spM[TR * TW];
  __shared__ double spS[TR * TW];
  __shared__ int soff[M];
  const int tid = threadIdx.x;
  const int nS = *nS_ptr;
  const int c0 = bx * TW;
  const int r0 = by * TR;
  const int mask = n - 1;
  for (int i = tid; i < nS; i += 256) sS[i] = S[i];
  for (int i = tid; i < nS * M; i += 256) sAct[i] = actab[i];
  for (int a = tid; a < M; a += 256) soff[a] = (a / W) * HC + a % W;
  for (int e = tid; e < HR * HC; e += 256) {
    const int hc = e % HC, hr = e / HC;
    halo[e] = v[(int64_t)((r0 - t + hr) & mask) * n + ((c0 - t + hc) & mask)];
  }
  __syncthreads();
  for (int pt = tid; pt < TR * TW; pt += 256) {
    const int r = pt / TW, c = pt % TW;
    const int best = nearest_shift(sS, nS, halo[(r + t) * HC + c + t]);
    spM[pt] = best * M;
    spS[pt] = sS[best];
    if (idx_out) idx_out[(int64_t)(r0 + r) * n + c0 + c] = best;
  }
  __syncthreads();
  // whole-point store steps as in assemble_body, once per row of the tile
  constexpr int VEC = 16 / (int)sizeof(PT);
  constexpr int SPAN = TW * M;
  constexpr int TACT = 256 - 256 % M;
  constexpr int STEP = VEC * TACT;
  constexpr int DP = STEP / M;
  static_assert(SPAN % VEC == 0 && STEP % M == 0, "whole stores, whole points per step");
  if (tid >= TACT) return;
  const int e0 = VEC * tid;
  const int pt0 = e0 / M;
  int aoff[VEC], hoff[VEC], pinc[VEC];
#pragma unroll
  for (int h = 0; h < VEC; ++h) {
    const int e = e0 + h;
    pinc[h] = e / M - pt0;
    aoff[h] = e % M;
    hoff[h] = soff[aoff[h]] + pinc[h];
  }
#pragma unroll 1
  for (int rr = 0; rr < TR; ++rr) {
    PT* Prow = P + ((int64_t)(r0 + rr) * n + c0) * M;
    const int qb = rr * TW;       // the row's first point in the tile
    const int hb = rr * HC;       // its halo row
    int pp = pt0;
    for (int e = e0; e < SPAN; e += STEP, pp += DP) {
      double outv[VEC];
#pragma unroll
      for (int h = 0; h < VEC; ++h) {
        const int q = qb + pp + pinc[h];
        const double s = spS[q];
        const double2 ac = sAct[spM[q] + aoff[h]];
        const double va = halo[hb + pp + hoff[h]];
        outv[h] = ac.x + ac.y * (va - s);
      }
      if constexpr (VEC == 2) {
        reinterpret_cast<double2*>(Prow)[e >> 1] = make_double2(outv[0], outv[1]);
      } else {
        reinterpret_cast<float4*>(Prow)[e >> 2] =
            make_float4((float)outv[0], (float)outv[1], (float)outv[2], (float)outv[3]);
      }
    }
  }
}

template <int W, int TR, int TW, typename PT>
__global__ __launch_bounds__(256) void assemble_lds_kernel(
    const double* __restrict__ v, int n, const double* __restrict__ S,
    const int* __restrict__ nS_ptr, const double2* __restrict__ actab, PT* __restrict__ P,
    int32_t* __restrict__ idx_out) {
  assemble_lds_body<W, TR, TW, PT>(blockIdx.x, blockIdx.y, v, n, S, nS_ptr, actab, P, idx_out);
}

// the same for the problems of a batch: block b is tile (map[b].y, map[b].z)
// of problem map[b].x
template <int W, int TR, int TW, typename PT>
__global__ __launch_bounds__(256) void assemble_lds_batched_kernel(const lsp::BatchRec* recs,
                                                                   const int4* map) {
  const int4 it = map[blockIdx.x];
  const lsp::BatchRec& r = recs[it.x];
  assemble_lds_body<W, TR, TW, PT, lsp::kBatchActLds>(it.y, it.z, r.v, r.n, r.S, r.nS,
                                                      reinterpret_cast<const double2*>(r.actab),
                                                      static_cast<PT*>(r.P), r.idx);
}

// one launch for the problems of a batch: block b is tile (map[b].y, map[b].z,
// map[b].w) of problem map[b].x
template <int D, int W, int TR, int TW, typename PT>
__global__ __launch_bounds__(256) void assemble_batched_kernel(const lsp::BatchRec* recs,
                                                               const int4* map) {
  const int4 it = map[blockIdx.x];
  const lsp::BatchRec& r = recs[it.x];
  assemble_body<D, W, TR, TW, PT>(it.y, it.z, it.w, r.v, r.n, r.S, r.nS,
                                  reinterpret_cast<const double2*>(r.actab),
                                  static_cast<PT*>(r.P), r.idx);
}

// --------------------------------------------------------------------------
// C-apply: z = C r, (C r)_j = sum_a C_{s_j}[a] r[(j + a) mod n] (eq. PC), complex r.
// Same tiling as assemble_kernel; s_j is recomputed from v and S exactly as
// the setup assigned it, so no per-point state is kept between calls. After a
// learned setup the C rows are per point (Crows [N][m]) instead; after a
// per-point-radius setup (leaf > 0) a point of radius 1 takes its row from
// the radius-1 table C1 (zero outside mu_0^1).
// --------------------------------------------------------------------------
// LC: the shift table C (nS x m <= kCApplyLds values, nS <= kCApplyShifts)
// is copied into LDS with the halo, so that a point's row is read from LDS
// and the only global round trip before the sums is the one of the halo
// (the point's v is loaded with it).
constexpr int kCApplyShifts = 128;
constexpr int kCApplyLds = 2048;

template <int D, int W, int TR, int TW, bool LC>
__global__ __launch_bounds__(256) void c_apply_kernel(const double2* __restrict__ rvec,
                                                      const double* __restrict__ v, int n,
                                                      const double* __restrict__ S,
                                                      const int* __restrict__ nS_ptr,
                                                      const double* __restrict__ Ctab,
                                                      const double* __restrict__ Crows,
                                                      const double* __restrict__ C1, int leaf,
                                                      double2* __restrict__ z) {
  constexpr int t = (W - 1) / 2;
  constexpr int M = Pow<D, W>::v;
  constexpr int PL = (D == 3) ? W : 1;
  constexpr int HR = TR + 2 * t;
  constexpr int HC = TW + 2 * t;
  static_assert(TR * TW <= 256, "one point per thread");
  __shared__ double2 halo[PL * HR * HC];
  __shared__ double sS[LC ? kCApplyShifts : lsp::kMaxShifts];
  __shared__ double sC[LC ? kCApplyLds : 1];
  const int tid = threadIdx.x;
  const int nS = *nS_ptr;
  const int c0 = blockIdx.x * TW;
  const int r0 = blockIdx.y * TR;
  const int p0 = (D == 3) ? (int)blockIdx.z : 0;
  const int mask = n - 1;
  // this thread's point (if any) and its potential, loaded with the halo
  const bool has_pt = tid < TR * TW;
  const int pr = tid / TW, pc = tid % TW;
  const int64_t gpt = (D == 3) ? (((int64_t)p0 * n + r0 + pr) * n + c0 + pc)
                               : ((int64_t)(r0 + pr) * n + c0 + pc);
  const double vpt = has_pt ? v[gpt] : 0.0;
  for (int i = tid; i < nS; i += 256) sS[i] = S[i];
  if constexpr (LC) {
    for (int i = tid; i < nS * M; i += 256) sC[i] = Ctab[i];
  }
  for (int e = tid; e < PL * HR * HC; e += 256) {
    const int hc = e % HC;
    const int hr = (e / HC) % HR;
    const int hp = e / (HC * HR);
    const int gc = (c0 - t + hc) & mask;
    const int gr = (r0 - t + hr) & mask;
    int64_t g;
    if constexpr (D == 3) {
      const int gp = (p0 - t + hp) & mask;
      g = ((int64_t)gp * n + gr) * n + gc;
    } else {
      g = (int64_t)gr * n + gc;
    }
    halo[e] = rvec[g];
  }
  __syncthreads();
  if (has_pt) {
    const int r = pr, c = pc;
    const int64_t g = gpt;
    const double* crow;
    const double* crow1 = nullptr;  // radius-1 row of a per-point-radius setup
    if (!LC && Crows) {
      crow = Crows + g * M;  // per-point rows of a learned setup
    } else {
      const int id = nearest_shift(sS, nS, vpt);
      if constexpr (LC) crow = sC + id * M;
      else crow = Ctab + (int64_t)id * M;
      if constexpr (W == 5 && !LC) {
        if (leaf > 0) {
          int cp[D];
          if constexpr (D == 3) {
            cp[0] = p0;
            cp[1] = r0 + r;
            cp[2] = c0 + c;
          } else {
            cp[0] = r0 + r;
            cp[1] = c0 + c;
          }
          if (lsp::nd_radius<D>(cp, leaf, 2) < 2) crow1 = C1 + (int64_t)id * Pow<D, 3>::v;
        }
      }
    }
    double zr = 0.0, zi = 0.0;
    // the row sum for a coefficient rule coef(a, da); two instances below,
    // so that the uniform loop keeps its loads free of branches
    auto row_sum = [&](auto coef) {
#pragma unroll
      for (int a = 0; a < M; ++a) {
        int da[D];
        int rem = a;
#pragma unroll
        for (int k = D - 1; k >= 0; --k) {
          da[k] = rem % W - t;
          rem /= W;
        }
        int hp = 0, hr, hc;
        if constexpr (D == 3) {
          hp = t + da[0];
          hr = r + t + da[1];
          hc = c + t + da[2];
        } else {
          hr = r + t + da[0];
          hc = c + t + da[1];
        }
        const double2 x = halo[(hp * HR + hr) * HC + hc];
        const double ca = coef(a, da);
        zr = fma(ca, x.x, zr);
        zi = fma(ca, x.y, zi);
      }
    };
    if (crow1) {
      // radius 1: the offsets of mu_0^1 from its table, zero elsewhere
      row_sum([&](int, const int* da) {
        bool in = true;
        int a1 = 0;
#pragma unroll
        for (int k = 0; k < D; ++k) {
          in = in && da[k] >= -1 && da[k] <= 1;
          a1 = a1 * 3 + da[k] + 1;
        }
        return in ? crow1[a1] : 0.0;
      });
    } else {
      row_sum([&](int a, const int*) { return crow[a]; });
    }
    z[g] = make_double2(zr, zi);
  }
}

template <int W, int TR, int TW>
hipError_t run_assemble_lds(lsp_problem* p, void* P, bool fp32, int32_t* idx) {
  const int n = p->n;
  dim3 grid(n / TW, n / TR);
  const double2* act = reinterpret_cast<const double2*>(p->ws.actab);
  if (fp32)
    hipLaunchKernelGGL((assemble_lds_kernel<W, TR, TW, float>), grid, dim3(256), 0, p->stream,
                       p->v, n, p->ws.S, p->ws.nS, act, static_cast<float*>(P), idx);
  else
    hipLaunchKernelGGL((assemble_lds_kernel<W, TR, TW, double>), grid, dim3(256), 0, p->stream,
                       p->v, n, p->ws.S, p->ws.nS, act, static_cast<double*>(P), idx);
  return hipGetLastError();
}

template <int D, int W, int TW, int TR>
hipError_t run_assemble_tile(lsp_problem* p, void* P, bool fp32, int32_t* idx) {
  const int n = p->n;
  if (n % TW != 0 || n % TR != 0) return hipErrorInvalidValue;
  dim3 grid(n / TW, n / TR, (D == 3) ? n : 1);
  const double2* act = reinterpret_cast<const double2*>(p->ws.actab);
  if (fp32)
    hipLaunchKernelGGL((assemble_kernel<D, W, TR, TW, float>), grid, dim3(256), 0, p->stream,
                       p->v, n, p->ws.S, p->ws.nS, act, static_cast<float*>(P), idx);
  else
    hipLaunchKernelGGL((assemble_kernel<D, W, TR, TW, double>), grid, dim3(256), 0, p->stream,
                       p->v, n, p->ws.S, p->ws.nS, act, static_cast<double*>(P), idx);
  return hipGetLastError();
}

template <int D, int W, int TW>
hipError_t run_c_apply_tw(const lsp_problem* p, const double* r, double* z) {
  constexpr int TR = 4;
  constexpr int M = Pow<D, W>::v;
  const int n = p->n;
  if (n % TW != 0 || n % TR != 0) return hipErrorInvalidValue;
  dim3 grid(n / TW, n / TR, (D == 3) ? n : 1);
  // the LDS table form for the shift tables of a uniform-radius exact setup
  // (the requested |S| bounds the one the setup kept), used in 3D with t = 1:
  // 6.5 -> 5.8 us at n = 64; in 2D (n = 1024, t = 2: 16.6 -> 18.3 us) the
  // copy of the table into every block of 256 points costs more than the
  // gathers it saves, and in 3D with t = 2 (17.1 us either way) its LDS halves
  // the residency
  const bool lc = D == 3 && W == 3 && !p->learned && p->nd_leaf == 0 &&
                  p->num_shifts <= kCApplyShifts && p->num_shifts * M <= kCApplyLds;
  if (lc)
    hipLaunchKernelGGL((c_apply_kernel<D, W, TR, TW, true>), grid, dim3(256), 0, p->stream,
                       reinterpret_cast<const double2*>(r), p->v, n, p->ws.S, p->ws.nS,
                       p->ws.Ctab, nullptr, nullptr, 0, reinterpret_cast<double2*>(z));
  else
    hipLaunchKernelGGL((c_apply_kernel<D, W, TR, TW, false>), grid, dim3(256), 0, p->stream,
                       reinterpret_cast<const double2*>(r), p->v, n, p->ws.S, p->ws.nS,
                       p->ws.Ctab, p->learned ? p->c_rows : nullptr, p->nd1.C,
                       p->learned ? 0 : p->nd_leaf, reinterpret_cast<double2*>(z));
  return hipGetLastError();
}

// assembly tiles: one row of up to 128 points (2D) or 64 points (3D)
template <int D, int W>
hipError_t run_assemble(lsp_problem* p, void* P, bool fp32, int32_t* idx) {
  switch (p->n) {
    case 8: return run_assemble_tile<D, W, 8, 1>(p, P, fp32, idx);
    case 16: return run_assemble_tile<D, W, 16, 1>(p, P, fp32, idx);
    case 32: return run_assemble_tile<D, W, 32, 1>(p, P, fp32, idx);
    default: break;
  }
  if constexpr (D == 2) {
    if (p->n == 64) return run_assemble_tile<D, W, 64, 1>(p, P, fp32, idx);
    // a tuned shape (lsp_autotune): 1-row tiles of 32, 64 or 128 points, or
    // (code 1) the LDS-table kernel
    const int tuned = p->tune[LSP_TUNE_ASSEMBLY_TILE];
    const bool lds_ok = p->num_shifts * W * W <= kActLds;
    if (tuned == 32) return run_assemble_tile<D, W, 32, 1>(p, P, fp32, idx);
    if (tuned == 64) return run_assemble_tile<D, W, 64, 1>(p, P, fp32, idx);
    if (tuned == 128) return run_assemble_tile<D, W, 128, 1>(p, P, fp32, idx);
    if (tuned == 1 && lds_ok) return run_assemble_lds<W, 4, 128>(p, P, fp32, idx);
    // FP32 rows: the tables fit in LDS (the requested |S| bounds the
    // effective one) and the grid of 4-row tiles still fills the chip
    if (fp32 && p->n >= 512 && lds_ok) return run_assemble_lds<W, 4, 128>(p, P, fp32, idx);
    return run_assemble_tile<D, W, 128, 1>(p, P, fp32, idx);
  } else {
    // t = 1 at n = 64: tiles of two whole rows (128 points; 3D n = 64 setup
    // 35.7 -> 34.5 us; with t = 2 the same time either way)
    if (W == 3 && p->n == 64) return run_assemble_tile<D, W, 64, 2>(p, P, fp32, idx);
    return run_assemble_tile<D, W, 64, 1>(p, P, fp32, idx);
  }
}

// C-apply tiles: 4 rows of up to 64 points, one point per thread (wider
// tiles put several points on a thread, whose table gathers then wait in
// sequence: 23.2 us against 17.1 us at 2D n = 1024)
template <int D, int W>
hipError_t run_c_apply(const lsp_problem* p, const double* r, double* z) {
  const int cap = 64;
  const int tw = p->n < cap ? p->n : cap;
  switch (tw) {
    case 8: return run_c_apply_tw<D, W, 8>(p, r, z);
    case 16: return run_c_apply_tw<D, W, 16>(p, r, z);
    case 32: return run_c_apply_tw<D, W, 32>(p, r, z);
    case 64: return run_c_apply_tw<D, W, 64>(p, r, z);
  }
  return hipErrorInvalidValue;
}

#define LSP_DISPATCH_DW(D_, W_, CALL) \
  if (p->d == D_ && 2 * p->t + 1 == W_) return CALL;

}  // namespace

namespace lsp {

hipError_t launch_assemble(lsp_problem* p, void* P, bool fp32, int32_t* idx) {
  LSP_DISPATCH_DW(2, 3, (run_assemble<2, 3>(p, P, fp32, idx)))
  LSP_DISPATCH_DW(2, 5, (run_assemble<2, 5>(p, P, fp32, idx)))
  LSP_DISPATCH_DW(2, 7, (run_assemble<2, 7>(p, P, fp32, idx)))
  LSP_DISPATCH_DW(3, 3, (run_assemble<3, 3>(p, P, fp32, idx)))
  LSP_DISPATCH_DW(3, 5, (run_assemble<3, 5>(p, P, fp32, idx)))
  return hipErrorInvalidValue;
}

hipError_t launch_assemble_batched(int d, int t, int tw, bool fp32, const BatchRec* recs,
                                   const int4* map, int blocks, hipStream_t s) {
  const int W = 2 * t + 1;
  // tw = kBatchLdsTile: 8 x 64 tiles with the shift tables in LDS (2D)
#define LSP_ASM_LDS_B(W_)                                                                    \
  if (d == 2 && W == W_ && tw == kBatchLdsTile) {                                            \
    if (fp32)                                                                                \
      hipLaunchKernelGGL((assemble_lds_batched_kernel<W_, 8, 64, float>), dim3(blocks),      \
                         dim3(256), 0, s, recs, map);                                        \
    else                                                                                     \
      hipLaunchKernelGGL((assemble_lds_batched_kernel<W_, 8, 64, double>), dim3(blocks),     \
                         dim3(256), 0, s, recs, map);                                        \
    return hipGetLastError();                                                                \
  }
  LSP_ASM_LDS_B(3)
  LSP_ASM_LDS_B(5)
  LSP_ASM_LDS_B(7)
#undef LSP_ASM_LDS_B
#define LSP_ASM_B(D_, W_, TW_)                                                               \
  if (d == D_ && W == W_ && tw == TW_) {                                                     \
    if (fp32)                                                                                \
      hipLaunchKernelGGL((assemble_batched_kernel<D_, W_, 1, TW_, float>), dim3(blocks),      \
                         dim3(256), 0, s, recs, map);                                        \
    else                                                                                     \
      hipLaunchKernelGGL((assemble_batched_kernel<D_, W_, 1, TW_, double>), dim3(blocks),     \
                         dim3(256), 0, s, recs, map);                                        \
    return hipGetLastError();                                                                \
  }
#define LSP_ASM_B_TW(D_, W_) \
  LSP_ASM_B(D_, W_, 16) LSP_ASM_B(D_, W_, 32) LSP_ASM_B(D_, W_, 64) LSP_ASM_B(D_, W_, 128)
  LSP_ASM_B_TW(2, 3)
  LSP_ASM_B_TW(2, 5)
  LSP_ASM_B_TW(2, 7)
  LSP_ASM_B_TW(3, 3)
#undef LSP_ASM_B_TW
#undef LSP_ASM_B
  return hipErrorInvalidValue;
}

hipError_t launch_c_apply(const lsp_problem* p, const double* r, double* z) {
  LSP_DISPATCH_DW(2, 3, (run_c_apply<2, 3>(p, r, z)))
  LSP_DISPATCH_DW(2, 5, (run_c_apply<2, 5>(p, r, z)))
  LSP_DISPATCH_DW(2, 7, (run_c_apply<2, 7>(p, r, z)))
  LSP_DISPATCH_DW(3, 3, (run_c_apply<3, 3>(p, r, z)))
  LSP_DISPATCH_DW(3, 5, (run_c_apply<3, 5>(p, r, z)))
  return hipErrorInvalidValue;
}

}  // namespace lsp
