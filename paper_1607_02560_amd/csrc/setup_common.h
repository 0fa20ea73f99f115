// Compile-time geometry of the neighbourhood mu_0^t and small device helpers
// shared by the stencil-setup kernels.
#pragma once

#include "lsp_internal.h"

namespace lsp {

// Radius t_j of point c (coordinates per axis) in the per-point-radius setup
// with leaf box b (Sec. 4.2, Fig. 3): the separators are the grid planes
// c_i = 0 mod b; a vertex (every coordinate on a separator) may reach b, any
// other point reaches up to the nearest separator plane across its
// coordinates off the separators; capped at tmax.
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

template <int D, int W>
struct Pow {
  static constexpr int v = W * Pow<D - 1, W>::v;
};
template <int W>
struct Pow<0, W> {
  static constexpr int v = 1;
};

// Offsets of mu_0^t = [-t, t]^D in lexicographic order (last axis fastest),
// t = (W - 1)/2; the Green's tables hold offsets [0, 2t]^D in the same order.
template <int D, int W>
struct Nbhd {
  static constexpr int t = (W - 1) / 2;
  static constexpr int M = Pow<D, W>::v;
  // component i of offset a
  __host__ __device__ static constexpr int comp(int a, int i) {
    int rem = a;
    for (int j = D - 1; j > i; --j) rem /= W;
    return rem % W - t;
  }
  // index in the [0, 2t]^D table of the componentwise |a - b|
  __host__ __device__ static constexpr int diff_index(int a, int b) {
    int idx = 0;
    for (int i = 0; i < D; ++i) {
      int dd = comp(a, i) - comp(b, i);
      if (dd < 0) dd = -dd;
      idx = idx * W + dd;
    }
    return idx;
  }
};

// Parity classes of the neighbourhood.
// The Green's kernel is even in every coordinate, so G[mu,mu], A1 and
// M = A1 - A2 commute with the reflection of any axis. With the orthonormal
// 1D basis {e_0, (e_j + e_-j)/sqrt2 : j = 1..t} (even) and
// {(e_j - e_-j)/sqrt2 : j = 1..t} (odd), their tensor products split
// [-t,t]^D into 2^D classes c (bit D-1-i of c = parity along axis i) and the
// matrices are block diagonal. Class c has size prod_i (odd_i ? t : t+1);
// row p of a block is the tensor product of the 1D basis vectors with
// indices j_i = coord(c, p, i) (1..t for odd axes, 0..t for even ones).
template <int D, int W>
struct Parity {
  static constexpr int t = (W - 1) / 2;
  static constexpr int NC = 1 << D;
  __host__ __device__ static constexpr int odd(int c, int i) { return (c >> (D - 1 - i)) & 1; }
  __host__ __device__ static constexpr int count(int c, int i) { return odd(c, i) ? t : t + 1; }
  __host__ __device__ static constexpr int size(int c) {
    int b = 1;
    for (int i = 0; i < D; ++i) b *= count(c, i);
    return b;
  }
  __host__ __device__ static constexpr int offset(int c) {  // packed block storage
    int o = 0;
    for (int k = 0; k < c; ++k) o += size(k) * size(k);
    return o;
  }
  __host__ __device__ static constexpr int coord(int c, int p, int i) {
    int rem = p;
    for (int ax = D - 1; ax > i; --ax) rem /= count(c, ax);
    return rem % count(c, i) + odd(c, i);
  }
};

constexpr double kInvSqrt2 = 0.70710678118654752440;

// 1/x: hardware estimate refined by two Newton steps (within an ulp or two).
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// 1/x: hardware estimate r refined by one third-order step r (1 + e + e^2),
// e = 1 - x r (the truncation error e^3 is far below FP64 rounding for the
// estimate's error), three FMAs in place of two Newton steps.
__device__ __forceinline__ double rcp_cubic(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  const double e = fma(-x, r, 1.0);
  return fma(r, fma(e, e, e), r);
}

// 1/sqrt(x) for x > 0: hardware estimate and two Newton steps.
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double hx = 0.5 * x;
  y = y * fma(-hx * y, y, 1.5);
  y = y * fma(-hx * y, y, 1.5);
  return y;
}

// Broadcast lane `src` (wave-uniform) of a double to every lane.
__device__ __forceinline__ double bcast(double x, int src) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), src);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Lane exchange of a double within each 16-lane row (DPP; no LDS traffic).
template <int CTRL>
__device__ __forceinline__ double dpp_move(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// DPP controls: rotate a 16-lane row by 8 (partner lane ^ 8), mirror each
// 8-lane half row (partner 7 - i, which differs in bit 2), quad permutations
// [2,3,0,1] (lane ^ 2) and [1,0,3,2] (lane ^ 1).
constexpr int kDppRowRor8 = 0x128;
constexpr int kDppHalfMirror = 0x141;
constexpr int kDppQuadXor2 = 0x4E;
constexpr int kDppQuadXor1 = 0xB1;

// Index of the shift of the sorted list S closest to vj (Sec. 4.1); the two
// neighbours of the insertion point are compared and ties go to the lower index.
__device__ __forceinline__ int nearest_shift(const double* S, int nS, double vj) {
  int lo = 0, hi = nS;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (S[mid] < vj) lo = mid + 1;
    else hi = mid;
  }
  if (lo == 0) return 0;
  if (lo == nS) return nS - 1;
  const double d0 = fabs(S[lo - 1] - vj);
  const double d1 = fabs(S[lo] - vj);
  return (d1 < d0) ? lo : lo - 1;
}

// Snapped bin centre i of the shift list (Sec. 4.1):
// snap(v_min + (i + 1/2) width) with snap(x) = (4 floor(x / (4 pi^2)) + 2) pi^2,
// the value of the form (4m+2) pi^2 nearest to x. Contraction is off, so every
// step is one IEEE rounding.
__device__ __forceinline__ double snapped_centre(double vmin, double width, int i) {
#pragma clang fp contract(off)
  const double centre = vmin + ((double)i + 0.5) * width;
  return (4.0 * floor(centre / kFourPi2) + 2.0) * kPi2;
}

// Shift list S from the kMinMaxBlocks (min, max) partials of v, computed by
// every thread of a block of NT threads (NT a multiple of 64 dividing
// kMinMaxBlocks). All partial loads are issued before the first use.
// The bin centres increase with i and snap is monotone, so duplicates are
// adjacent; they are dropped by a ballot-based stream compaction.
// Results in LDS: sS[0..*sNS), sRange[0] = v_min, sRange[1] = v_max.
template <int NT>
__device__ inline void shift_list_block(const double* __restrict__ part, int nreq, double* sS,
                                        int* sNS, double* sRange, int* sWave, double* sRed) {
  static_assert(NT % 64 == 0 && kMinMaxBlocks % NT == 0, "block shape");
  constexpr int NW = NT / 64;
  constexpr int PER = kMinMaxBlocks / NT;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wid = tid >> 6;
  const double2* p2 = reinterpret_cast<const double2*>(part);
  double2 x[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) x[i] = p2[tid + i * NT];
  double lo = x[0].x, hi = x[0].y;
#pragma unroll
  for (int i = 1; i < PER; ++i) {
    lo = fmin(lo, x[i].x);
    hi = fmax(hi, x[i].y);
  }
  // wave reduction: in-row lane moves first (DPP), then across rows
  lo = fmin(lo, dpp_move<kDppRowRor8>(lo));
  hi = fmax(hi, dpp_move<kDppRowRor8>(hi));
  lo = fmin(lo, dpp_move<kDppHalfMirror>(lo));
  hi = fmax(hi, dpp_move<kDppHalfMirror>(hi));
  lo = fmin(lo, dpp_move<kDppQuadXor2>(lo));
  hi = fmax(hi, dpp_move<kDppQuadXor2>(hi));
  lo = fmin(lo, dpp_move<kDppQuadXor1>(lo));
  hi = fmax(hi, dpp_move<kDppQuadXor1>(hi));
  lo = fmin(lo, __shfl_xor(lo, 16));
  hi = fmax(hi, __shfl_xor(hi, 16));
  lo = fmin(lo, __shfl_xor(lo, 32));
  hi = fmax(hi, __shfl_xor(hi, 32));
  double vmin = lo, vmax = hi;
  if constexpr (NW > 1) {
    if (lane == 0) {
      sRed[2 * wid] = lo;
      sRed[2 * wid + 1] = hi;
    }
    __syncthreads();
    vmin = sRed[0];
    vmax = sRed[1];
#pragma unroll
    for (int w = 1; w < NW; ++w) {
      vmin = fmin(vmin, sRed[2 * w]);
      vmax = fmax(vmax, sRed[2 * w + 1]);
    }
  }
  const double width = (vmax - vmin) / (double)nreq;
  int base = 0;
  for (int c0 = 0; c0 < nreq; c0 += NT) {
    const int k = c0 + tid;
    double s = 0.0;
    bool keep = false;
    if (k < nreq) {
      s = snapped_centre(vmin, width, k);
      keep = (k == 0) || (s != snapped_centre(vmin, width, k - 1));
    }
    const unsigned long long bal = __ballot(keep);
    const int before = __popcll(bal & ((1ull << lane) - 1ull));
    if constexpr (NW == 1) {
      if (keep) sS[base + before] = s;
      base += __popcll(bal);
    } else {
      if (lane == 0) sWave[wid] = __popcll(bal);
      __syncthreads();
      int off = base, total = 0;
      for (int w = 0; w < NW; ++w) {
        if (w < wid) off += sWave[w];
        total += sWave[w];
      }
      if (keep) sS[off + before] = s;
      base += total;
      __syncthreads();
    }
  }
  if (tid == 0) {
    *sNS = base;
    sRange[0] = vmin;
    sRange[1] = vmax;
  }
  __syncthreads();
}

// The one shift of the non-localized method (Sec. 3) from the min/max/sum
// partials, computed by every thread of the block: s = mean of v, moved to
// (2 - 4K) pi^2 (the form (4m+2) pi^2 with m = -K, 2 pi^2 above the singular
// point) only when L + s is singular, i.e. when x = -s / (4 pi^2) lies within
// 2^-30 max(1, |x|) of an integer K >= 0.
// The partial sums are added in a fixed order (per thread, butterfly over
// the lanes, waves in index order), so every thread gets the same s.
// Results in LDS like lsp::shift_list_block: sS[0], *sNS = 1, sRange.
template <int NT>
__device__ inline void global_shift_block(const double* __restrict__ part, int64_t N, double* sS,
                                          int* sNS, double* sRange, double* sRed) {
  static_assert(NT % 64 == 0 && kMinMaxBlocks % NT == 0, "block shape");
  constexpr int NW = NT / 64;
  constexpr int PER = kMinMaxBlocks / NT;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wid = tid >> 6;
  const double2* p2 = reinterpret_cast<const double2*>(part);
  const double* ps = part + 2 * kMinMaxBlocks;
  double2 x[PER];
  double xs[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    x[i] = p2[tid + i * NT];
    xs[i] = ps[tid + i * NT];
  }
  double lo = x[0].x, hi = x[0].y, sum = xs[0];
#pragma unroll
  for (int i = 1; i < PER; ++i) {
    lo = fmin(lo, x[i].x);
    hi = fmax(hi, x[i].y);
    sum += xs[i];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, o));
    hi = fmax(hi, __shfl_xor(hi, o));
    sum += __shfl_xor(sum, o);
  }
  if (lane == 0) {
    sRed[3 * wid] = lo;
    sRed[3 * wid + 1] = hi;
    sRed[3 * wid + 2] = sum;
  }
  __syncthreads();
  lo = sRed[0];
  hi = sRed[1];
  sum = sRed[2];
#pragma unroll
  for (int w = 1; w < NW; ++w) {
    lo = fmin(lo, sRed[3 * w]);
    hi = fmax(hi, sRed[3 * w + 1]);
    sum += sRed[3 * w + 2];
  }
  double s = sum / (double)N;
  const double xr = -s / kFourPi2;
  const double K = floor(xr + 0.5);
  if (K >= 0.0 && fabs(xr - K) <= 0x1p-30 * fmax(1.0, fabs(xr)))
    s = (2.0 - 4.0 * K) * kPi2;
  if (tid == 0) {
    sS[0] = s;
    *sNS = 1;
    sRange[0] = lo;
    sRange[1] = hi;
  }
  __syncthreads();
}

}  // namespace lsp
