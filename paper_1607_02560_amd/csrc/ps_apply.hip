// Pseudospectral apply y = (L + diag v) u on the periodic grid (Sec. 2, eq. dmodel).
//
// L = F^-1 diag(4 pi^2 |k|^2) F and |k|^2 = k_1^2 + ... + k_d^2, so L is the sum
// over axes of the 1D operator L_1 = F_1^-1 diag(4 pi^2 k^2) F_1 acting along
// that axis. Each axis is one streaming pass over the grid: a work-group loads
// whole lines along the axis, runs a forward DFT, scales by 4 pi^2 k^2 / n and
// runs the inverse DFT, all in registers and LDS, then stores. The passes
// accumulate:  z = L_ax0 u,  z += L_ax1 u (3D),  y = L_last u + z + v u.
// For d = 2 that is two passes (88 bytes per point) instead of the three of a
// row-FFT / column-FFT / row-IFFT pipeline.
//
// One line of length n = N1*N2 is transformed by the two-factor (four-step)
// decomposition: N2 threads each hold N1 points x[N2*a + b] (a = 0..N1-1) and
// run an N1-point DFT in registers; twiddles exp(-2 pi i b k1 / n) are applied;
// an LDS exchange gives each of N1 threads the N2 values of one k1, which run
// an N2-point DFT. The scaled spectrum is transformed back by the same two
// steps in reverse order, so the spectrum never leaves registers.
#include "lsp_internal.h"
#include "setup_common.h"

namespace {

// ---------------------------------------------------------------------------
// Compile-time cos/sin of 2 pi k / R for the register DFTs.
// The angle is reduced exactly in integers to [0, pi/4], where a Taylor series
// of 12 terms is exact to rounding.
// ---------------------------------------------------------------------------
struct CS {
  double c, s;
};

constexpr double kPiC = 3.141592653589793238462643383279502884;

constexpr double sin_taylor(double x) {
  double x2 = x * x, term = x, sum = x;
  for (int i = 1; i < 12; ++i) {
    term = -term * x2 / ((2.0 * i) * (2.0 * i + 1.0));
    sum += term;
  }
  return sum;
}

constexpr double cos_taylor(double x) {
  double x2 = x * x, term = 1.0, sum = 1.0;
  for (int i = 1; i < 12; ++i) {
    term = -term * x2 / ((2.0 * i - 1.0) * (2.0 * i));
    sum += term;
  }
  return sum;
}

constexpr CS cs2pi(long k, long R) {
  k %= R;
  if (k < 0) k += R;
  long q = (4 * k) / R;      // quarter turns
  long rem = 4 * k - q * R;  // angle within quarter = (pi/2) rem / R
  double cf = 0.0, sf = 0.0;
  if (2 * rem <= R) {
    double f = (kPiC / 2.0) * (double)rem / (double)R;
    cf = cos_taylor(f);
    sf = sin_taylor(f);
  } else {
    double f = (kPiC / 2.0) * (double)(R - rem) / (double)R;
    cf = sin_taylor(f);
    sf = cos_taylor(f);
  }
  switch (q) {
    case 0: return CS{cf, sf};
    case 1: return CS{-sf, cf};
    case 2: return CS{-cf, -sf};
    default: return CS{sf, -cf};
  }
}

// y[k] = sum_j x[j*IS] exp(SIGN * 2 pi i j k / R), radix-2 decimation in time,
// fully unrolled; natural order in and out.
template <int R, int SIGN>
struct RegDft {
  template <int IS>
  __device__ static __forceinline__ void run(const double* xr, const double* xi, double* yr,
                                             double* yi) {
    if constexpr (R == 1) {
      yr[0] = xr[0];
      yi[0] = xi[0];
    } else if constexpr (R == 2) {
      yr[0] = xr[0] + xr[IS];
      yi[0] = xi[0] + xi[IS];
      yr[1] = xr[0] - xr[IS];
      yi[1] = xi[0] - xi[IS];
    } else {
      constexpr int H = R / 2;
      double er[H], ei[H], orr[H], oi[H];
      RegDft<H, SIGN>::template run<2 * IS>(xr, xi, er, ei);
      RegDft<H, SIGN>::template run<2 * IS>(xr + IS, xi + IS, orr, oi);
      combine<0>(er, ei, orr, oi, yr, yi);
    }
  }

  template <int K>
  __device__ static __forceinline__ void combine(const double* er, const double* ei,
                                                 const double* orr, const double* oi, double* yr,
                                                 double* yi) {
    if constexpr (K < R / 2) {
      double tr, ti;
      if constexpr (K == 0) {
        tr = orr[0];
        ti = oi[0];
      } else if constexpr (4 * K == R) {
        // w = exp(SIGN i pi/2) = SIGN i
        tr = (SIGN > 0) ? -oi[K] : oi[K];
        ti = (SIGN > 0) ? orr[K] : -orr[K];
      } else {
        constexpr CS w = cs2pi(K, R);
        constexpr double c = w.c;
        constexpr double s = SIGN * w.s;
        tr = c * orr[K] - s * oi[K];
        ti = c * oi[K] + s * orr[K];
      }
      yr[K] = er[K] + tr;
      yi[K] = ei[K] + ti;
      yr[K + R / 2] = er[K] - tr;
      yi[K + R / 2] = ei[K] - ti;
      combine<K + 1>(er, ei, orr, oi, yr, yi);
    }
  }
};

enum { kFirst = 0, kAccum = 1, kFinal = 2 };

// ---------------------------------------------------------------------------
// Line operator for n = 256 R3 (R3 = 1, 2, 4: n = 256, 512, 1024).
// T = 16 R3 threads own a line; n = 16 * 16 * R3. With j = T a + t and
// k = k1 + 16 (k2a + 16 k2b):
//   1. thread t: 16-point DFT over a of x[T a + t], times w_n^(t k1);
//   2. LDS transpose: thread (k1, c) = (tau / R3, tau % R3) takes the values
//      t = R3 b + c, runs the 16-point DFT over b, times w_T^(c k2a);
//   3. the R3-point DFT over c runs across the R3 neighbouring lanes with DPP
//      quad permutations (radix 2), which leaves k2b = bitrev(c) in lane c;
// every thread then holds 16 spectrum values, scales them by 4 pi^2 kk^2 / n
// and runs the same steps backwards (conjugate twiddles), ending with
// x[T a + t] in natural order. Two LDS transposes per line in total; 16
// complex values per thread.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void cmul(double& xr, double& xi, double wr, double wi) {
  const double r = xr * wr - xi * wi;
  const double i = xr * wi + xi * wr;
  xr = r;
  xi = i;
}

// x * conj(w)
__device__ __forceinline__ void cmulc(double& xr, double& xi, double wr, double wi) {
  const double r = xr * wr + xi * wi;
  const double i = xi * wr - xr * wi;
  xr = r;
  xi = i;
}

// w^(m j) for j = 0..15 with w^i = tw[i] (tw[i] = exp(-2 pi i i / n)) and
// 12 m < n: six table loads, the rest as one product each.
__device__ __forceinline__ void twiddle16(const double2* __restrict__ tw, int m, double* wr,
                                          double* wi) {
  double2 lo[4], hi[4];
  lo[0] = make_double2(1.0, 0.0);
  hi[0] = make_double2(1.0, 0.0);
#pragma unroll
  for (int r = 1; r < 4; ++r) {
    lo[r] = tw[m * r];
    hi[r] = tw[4 * m * r];
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      double a = hi[q].x, b = hi[q].y;
      if (r > 0) {
        if (q > 0) {
          cmul(a, b, lo[r].x, lo[r].y);
        } else {
          a = lo[r].x;
          b = lo[r].y;
        }
      }
      wr[4 * q + r] = a;
      wi[4 * q + r] = b;
    }
  }
}

// Radix-2 step of the R3-point DFT across lanes: lane c pairs with c ^ (1 << BIT);
// the lower lane keeps p + v, the upper p - v (one FMA with the lane's sign).
template <int BIT>
__device__ __forceinline__ void lane_butterfly(double& vr, double& vi, int c) {
  constexpr int ctrl = (BIT == 0) ? lsp::kDppQuadXor1 : lsp::kDppQuadXor2;
  const double sgn = ((c >> BIT) & 1) ? -1.0 : 1.0;
  const double pr = lsp::dpp_move<ctrl>(vr);
  const double pi = lsp::dpp_move<ctrl>(vi);
  vr = fma(sgn, vr, pr);
  vi = fma(sgn, vi, pi);
}

// Forward R3-point DFT over the lanes c (decimation in frequency); lane c ends
// with frequency bitrev(c).
template <int R3>
__device__ __forceinline__ void lane_dft_fwd(double& vr, double& vi, int c) {
  if constexpr (R3 == 2) {
    lane_butterfly<0>(vr, vi, c);
  } else if constexpr (R3 == 4) {
    lane_butterfly<1>(vr, vi, c);
    if (c == 3) {  // times exp(-i pi/2) = -i
      const double t = vr;
      vr = vi;
      vi = -t;
    }
    lane_butterfly<0>(vr, vi, c);
  }
}

// Inverse (conjugate) R3-point DFT: lane c holds frequency bitrev(c) and ends
// with index c (decimation in time).
template <int R3>
__device__ __forceinline__ void lane_dft_inv(double& vr, double& vi, int c) {
  if constexpr (R3 == 2) {
    lane_butterfly<0>(vr, vi, c);
  } else if constexpr (R3 == 4) {
    lane_butterfly<0>(vr, vi, c);
    if (c == 3) {  // times exp(+i pi/2) = +i
      const double t = vr;
      vr = -vi;
      vi = t;
    }
    lane_butterfly<1>(vr, vi, c);
  }
}

template <int R3>
__device__ __forceinline__ int bitrev_lane(int c) {
  if constexpr (R3 == 4) return ((c & 1) << 1) | (c >> 1);
  return c;
}

constexpr int kFftThreads = 256;

// Blocks of the strided passes: groups 2j and 2j+1 cover the two halves of
// the same 128-byte rows, so they are placed on the same XCD (block b runs
// on XCD b mod 8) and share its L2.
__device__ __forceinline__ int64_t xcd_paired_group(int64_t b, int64_t nb) {
  const int64_t full = nb & ~(int64_t)15;
  if (b >= full) return b;
  const int64_t x = b & 7, q = b >> 3;
  return (((q >> 1) << 3) + x) * 2 + (q & 1);
}

// One pass of L_1 along one axis for n = 256 R3.
//   CONTIG: the axis is the last; line L starts at L n.
//   !CONTIG: the axis has stride st; line L = (o, i) = (L / st, L % st)
//            starts at o n st + i; a block's LPB lines are adjacent i, so a
//            row of the block is LPB consecutive elements.
// Loads and stores use the "memory" thread map (line, t): for CONTIG a line's
// T threads are consecutive lanes (consecutive addresses); for !CONTIG the
// LPB lines of a row are consecutive lanes, so one instruction covers
// 64 / LPB rows of LPB * 16 bytes. The spectral steps use the "line" map
// (line = tid / T, tau = tid % T), which keeps the R3 lanes of step 3 in one
// quad. Both maps meet in the LDS layout sh[line][k1][t].
// MODE: kFirst out = L_1 u; kAccum out = L_1 u + acc; kFinal out = L_1 u + acc + v u.
template <int R3, bool CONTIG, int MODE>
__global__ __launch_bounds__(kFftThreads) void fft_line_kernel(
    const double2* __restrict__ u, double2* __restrict__ out, const double2* __restrict__ acc,
    const double* __restrict__ v, const double2* __restrict__ tw, int64_t nlines, int64_t st) {
  constexpr int T = 16 * R3;
  constexpr int n = 16 * T;
  constexpr int LPB = kFftThreads / T;  // lines per block
  constexpr int RS = T + 1;             // padded LDS row
  constexpr int LS = 16 * RS + 2;       // LDS stride between lines (padded)
  __shared__ double2 sh[LPB * LS];

  const int tid = threadIdx.x;
  const int64_t g = CONTIG ? (int64_t)blockIdx.x : xcd_paired_group(blockIdx.x, gridDim.x);
  // memory map
  const int ml = CONTIG ? tid / T : tid % LPB;
  const int t = CONTIG ? tid % T : tid / LPB;
  const int64_t Lm = g * LPB + ml;
  const bool active = Lm < nlines;
  int64_t base, es;
  if constexpr (CONTIG) {
    base = Lm * n;
    es = 1;
  } else {
    const int64_t o = Lm / st, i = Lm % st;
    base = o * n * st + i;
    es = st;
  }
  double2* Sm = sh + ml * LS;

  // 1. 16-point DFT over a, twiddle w_n^(t k1)
  double xr[16], xi[16], yr[16], yi[16], wr[16], wi[16];
  double2 zacc[16];
  double vv[16];
#pragma unroll
  for (int a = 0; a < 16; ++a) {
    double2 val = make_double2(0.0, 0.0);
    if (active) val = u[base + (int64_t)(T * a + t) * es];
    xr[a] = val.x;
    xi[a] = val.y;
  }
  if constexpr (MODE == kAccum || MODE == kFinal) {
    // the addends are loaded up front so their latency overlaps the transform
#pragma unroll
    for (int a = 0; a < 16; ++a)
      zacc[a] = active ? acc[base + (int64_t)(T * a + t) * es] : make_double2(0.0, 0.0);
  }
  if constexpr (MODE == kFinal) {
#pragma unroll
    for (int a = 0; a < 16; ++a) vv[a] = active ? v[base + (int64_t)(T * a + t) * es] : 0.0;
  }
  double ur[16], ui[16];
  if constexpr (MODE == kFinal) {
#pragma unroll
    for (int a = 0; a < 16; ++a) {
      ur[a] = xr[a];
      ui[a] = xi[a];
    }
  }
  RegDft<16, -1>::template run<1>(xr, xi, yr, yi);
  twiddle16(tw, t, wr, wi);
#pragma unroll
  for (int k1 = 0; k1 < 16; ++k1) {
    cmul(yr[k1], yi[k1], wr[k1], wi[k1]);
    Sm[k1 * RS + t] = make_double2(yr[k1], yi[k1]);
  }
  __syncthreads();

  // 2. line map: thread (k1, c) runs the 16-point DFT over b of t = R3 b + c
  const int sl = tid / T;
  const int tau = tid % T;
  double2* Ss = sh + sl * LS;
  const int k1 = tau / R3;
  const int c = tau % R3;
#pragma unroll
  for (int b = 0; b < 16; ++b) {
    const double2 val = Ss[k1 * RS + R3 * b + c];
    xr[b] = val.x;
    xi[b] = val.y;
  }
  RegDft<16, -1>::template run<1>(xr, xi, yr, yi);
  if constexpr (R3 > 1) {
    twiddle16(tw, 16 * c, wr, wi);
#pragma unroll
    for (int k2a = 0; k2a < 16; ++k2a) {
      cmul(yr[k2a], yi[k2a], wr[k2a], wi[k2a]);
      // 3. R3-point DFT across the lanes
      lane_dft_fwd<R3>(yr[k2a], yi[k2a], c);
    }
  }
  // scale by 4 pi^2 kk^2 / n (1/n: the inverse transform is unnormalised)
  const int k2b = bitrev_lane<R3>(c);
#pragma unroll
  for (int k2a = 0; k2a < 16; ++k2a) {
    const int k = k1 + 16 * (k2a + 16 * k2b);
    const int kk = (k < n / 2) ? k : k - n;
    const double fac = (lsp::kFourPi2 / n) * (double)(kk * kk);
    yr[k2a] *= fac;
    yi[k2a] *= fac;
  }
  if constexpr (R3 > 1) {
#pragma unroll
    for (int k2a = 0; k2a < 16; ++k2a) {
      lane_dft_inv<R3>(yr[k2a], yi[k2a], c);
      cmulc(yr[k2a], yi[k2a], wr[k2a], wi[k2a]);
    }
  }
  RegDft<16, +1>::template run<1>(yr, yi, xr, xi);
  // each thread rewrites exactly the LDS entries it read
#pragma unroll
  for (int b = 0; b < 16; ++b) Ss[k1 * RS + R3 * b + c] = make_double2(xr[b], xi[b]);
  __syncthreads();

  // 4. memory map: conjugate twiddle, 16-point inverse DFT over k1
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const double2 val = Sm[q * RS + t];
    xr[q] = val.x;
    xi[q] = val.y;
  }
  twiddle16(tw, t, wr, wi);
#pragma unroll
  for (int q = 0; q < 16; ++q) cmulc(xr[q], xi[q], wr[q], wi[q]);
  RegDft<16, +1>::template run<1>(xr, xi, yr, yi);
  if (!active) return;
#pragma unroll
  for (int a = 0; a < 16; ++a) {
    const int64_t e = base + (int64_t)(T * a + t) * es;
    double2 r = make_double2(yr[a], yi[a]);
    if constexpr (MODE == kAccum || MODE == kFinal) {
      r.x += zacc[a].x;
      r.y += zacc[a].y;
    }
    if constexpr (MODE == kFinal) {
      r.x += vv[a] * ur[a];
      r.y += vv[a] * ui[a];
    }
    out[e] = r;
  }
}

// ---------------------------------------------------------------------------
// Line operator with 8 values per thread, n = 64 R (R = 4, 8, 16: n = 256,
// 512, 1024). T = 8 R threads own a line (two waves at n = 1024), so a pass
// runs twice as many waves as the 16-value form and a SIMD holds two lines
// in different phases (one loading or storing while the other transforms).
// With j = T a + t, t = R b + c and k = k1 + 8 (k2a + 8 k2b):
//   1. thread t: 8-point DFT over a, times w_n^(t k1);
//   2. LDS transpose: thread (k1, c) takes t = R b + c, 8-point DFT over b,
//      times w_n^(8 c k2a);
//   3. the R-point DFT over c across R neighbouring lanes (one DPP row):
//      radix-2 decimation in frequency, partner lane c ^ h for h = R/2 .. 1
//      (row rotate by 8, half-row mirror then quad swap, quad swaps), the
//      upper lane of each pair times w_{2h}^(c mod h); lane c ends with
//      k2b = bitrev(c);
// then the scaled spectrum goes back through the same steps (decimation in
// time, conjugate twiddles) to natural order.
// ---------------------------------------------------------------------------
constexpr int kFft8Threads = 512;

// w^(m j) for j = 0..7 (w^i = tw[i]): five table loads, three products.
__device__ __forceinline__ void twiddle8(const double2* __restrict__ tw, int m, double* wr,
                                         double* wi) {
  double2 lo[4], hi;
  lo[0] = make_double2(1.0, 0.0);
#pragma unroll
  for (int r = 1; r < 4; ++r) lo[r] = tw[m * r];
  hi = tw[4 * m];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    wr[r] = lo[r].x;
    wi[r] = lo[r].y;
    double a = hi.x, b = hi.y;
    if (r > 0) cmul(a, b, lo[r].x, lo[r].y);
    wr[4 + r] = a;
    wi[4 + r] = b;
  }
}

// the four table entries twiddle8 reads for m, loaded ahead of their use
struct Tw8Base {
  double2 lo[3], hi;
  __device__ __forceinline__ void load(const double2* __restrict__ tw, int m) {
#pragma unroll
    for (int r = 1; r < 4; ++r) lo[r - 1] = tw[m * r];
    hi = tw[4 * m];
  }
  // w^(m k), k = 0..7, exactly as twiddle8 forms them
  __device__ __forceinline__ void expand(double* wr, double* wi) const {
    wr[0] = 1.0;
    wi[0] = 0.0;
#pragma unroll
    for (int r = 1; r < 4; ++r) {
      wr[r] = lo[r - 1].x;
      wi[r] = lo[r - 1].y;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      double a = hi.x, b = hi.y;
      if (r > 0) cmul(a, b, lo[r - 1].x, lo[r - 1].y);
      wr[4 + r] = a;
      wi[4 + r] = b;
    }
  }
};

// a double from lane c ^ h of the same 16-lane row
template <int H>
__device__ __forceinline__ double lane_xor(double x) {
  if constexpr (H == 1) return lsp::dpp_move<lsp::kDppQuadXor1>(x);
  if constexpr (H == 2) return lsp::dpp_move<lsp::kDppQuadXor2>(x);
  if constexpr (H == 4) {
    // mirror within 8 lanes (i -> 7 - i), then swap within quads (i -> i ^ 3)
    return lsp::dpp_move<0x1B>(lsp::dpp_move<lsp::kDppHalfMirror>(x));
  }
  return lsp::dpp_move<lsp::kDppRowRor8>(x);  // H == 8
}

template <int H>
__device__ __forceinline__ void lane_pair(double& vr, double& vi, int c) {
  const double sgn = (c & H) ? -1.0 : 1.0;
  const double pr = lane_xor<H>(vr);
  const double pi = lane_xor<H>(vi);
  vr = fma(sgn, vr, pr);
  vi = fma(sgn, vi, pi);
}

// Per-lane twiddles of the R-point lane DFT: stage s (h = 2^s) multiplies
// the upper lanes (c & h) by w_{2h}^(c mod h), w_m = exp(-2 pi i / m).
template <int R>
struct LaneTw {
  double r[4], i[4];
  __device__ __forceinline__ void load(const double2* __restrict__ tw, int n, int c) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int h = 1 << s;
      r[s] = 1.0;
      i[s] = 0.0;
      if (h < R && (c & h)) {
        const double2 w = tw[(c % h) * (n / (2 * h))];
        r[s] = w.x;
        i[s] = w.y;
      }
    }
  }
};

template <int R, int S>
__device__ __forceinline__ void lane_dif_stage(double& vr, double& vi, int c,
                                               const LaneTw<R>& lt) {
  lane_pair<(1 << S)>(vr, vi, c);
  cmul(vr, vi, lt.r[S], lt.i[S]);
}

template <int R>
__device__ __forceinline__ void lane_dft8_fwd(double& vr, double& vi, int c, const LaneTw<R>& lt) {
  if constexpr (R >= 16) lane_dif_stage<R, 3>(vr, vi, c, lt);
  if constexpr (R >= 8) lane_dif_stage<R, 2>(vr, vi, c, lt);
  if constexpr (R >= 4) lane_dif_stage<R, 1>(vr, vi, c, lt);
  if constexpr (R >= 2) lane_pair<1>(vr, vi, c);
}

template <int R, int S>
__device__ __forceinline__ void lane_dit_stage(double& vr, double& vi, int c,
                                               const LaneTw<R>& lt) {
  cmulc(vr, vi, lt.r[S], lt.i[S]);
  lane_pair<(1 << S)>(vr, vi, c);
}

template <int R>
__device__ __forceinline__ void lane_dft8_inv(double& vr, double& vi, int c, const LaneTw<R>& lt) {
  if constexpr (R >= 2) lane_pair<1>(vr, vi, c);
  if constexpr (R >= 4) lane_dit_stage<R, 1>(vr, vi, c, lt);
  if constexpr (R >= 8) lane_dit_stage<R, 2>(vr, vi, c, lt);
  if constexpr (R >= 16) lane_dit_stage<R, 3>(vr, vi, c, lt);
}

template <int R>
__device__ __forceinline__ int bitrev_bits(int c) {
  int r = 0;
#pragma unroll
  for (int b = 1; b < R; b <<= 1) {
    r = (r << 1) | (c & 1);
    c >>= 1;
  }
  return r;
}

template <int R, bool CONTIG, int MODE>
__global__ __launch_bounds__(kFft8Threads) void fft8_line_kernel(
    const double2* __restrict__ u, double2* __restrict__ out, const double2* __restrict__ acc,
    const double* __restrict__ v, const double2* __restrict__ tw, int64_t nlines, int64_t st) {
  constexpr int T = 8 * R;
  constexpr int n = 8 * T;
  constexpr int LPB = kFft8Threads / T;  // lines per block
  constexpr int RS = T + 1;              // padded LDS row
  constexpr int LS = 8 * RS + 2;         // LDS stride between lines (padded)
  __shared__ double2 sh[LPB * LS];

  const int tid = threadIdx.x;
  const int64_t g = CONTIG ? (int64_t)blockIdx.x : xcd_paired_group(blockIdx.x, gridDim.x);
  // memory map
  const int ml = CONTIG ? tid / T : tid % LPB;
  const int t = CONTIG ? tid % T : tid / LPB;
  const int64_t Lm = g * LPB + ml;
  const bool active = Lm < nlines;
  int64_t base, es;
  if constexpr (CONTIG) {
    base = Lm * n;
    es = 1;
  } else {
    const int64_t o = Lm / st, i = Lm % st;
    base = o * n * st + i;
    es = st;
  }
  double2* Sm = sh + ml * LS;
  // line map of steps 2-3: thread (k1, c) of line sl
  const int sl = tid / T;
  const int tau = tid % T;
  const int k1 = tau / R;
  const int c = tau % R;

  // 1. 8-point DFT over a, twiddle w_n^(t k1)
  double xr[8], xi[8], yr[8], yi[8], wr[8], wi[8];
  double2 zacc[8];
  double vv[8];
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    double2 val = make_double2(0.0, 0.0);
    if (active) val = u[base + (int64_t)(T * a + t) * es];
    xr[a] = val.x;
    xi[a] = val.y;
  }
  // every twiddle of the kernel is loaded with the line, not after a barrier
  Tw8Base tw_t, tw_c;
  tw_t.load(tw, t);
  tw_c.load(tw, 8 * c);
  LaneTw<R> lt;
  lt.load(tw, n, c);
  if constexpr (MODE == kAccum || MODE == kFinal) {
#pragma unroll
    for (int a = 0; a < 8; ++a)
      zacc[a] = active ? acc[base + (int64_t)(T * a + t) * es] : make_double2(0.0, 0.0);
  }
  if constexpr (MODE == kFinal) {
#pragma unroll
    for (int a = 0; a < 8; ++a) vv[a] = active ? v[base + (int64_t)(T * a + t) * es] : 0.0;
  }
  double ur[8], ui[8];
  if constexpr (MODE == kFinal) {
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      ur[a] = xr[a];
      ui[a] = xi[a];
    }
  }
  RegDft<8, -1>::template run<1>(xr, xi, yr, yi);
  tw_t.expand(wr, wi);
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    cmul(yr[q], yi[q], wr[q], wi[q]);
    Sm[q * RS + t] = make_double2(yr[q], yi[q]);
  }
  __syncthreads();

  // 2. line map: thread (k1, c) runs the 8-point DFT over b of t = R b + c
  double2* Ss = sh + sl * LS;
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const double2 val = Ss[k1 * RS + R * b + c];
    xr[b] = val.x;
    xi[b] = val.y;
  }
  RegDft<8, -1>::template run<1>(xr, xi, yr, yi);
  tw_c.expand(wr, wi);
#pragma unroll
  for (int k2a = 0; k2a < 8; ++k2a) {
    cmul(yr[k2a], yi[k2a], wr[k2a], wi[k2a]);
    // 3. R-point DFT across the lanes
    lane_dft8_fwd<R>(yr[k2a], yi[k2a], c, lt);
  }
  // scale by 4 pi^2 kk^2 / n (1/n: the inverse transform is unnormalised)
  const int k2b = bitrev_bits<R>(c);
#pragma unroll
  for (int k2a = 0; k2a < 8; ++k2a) {
    const int k = k1 + 8 * (k2a + 8 * k2b);
    const int kk = (k < n / 2) ? k : k - n;
    const double fac = (lsp::kFourPi2 / n) * (double)(kk * kk);
    yr[k2a] *= fac;
    yi[k2a] *= fac;
  }
#pragma unroll
  for (int k2a = 0; k2a < 8; ++k2a) {
    lane_dft8_inv<R>(yr[k2a], yi[k2a], c, lt);
    cmulc(yr[k2a], yi[k2a], wr[k2a], wi[k2a]);
  }
  RegDft<8, +1>::template run<1>(yr, yi, xr, xi);
  // each thread rewrites exactly the LDS entries it read
#pragma unroll
  for (int b = 0; b < 8; ++b) Ss[k1 * RS + R * b + c] = make_double2(xr[b], xi[b]);
  __syncthreads();

  // 4. memory map: conjugate twiddle, 8-point inverse DFT over k1
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const double2 val = Sm[q * RS + t];
    xr[q] = val.x;
    xi[q] = val.y;
  }
  tw_t.expand(wr, wi);
#pragma unroll
  for (int q = 0; q < 8; ++q) cmulc(xr[q], xi[q], wr[q], wi[q]);
  RegDft<8, +1>::template run<1>(xr, xi, yr, yi);
  if (!active) return;
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const int64_t e = base + (int64_t)(T * a + t) * es;
    double2 r = make_double2(yr[a], yi[a]);
    if constexpr (MODE == kAccum || MODE == kFinal) {
      r.x += zacc[a].x;
      r.y += zacc[a].y;
    }
    if constexpr (MODE == kFinal) {
      r.x += vv[a] * ur[a];
      r.y += vv[a] * ui[a];
    }
    out[e] = r;
  }
}

template <int R>
hipError_t run_fft8_apply(const lsp_problem* p, const double2* u, double2* y, hipStream_t s) {
  constexpr int n = 64 * R;
  constexpr int LPB = kFft8Threads / (8 * R);
  const double2* tw = reinterpret_cast<const double2*>(p->tw);
  double2* z = reinterpret_cast<double2*>(p->z);
  const int64_t N = p->N;
  const int64_t nlines = N / n;
  const int64_t blocks = (nlines + LPB - 1) / LPB;
  for (int ax = 0; ax < p->d - 1; ++ax) {
    int64_t st = 1;
    for (int b = ax + 1; b < p->d; ++b) st *= n;
    if (ax == 0) {
      hipLaunchKernelGGL((fft8_line_kernel<R, false, kFirst>), dim3((unsigned)blocks),
                         dim3(kFft8Threads), 0, s, u, z, (const double2*)nullptr, p->v,
                         tw, nlines, st);
    } else {
      hipLaunchKernelGGL((fft8_line_kernel<R, false, kAccum>), dim3((unsigned)blocks),
                         dim3(kFft8Threads), 0, s, u, z, (const double2*)z, p->v, tw,
                         nlines, st);
    }
  }
  hipLaunchKernelGGL((fft8_line_kernel<R, true, kFinal>), dim3((unsigned)blocks),
                     dim3(kFft8Threads), 0, s, u, y, (const double2*)z, p->v, tw, nlines,
                     (int64_t)1);
  return hipGetLastError();
}

template <int R3>
hipError_t run_fft_apply(const lsp_problem* p, const double2* u, double2* y, hipStream_t s) {
  constexpr int n = 256 * R3;
  constexpr int LPB = kFftThreads / (16 * R3);
  const double2* tw = reinterpret_cast<const double2*>(p->tw);
  double2* z = reinterpret_cast<double2*>(p->z);
  const int64_t N = p->N;
  const int64_t nlines = N / n;
  const int64_t blocks = (nlines + LPB - 1) / LPB;
  for (int ax = 0; ax < p->d - 1; ++ax) {
    int64_t st = 1;
    for (int b = ax + 1; b < p->d; ++b) st *= n;
    if (ax == 0) {
      hipLaunchKernelGGL((fft_line_kernel<R3, false, kFirst>), dim3((unsigned)blocks),
                         dim3(kFftThreads), 0, s, u, z, (const double2*)nullptr, p->v,
                         tw, nlines, st);
    } else {
      hipLaunchKernelGGL((fft_line_kernel<R3, false, kAccum>), dim3((unsigned)blocks),
                         dim3(kFftThreads), 0, s, u, z, (const double2*)z, p->v, tw,
                         nlines, st);
    }
  }
  hipLaunchKernelGGL((fft_line_kernel<R3, true, kFinal>), dim3((unsigned)blocks),
                     dim3(kFftThreads), 0, s, u, y, (const double2*)z, p->v, tw, nlines,
                     (int64_t)1);
  return hipGetLastError();
}


// One pass of L_1 along one axis.
//   CONTIG: the axis is the last (unit stride); lines are rows, nlines of them.
//   !CONTIG: the axis has stride st; lines are indexed (o, i), o < nouter,
//            i < st, and start at o*n*st + i; lanes of a wave run over i so
//            that loads and stores are coalesced.
// MODE: kFirst out = L_1 u; kAccum out = L_1 u + acc; kFinal out = L_1 u + acc + v u.
template <int N1, int N2, int TPB, bool CONTIG, int MODE>
__global__ __launch_bounds__(TPB) void line_op_kernel(const double2* u, double2* out,
                                                      const double2* acc,
                                                      const double* __restrict__ v,
                                                      const double2* __restrict__ tw,
                                                      int64_t nouter, int64_t st) {
  constexpr int n = N1 * N2;
  constexpr int L = TPB / N2;  // lines per work-group
  constexpr int RS = N2 + 1;   // padded LDS row
  __shared__ double2 sh[L * N1 * RS];

  const int tid = threadIdx.x;
  int l, c;
  if constexpr (CONTIG) {
    l = tid / N2;
    c = tid % N2;
  } else {
    l = tid % L;
    c = tid / L;
  }
  int64_t base;
  int64_t es;  // element stride along the line
  bool active;
  if constexpr (CONTIG) {
    int64_t line = (int64_t)blockIdx.x * L + l;
    active = line < nouter;
    base = line * n;
    es = 1;
  } else {
    const int64_t nblk_inner = (st + L - 1) / L;
    const int64_t o = blockIdx.x / nblk_inner;
    const int64_t i = (blockIdx.x % nblk_inner) * L + l;
    active = i < st;
    base = o * n * st + i;
    es = st;
  }

  // ---- phase 1: load x[N2*a + c], N1-point forward DFT over a ----
  double xr[N1], xi[N1];
#pragma unroll
  for (int a = 0; a < N1; ++a) {
    double2 val = make_double2(0.0, 0.0);
    if (active) val = u[base + (int64_t)(N2 * a + c) * es];
    xr[a] = val.x;
    xi[a] = val.y;
  }
  double ur[N1], ui[N1];
  if constexpr (MODE == kFinal) {
#pragma unroll
    for (int a = 0; a < N1; ++a) {
      ur[a] = xr[a];
      ui[a] = xi[a];
    }
  }
  double yr[N1], yi[N1];
  RegDft<N1, -1>::template run<1>(xr, xi, yr, yi);
  {
    // twiddle exp(-2 pi i c k1 / n); products of the table entry are
    // re-seeded from the table every 8 steps to bound rounding growth.
    const double2 w1 = tw[c];
    double2 wk = make_double2(1.0, 0.0);
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) {
      if (k1 % 8 == 0) {
        wk = (k1 == 0) ? make_double2(1.0, 0.0) : tw[c * k1];
      } else {
        const double2 t = wk;
        wk.x = t.x * w1.x - t.y * w1.y;
        wk.y = t.x * w1.y + t.y * w1.x;
      }
      const double a_r = yr[k1], a_i = yi[k1];
      sh[(l * N1 + k1) * RS + c] = make_double2(a_r * wk.x - a_i * wk.y, a_r * wk.y + a_i * wk.x);
    }
  }
  __syncthreads();

  // ---- phase 2/3: thread c = k1 < N1 owns X[k1 + N1 k2], k2 = 0..N2-1 ----
  if (c < N1) {
    const int k1 = c;
    double pr[N2], pi[N2], qr[N2], qi[N2];
#pragma unroll
    for (int b = 0; b < N2; ++b) {
      const double2 val = sh[(l * N1 + k1) * RS + b];
      pr[b] = val.x;
      pi[b] = val.y;
    }
    RegDft<N2, -1>::template run<1>(pr, pi, qr, qi);
    // scale by 4 pi^2 kk^2 / n, kk = k folded to [-n/2, n/2)
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) {
      const int k = k1 + N1 * k2;
      const int kk = (k < n / 2) ? k : k - n;
      const double fac = (lsp::kFourPi2 / n) * (double)(kk * kk);
      qr[k2] *= fac;
      qi[k2] *= fac;
    }
    RegDft<N2, +1>::template run<1>(qr, qi, pr, pi);
    const double2 w1 = tw[k1];  // conj applied below
    double2 wk = make_double2(1.0, 0.0);
#pragma unroll
    for (int b = 0; b < N2; ++b) {
      if (b % 8 == 0) {
        wk = (b == 0) ? make_double2(1.0, 0.0) : tw[b * k1];
      } else {
        const double2 t = wk;
        wk.x = t.x * w1.x - t.y * w1.y;
        wk.y = t.x * w1.y + t.y * w1.x;
      }
      // multiply by conj(wk) = exp(+2 pi i b k1 / n)
      const double a_r = pr[b], a_i = pi[b];
      sh[(l * N1 + k1) * RS + b] = make_double2(a_r * wk.x + a_i * wk.y, a_i * wk.x - a_r * wk.y);
    }
  }
  __syncthreads();

  // ---- phase 4: N1-point inverse DFT over k1, store ----
#pragma unroll
  for (int k1 = 0; k1 < N1; ++k1) {
    const double2 val = sh[(l * N1 + k1) * RS + c];
    xr[k1] = val.x;
    xi[k1] = val.y;
  }
  RegDft<N1, +1>::template run<1>(xr, xi, yr, yi);
  if (!active) return;
#pragma unroll
  for (int a = 0; a < N1; ++a) {
    const int64_t e = base + (int64_t)(N2 * a + c) * es;
    double2 r = make_double2(yr[a], yi[a]);
    if constexpr (MODE == kAccum || MODE == kFinal) {
      const double2 z = acc[e];
      r.x += z.x;
      r.y += z.y;
    }
    if constexpr (MODE == kFinal) {
      const double ve = v[e];
      r.x += ve * ur[a];
      r.y += ve * ui[a];
    }
    out[e] = r;
  }
}

template <int N1, int N2>
hipError_t run_ps_apply(const lsp_problem* p, const double2* u, double2* y, hipStream_t s) {
  constexpr int n = N1 * N2;
  constexpr int TPB_C = (N2 >= 128) ? N2 : 128;
  constexpr int TPB_S = (N2 >= 128) ? N2 : 128;
  const double2* tw = reinterpret_cast<const double2*>(p->tw);
  double2* z = reinterpret_cast<double2*>(p->z);
  const int64_t N = p->N;
  // strided axes 0 .. d-2
  for (int ax = 0; ax < p->d - 1; ++ax) {
    int64_t st = 1;
    for (int b = ax + 1; b < p->d; ++b) st *= n;
    const int64_t nouter = N / (st * n);
    constexpr int L = TPB_S / N2;
    const int64_t blocks = nouter * ((st + L - 1) / L);
    if (ax == 0) {
      hipLaunchKernelGGL((line_op_kernel<N1, N2, TPB_S, false, kFirst>), dim3((unsigned)blocks),
                         dim3(TPB_S), 0, s, u, z, (const double2*)nullptr, p->v, tw,
                         nouter, st);
    } else {
      hipLaunchKernelGGL((line_op_kernel<N1, N2, TPB_S, false, kAccum>), dim3((unsigned)blocks),
                         dim3(TPB_S), 0, s, u, z, (const double2*)z, p->v, tw, nouter,
                         st);
    }
  }
  // contiguous last axis, adds z and v u
  {
    constexpr int L = TPB_C / N2;
    const int64_t nlines = N / n;
    const int64_t blocks = (nlines + L - 1) / L;
    hipLaunchKernelGGL((line_op_kernel<N1, N2, TPB_C, true, kFinal>), dim3((unsigned)blocks),
                       dim3(TPB_C), 0, s, u, y, (const double2*)z, p->v, tw, nlines,
                       (int64_t)1);
  }
  return hipGetLastError();
}

__global__ void count_nonfinite_kernel(const double* __restrict__ x, int64_t count, int* flag) {
  int local = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (!isfinite(x[i])) ++local;
  }
  if (local) atomicAdd(flag, local);
}

}  // namespace

namespace lsp {

hipError_t launch_ps_apply(const lsp_problem* p, const double* u, double* y) {
  return launch_ps_apply(p, u, y, p->stream);
}

hipError_t launch_ps_apply(const lsp_problem* p, const double* u, double* y, hipStream_t s) {
  const double2* u2 = reinterpret_cast<const double2*>(u);
  double2* y2 = reinterpret_cast<double2*>(y);
  switch (p->n) {
    case 8: return run_ps_apply<2, 4>(p, u2, y2, s);
    case 16: return run_ps_apply<4, 4>(p, u2, y2, s);
    case 32: return run_ps_apply<4, 8>(p, u2, y2, s);
    case 64: return run_ps_apply<8, 8>(p, u2, y2, s);
    case 128: return run_ps_apply<8, 16>(p, u2, y2, s);
    // measured per pass at n = 1024: 12.7 + 14.9 us (8 values per thread)
    // against 12.8 + 15.5 us (16 values); at 256 and 512 the 16-value form
    // is 0.1-0.4 us faster
    case 256:
      return p->tune[LSP_TUNE_APPLY_FORM] == 8 ? run_fft8_apply<4>(p, u2, y2, s)
                                               : run_fft_apply<1>(p, u2, y2, s);
    case 512:
      return p->tune[LSP_TUNE_APPLY_FORM] == 8 ? run_fft8_apply<8>(p, u2, y2, s)
                                               : run_fft_apply<2>(p, u2, y2, s);
    case 1024:
      return p->tune[LSP_TUNE_APPLY_FORM] == 16 ? run_fft_apply<4>(p, u2, y2, s)
                                                : run_fft8_apply<16>(p, u2, y2, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_count_nonfinite(const double* x, int64_t count, int* flag, hipStream_t s) {
  hipError_t e = hipMemsetAsync(flag, 0, sizeof(int), s);
  if (e != hipSuccess) return e;
  int64_t blocks = (count + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(count_nonfinite_kernel, dim3((unsigned)blocks), dim3(256), 0, s, x, count,
                     flag);
  return hipGetLastError();
}

}  // namespace lsp
