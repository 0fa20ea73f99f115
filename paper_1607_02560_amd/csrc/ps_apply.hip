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
hipError_t run_ps_apply(const lsp_problem* p, const double2* u, double2* y) {
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
                         dim3(TPB_S), 0, p->stream, u, z, (const double2*)nullptr, p->v, tw,
                         nouter, st);
    } else {
      hipLaunchKernelGGL((line_op_kernel<N1, N2, TPB_S, false, kAccum>), dim3((unsigned)blocks),
                         dim3(TPB_S), 0, p->stream, u, z, (const double2*)z, p->v, tw, nouter,
                         st);
    }
  }
  // contiguous last axis, adds z and v u
  {
    constexpr int L = TPB_C / N2;
    const int64_t nlines = N / n;
    const int64_t blocks = (nlines + L - 1) / L;
    hipLaunchKernelGGL((line_op_kernel<N1, N2, TPB_C, true, kFinal>), dim3((unsigned)blocks),
                       dim3(TPB_C), 0, p->stream, u, y, (const double2*)z, p->v, tw, nlines,
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
  const double2* u2 = reinterpret_cast<const double2*>(u);
  double2* y2 = reinterpret_cast<double2*>(y);
  switch (p->n) {
    case 8: return run_ps_apply<2, 4>(p, u2, y2);
    case 16: return run_ps_apply<4, 4>(p, u2, y2);
    case 32: return run_ps_apply<4, 8>(p, u2, y2);
    case 64: return run_ps_apply<8, 8>(p, u2, y2);
    case 128: return run_ps_apply<8, 16>(p, u2, y2);
    case 256: return run_ps_apply<16, 16>(p, u2, y2);
    case 512: return run_ps_apply<16, 32>(p, u2, y2);
    case 1024: return run_ps_apply<32, 32>(p, u2, y2);
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
