// Fused learned setup: for every grid point, the surrogate network's proposed
// stencil, its check against the exact Gram matrices of eq. (A), and the rows
// of P and C it defines (or the exact rows where the check fails), in one
// pass over the grid.
//
// One block of 8 waves per CU keeps the network's BF16 weights, biases,
// standardisation, the shift list and, per shift, the upper triangles of the
// parity blocks of A1, M and G (see PForms) and rho*(s) in LDS; each wave
// then works alone (no block barrier after the loads) on chunks of 32 points:
//   * one lane per point finds its shift s_j (also the network's last input);
//   * the wave evaluates its 32 points as 2 groups of 16 in the transposed
//     form Z^T = W X^T, so that the accumulator layout of one layer (lane l
//     holds rows 4(l/16)+i, column l%16) is the B-operand layout of the next:
//     two such 16-row tiles side by side are one 32-wide k operand of
//     v_mfma_f32_16x16x32_bf16 (lane group q holds k = 4q .. 4q+3 of each);
//     activations never leave registers, and the output layer accumulates
//     while the second hidden layer is produced tile pair by tile pair; the
//     check's gathers v[mu_j] are issued before the network so that it hides
//     their latency;
//   * the de-standardised FP32 outputs go to the wave's staging rows in LDS;
//     lanes j and j + 32 read point j's row, form the stencil
//     q = p - c (v[mu_j] - s_j), take its parity coordinates and split the
//     forms of eq. (A): one accumulates q^T A1 q, the other q^T M q
//     (M = A1 - G G), each from the block triangles of the point's shift; the
//     point falls back when q^T M q > (rho*(s) + threshold)^2 q^T A1 q;
//   * a kept point's rows are the ones its stencil defines, C = G_mu,mu q
//     (from the G blocks) and P = q + C (v[mu_j] - s_j); a failed point's are
//     the exact rows alpha + C (v[mu_j] - s_j) and C of its shift;
//   * the FP64 rows go through the staging area and leave as contiguous
//     (coalesced) stores of the wave's 32 x m blocks of C and P.
// The network's numerics equal the unfused path's (the same BF16 roundings,
// FP32 bias and SiLU, FP32 de-standardisation); the unfused check sums the
// dense forms instead of the parity blocks, so the two decide alike except
// within rounding of the boundary, and their rows agree to rounding.
#include <map>
#include <mutex>
#include <utility>

#include "setup_common.h"

namespace {

using lsp::nearest_shift;
using lsp::Nbhd;
using lsp::Parity;
using lsp::Pow;

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef short s16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// the operand of one v_mfma_f32_16x16x32_bf16 from two 16-wide k tiles: lane
// group q holds k = 4q .. 4q+3 of the first and of the second tile (the
// placement the network GEMM kernel uses, so both sum in the same order)
__device__ __forceinline__ bf16x8 cat8(bf16x4 lo, bf16x4 hi) {
  s16x8 v;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    v[i] = lo[i];
    v[4 + i] = hi[i];
  }
  return __builtin_bit_cast(bf16x8, v);
}
typedef __bf16 hbf16x4 __attribute__((ext_vector_type(4)));

constexpr int kH = 128;           // hidden width of the fused kernel
constexpr int kWaves = 8;         // waves per block, one block per CU
constexpr int kThreads = 64 * kWaves;
constexpr int kPW = 32;           // points per wave pass
constexpr int kGroups = kPW / 16; // MFMA column groups per pass
constexpr int kWStride = kH + 8;  // LDS row stride (bf16) of W2 and W3: 68 dwords
constexpr size_t kLdsLimit = 163840;  // LDS bytes one workgroup may hold on gfx950

// four FP32 values -> BF16 bits, round to nearest even (v_cvt_pk_bf16_f32),
// the rounding of the unfused kernels
__device__ __forceinline__ bf16x4 to_bf16x4(f32x4 x) {
  return __builtin_bit_cast(bf16x4, __builtin_convertvector(x, hbf16x4));
}

// SiLU with the logistic function of the unfused kernels (hardware reciprocal)
__device__ __forceinline__ float silu(float z) {
  return z * __builtin_amdgcn_rcpf(1.0f + __expf(-z));
}

// The check's forms in the parity basis of the neighbourhood. M = A1 - G G
// and A1 are block diagonal there (one block per parity class; the exact
// setup stores both per shift as packed blocks), so
//   q^T A1 q = sum_c u_c^T A1'_c u_c,   q^T M q = sum_c u_c^T M'_c u_c,
// with u the coordinates of q in the unnormalised basis (entries +-1, the
// orthonormal basis without its 1/sqrt2 factors: u = sums and differences of
// reflected entries of q) and A1' = S A1_b S, M' = S M_b S, S the diagonal
// of those factors. Only the upper triangles are kept, off-diagonal entries
// doubled: 76 entries per form for d = 3, t = 1 instead of the m^2 = 729 of
// the dense forms.
template <int D, int W>
struct PForms {
  using Pa = Parity<D, W>;
  using Nb = Nbhd<D, W>;
  static constexpr int NC = Pa::NC;
  static constexpr int M = Pow<D, W>::v;
  __host__ __device__ static constexpr int base(int c) {  // first coordinate of class c
    int b = 0;
    for (int k = 0; k < c; ++k) b += Pa::size(k);
    return b;
  }
  __host__ __device__ static constexpr int tri(int c) {  // first triangle entry of class c
    int o = 0;
    for (int k = 0; k < c; ++k) o += Pa::size(k) * (Pa::size(k) + 1) / 2;
    return o;
  }
  static constexpr int TRI = tri(NC);
  static constexpr int TRIP = TRI | 1;  // odd stride: shifts fall on different LDS banks
  // number of axes with a nonzero 1D index in row p of class c
  __host__ __device__ static constexpr int nz(int c, int p) {
    int z = 0;
    for (int i = 0; i < D; ++i) z += (Pa::coord(c, p, i) != 0) ? 1 : 0;
    return z;
  }
  // class, row and column of upper-triangle entry k (rows in order, then columns)
  __host__ __device__ static constexpr int cls(int k) {
    int c = 0;
    while (k >= tri(c + 1)) ++c;
    return c;
  }
  __host__ __device__ static constexpr int row(int k) {
    const int c = cls(k), B = Pa::size(c);
    int e = k - tri(c), pr = 0;
    while (e >= B - pr) {
      e -= B - pr;
      ++pr;
    }
    return pr;
  }
  __host__ __device__ static constexpr int col(int k) {
    const int c = cls(k), B = Pa::size(c);
    int e = k - tri(c), pr = 0;
    while (e >= B - pr) {
      e -= B - pr;
      ++pr;
    }
    return pr + e;
  }
  // contribution of offset a to class c: 0 if none, else +-(row + 1)
  __host__ __device__ static constexpr int term(int a, int c) {
    int pidx = 0, sgn = 1;
    for (int i = 0; i < D; ++i) {
      const int x = Nb::comp(a, i);
      const int j = x < 0 ? -x : x;
      const int o = Pa::odd(c, i);
      if (o && j == 0) return 0;
      if (o && x < 0) sgn = -sgn;
      pidx = pidx * Pa::count(c, i) + (j - o);
    }
    return sgn * (pidx + 1);
  }
};

// u += the contribution of q[A] to class C (indices are template constants,
// so u stays in registers)
template <int D, int W, int A, int C>
__device__ __forceinline__ void parity_term(const double* q, double* u) {
  using PF = PForms<D, W>;
  constexpr int tm = PF::term(A, C);
  if constexpr (tm > 0) u[PF::base(C) + tm - 1] += q[A];
  if constexpr (tm < 0) u[PF::base(C) - tm - 1] -= q[A];
}
template <int D, int W, int... I>
__device__ __forceinline__ void parity_coords(const double* q, double* u,
                                              std::integer_sequence<int, I...>) {
  constexpr int NC = 1 << D;
  (parity_term<D, W, I / NC, I % NC>(q, u), ...);
}

// one triangle entry K of the form u^T T u = sum_p u_p (sum_{q >= p} T'_pq u_q)
template <int D, int W, int K>
__device__ __forceinline__ void form_term(const double* tb, const double* u, double& r,
                                          double& acc) {
  using PF = PForms<D, W>;
  constexpr int c = PF::cls(K), pr = PF::row(K), qc = PF::col(K), b0 = PF::base(c);
  if constexpr (qc == pr) r = 0.0;
  r = fma(tb[2 * K], u[b0 + qc], r);
  if constexpr (qc == Parity<D, W>::size(c) - 1) acc = fma(u[b0 + pr], r, acc);
}
template <int D, int W, int... K>
__device__ __forceinline__ double parity_form(const double* tb, const double* u,
                                              std::integer_sequence<int, K...>) {
  double r = 0.0, acc = 0.0;
  (form_term<D, W, K>(tb, u, r, acc), ...);
  return acc;
}

// C = G_mu,mu q in the same basis: G_mu,mu = sum_c U_c G'_c U_c^T with U_c the
// +-1 map of parity_coords and G'_c = S G_b S (full symmetric block, upper
// triangle stored, entries not doubled), so C = sum_c U_c (G'_c u_c). Class
// by class: y_c = G'_c u_c from the triangle, then its entries are scattered
// back to the offsets (the transpose of parity_coords).
template <int D, int W, int K>
__device__ __forceinline__ void gvec_term(const double* gt, const double* u, double* y) {
  using PF = PForms<D, W>;
  constexpr int c = PF::cls(K), pr = PF::row(K), qc = PF::col(K), b0 = PF::base(c);
  const double gv = gt[K];
  y[b0 + pr] = fma(gv, u[b0 + qc], y[b0 + pr]);
  if constexpr (qc != pr) y[b0 + qc] = fma(gv, u[b0 + pr], y[b0 + qc]);
}
template <int D, int W, int A, int C>
__device__ __forceinline__ void unparity_term(const double* y, double* out) {
  using PF = PForms<D, W>;
  constexpr int tm = PF::term(A, C);
  if constexpr (tm > 0) out[A] += y[PF::base(C) + tm - 1];
  if constexpr (tm < 0) out[A] -= y[PF::base(C) - tm - 1];
}
template <int D, int W, int C, int... K>
__device__ __forceinline__ void gvec_class(const double* gt, const double* u, double* y,
                                           std::integer_sequence<int, K...>) {
  (gvec_term<D, W, PForms<D, W>::tri(C) + K>(gt, u, y), ...);
}
template <int D, int W, int C, int... A>
__device__ __forceinline__ void unparity_class(const double* y, double* out,
                                               std::integer_sequence<int, A...>) {
  (unparity_term<D, W, A, C>(y, out), ...);
}
template <int D, int W, int... C>
__device__ __forceinline__ void g_times(const double* gt, const double* u, double* out,
                                        std::integer_sequence<int, C...>) {
  using PF = PForms<D, W>;
  constexpr int M = PF::M;
  double y[M];
#pragma unroll
  for (int k = 0; k < M; ++k) y[k] = 0.0;
  ((gvec_class<D, W, C>(gt, u, y, std::make_integer_sequence<int, PF::tri(C + 1) - PF::tri(C)>{}),
    unparity_class<D, W, C>(y, out, std::make_integer_sequence<int, M>{})),
   ...);
}

// Compile-time geometry of the fused kernel for neighbourhood mu_0^t in D dims.
template <int D, int W>
struct Fused {
  static constexpr int M = Pow<D, W>::v;
  static constexpr int NI = M + 2, NO = 2 * M;
  static constexpr int IP = (NI + 15) / 16 * 16, OP = (NO + 15) / 16 * 16;
  static constexpr int W1S = IP + 8;     // LDS row stride of W1 (bf16): 12 or 20 dwords
  // staging row stride (floats): at least NO rounded up to 4, with stride / 4
  // odd so that 16 lanes' 16-byte accesses to 16 consecutive rows hit
  // distinct banks
  static constexpr int SST0 = (NO + 3) / 4 * 4;
  static constexpr int SST = ((SST0 / 4) % 2) ? SST0 : SST0 + 4;
  static constexpr int NR = (NO + 3) / 4;  // 16-byte reads of one staged row
  static constexpr size_t oW1 = 0;
  static constexpr size_t oW2 = oW1 + 2 * (size_t)kH * W1S;
  static constexpr size_t oW3 = oW2 + 2 * (size_t)kH * kWStride;
  static constexpr size_t oB1 = oW3 + 2 * (size_t)OP * kWStride;
  static constexpr size_t oB2 = oB1 + 4 * kH;
  static constexpr size_t oB3 = oB2 + 4 * kH;
  static constexpr size_t oMX = oB3 + 4 * OP;
  static constexpr size_t oSX = oMX + 4 * IP;
  static constexpr size_t oMY = oSX + 4 * IP;
  static constexpr size_t oSY = oMY + 4 * OP;
  // per-wave area: s_j, 1/|s_j|, staged outputs (FP32 network outputs, then
  // the FP64 rows)
  static constexpr size_t oWave = (oSY + 4 * OP + 15) / 16 * 16;
  static constexpr size_t wSV = 0;
  static constexpr size_t wINV = wSV + 8 * kPW;
  static constexpr size_t wSTG = (wINV + 8 * kPW + 15) / 16 * 16;
  static constexpr size_t WB = (wSTG + 4 * (size_t)kPW * SST + 15) / 16 * 16;
  // per shift: S, the Gram triangles {A1', M'} (PForms), the triangle of G'
  // and rho*(s); the triangles start 16-byte aligned after the (even-padded)
  // shift list
  static constexpr int TRIP = PForms<D, W>::TRIP;
  static constexpr size_t oS = oWave + WB * kWaves;
  static constexpr size_t tab_off(int shifts) { return oS + 8 * (size_t)((shifts + 1) & ~1); }
  static constexpr size_t gt_off(int shifts) { return tab_off(shifts) + 16 * (size_t)TRIP * shifts; }
  static constexpr size_t rho_off(int shifts) { return gt_off(shifts) + 8 * (size_t)TRIP * shifts; }
  // LDS bytes for a shift list of up to `shifts` entries
  static constexpr size_t bytes(int shifts) { return rho_off(shifts) + 8 * (size_t)shifts; }
  static_assert(IP <= 32 && OP <= 64, "fused kernel sizes");
  static_assert(NR * 4 <= SST && wSTG % 16 == 0, "staging layout");
  static_assert(2 * kPW * M <= kPW * SST, "FP64 rows of a pass fit the staging area");
};

// makes the wave's LDS writes visible to its other lanes (LDS operations of a
// wave complete in order; the fences keep the compiler from moving them)
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// the same entry as the exact setup's assembly: product and sum rounded separately
__device__ __forceinline__ double exact_entry(double alpha, double c, double v_minus_s) {
#pragma clang fp contract(off)
  return alpha + c * v_minus_s;
}

// flat index of (c + offset a) mod n for a runtime offset index a
template <int D, int W>
__device__ __forceinline__ int64_t neighbour_rt(const int* c, int logn, int a) {
  constexpr int t = (W - 1) / 2;
  const int mask = (1 << logn) - 1;
  int comp[D];
#pragma unroll
  for (int i = D - 1; i >= 0; --i) {
    comp[i] = a % W - t;
    a /= W;
  }
  int64_t g = 0;
#pragma unroll
  for (int i = 0; i < D; ++i) g = (g << logn) | ((c[i] + comp[i]) & mask);
  return g;
}

// flat index of (c + offset a) mod n for a compile-time offset index a
template <int D, int W>
__device__ __forceinline__ int64_t neighbour_ct(const int* c, int logn, int a) {
  using Nb = Nbhd<D, W>;
  const int mask = (1 << logn) - 1;
  int64_t g = 0;
#pragma unroll
  for (int i = 0; i < D; ++i) g = (g << logn) | ((c[i] + Nb::comp(a, i)) & mask);
  return g;
}

template <int D>
__device__ __forceinline__ void coords(int64_t j, int logn, int* c) {
  const int mask = (1 << logn) - 1;
#pragma unroll
  for (int i = D - 1; i >= 0; --i) {
    c[i] = (int)(j & mask);
    j >>= logn;
  }
}

struct NetPtrs {
  const unsigned short* W1;  // [kH][IP]
  const unsigned short* W2;  // [kH][kH]
  const unsigned short* W3;  // [OP][kH]
  const float* b1;
  const float* b2;
  const float* b3;           // [OP]
  const float* norm;         // mu_x [NI], sd_x [NI], mu_y [NO], sd_y [NO]
};

// One 8-wave block per CU (its LDS allows no second), i.e. two waves per
// SIMD: the attribute lets the compiler schedule for exactly that occupancy.
template <int D, int W>
__global__ __launch_bounds__(kThreads, 1)
__attribute__((amdgpu_waves_per_eu(2, 2))) void learned_fused_kernel(
    const double* __restrict__ v, int logn, int64_t N, double h2, const double* __restrict__ S,
    const int* __restrict__ nS_ptr, const double* __restrict__ Mtab,
    const double2* __restrict__ actab,
    const double* __restrict__ rho_star, double thr, NetPtrs net, int64_t nchunks,
    double* __restrict__ P, double* __restrict__ Crows, int32_t* __restrict__ fallback,
    int* __restrict__ nfall) {
  using Pa = Parity<D, W>;
  using PF = PForms<D, W>;
  using F = Fused<D, W>;
  constexpr int M = F::M, NI = F::NI, NO = F::NO, IP = F::IP, OP = F::OP, SST = F::SST;
  constexpr int KC1 = IP / 16, KC = kH / 16, OT = OP / 16;
  extern __shared__ __align__(16) char lds[];
  unsigned short* W1s = reinterpret_cast<unsigned short*>(lds + F::oW1);
  unsigned short* W2s = reinterpret_cast<unsigned short*>(lds + F::oW2);
  unsigned short* W3s = reinterpret_cast<unsigned short*>(lds + F::oW3);
  float* b1s = reinterpret_cast<float*>(lds + F::oB1);
  float* b2s = reinterpret_cast<float*>(lds + F::oB2);
  float* b3s = reinterpret_cast<float*>(lds + F::oB3);
  float* mxs = reinterpret_cast<float*>(lds + F::oMX);
  float* sxs = reinterpret_cast<float*>(lds + F::oSX);
  float* mys = reinterpret_cast<float*>(lds + F::oMY);
  float* sys = reinterpret_cast<float*>(lds + F::oSY);
  double* Ss = reinterpret_cast<double*>(lds + F::oS);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  char* wa = lds + F::oWave + wave * F::WB;
  double* sv = reinterpret_cast<double*>(wa + F::wSV);
  double* iv = reinterpret_cast<double*>(wa + F::wINV);
  float* stg = reinterpret_cast<float*>(wa + F::wSTG);

  // ---- network, shift list, Gram triangles and rho* into LDS (once per block) ----
  for (int e = tid; e < kH * IP / 4; e += kThreads) {
    const int r = e / (IP / 4), c = (e % (IP / 4)) * 4;
    *reinterpret_cast<uint2*>(W1s + r * F::W1S + c) =
        *reinterpret_cast<const uint2*>(net.W1 + (size_t)r * IP + c);
  }
  for (int e = tid; e < kH * kH / 4; e += kThreads) {
    const int r = e / (kH / 4), c = (e % (kH / 4)) * 4;
    *reinterpret_cast<uint2*>(W2s + r * kWStride + c) =
        *reinterpret_cast<const uint2*>(net.W2 + (size_t)r * kH + c);
  }
  for (int e = tid; e < OP * kH / 4; e += kThreads) {
    const int r = e / (kH / 4), c = (e % (kH / 4)) * 4;
    *reinterpret_cast<uint2*>(W3s + r * kWStride + c) =
        *reinterpret_cast<const uint2*>(net.W3 + (size_t)r * kH + c);
  }
  for (int e = tid; e < kH; e += kThreads) {
    b1s[e] = net.b1[e];
    b2s[e] = net.b2[e];
  }
  for (int e = tid; e < OP; e += kThreads) {
    b3s[e] = net.b3[e];
    mys[e] = (e < NO) ? net.norm[2 * NI + e] : 0.f;
    sys[e] = (e < NO) ? net.norm[2 * NI + NO + e] : 1.f;
  }
  for (int e = tid; e < IP; e += kThreads) {
    mxs[e] = (e < NI) ? net.norm[e] : 0.f;
    sxs[e] = (e < NI) ? 1.0f / net.norm[NI + e] : 1.f;  // reciprocal deviation
  }
  const int nS = *nS_ptr;
  double2* Tb = reinterpret_cast<double2*>(lds + F::tab_off(nS));
  double* Gt = reinterpret_cast<double*>(lds + F::gt_off(nS));
  double* rs = reinterpret_cast<double*>(lds + F::rho_off(nS));
  for (int e = tid; e < nS; e += kThreads) {
    Ss[e] = S[e];
    rs[e] = rho_star[e];
  }
  // triangle entry k of shift si: {A1'[p][q], M'[p][q]} of its class block,
  // scaled by the 1/sqrt2 factors of rows p and q, off-diagonals doubled
  // (decoded incrementally here: the generic helpers loop over the classes
  // once per call, which made this prologue several microseconds slower)
  for (int e = tid; e < nS * PF::TRI; e += kThreads) {
    const int si = e / PF::TRI, k = e - si * PF::TRI;
    int c = 0, rem = k;
    while (rem >= Pa::size(c) * (Pa::size(c) + 1) / 2) {
      rem -= Pa::size(c) * (Pa::size(c) + 1) / 2;
      ++c;
    }
    const int B = Pa::size(c);
    int pr = 0;
    while (rem >= B - pr) {
      rem -= B - pr;
      ++pr;
    }
    const int qc = pr + rem;
    const int z = PF::nz(c, pr) + PF::nz(c, qc);
    double f = ldexp(1.0, -(z / 2));
    if (z & 1) f *= lsp::kInvSqrt2;
    const double* blk = Mtab + (int64_t)si * M * M + Pa::offset(c) + pr * B + qc;
    Gt[si * PF::TRIP + k] = blk[2 * Pa::offset(Pa::NC)] * f;  // G' (not doubled)
    if (qc != pr) f *= 2.0;
    Tb[si * PF::TRIP + k] = make_double2(blk[Pa::offset(Pa::NC)] * f, blk[0] * f);
  }
  __syncthreads();  // the last block-wide barrier: from here on every wave works alone

  const int r16 = lane & 15, qd = lane >> 4;
  const int pl = lane & 31, half = lane >> 5;  // check: point pl, twice per wave
  int nf_local = 0;
  for (int64_t chunk = (int64_t)blockIdx.x * kWaves + wave; chunk < nchunks;
       chunk += (int64_t)gridDim.x * kWaves) {
    const int64_t wbase = chunk * kPW;
    // ---- the shift of each point ----
    const int64_t j = wbase + pl;
    const bool valid = j < N;
    int id = 0;
    if (valid) id = nearest_shift(Ss, nS, v[j]);
    const double s = Ss[id];
    if (half == 0) {
      sv[pl] = s;
      iv[pl] = 1.0 / fabs(s);
    }
    wave_sync();

    // ---- network: 2 groups of 16 points ----
    // inputs: h^2 v_j, the patch h^2 v[j + a], h^2 s_j; every lane loads its
    // 4 KC1 values unconditionally (clamped addresses) so the loads overlap
    bf16x4 xb[kGroups][KC1];
#pragma unroll
    for (int g = 0; g < kGroups; ++g) {
      const int64_t pt = wbase + 16 * g + r16;
      const bool pvalid = pt < N;
      const int64_t ptc = pvalid ? pt : 0;
      int c[D];
      coords<D>(ptc, logn, c);
      double raw[KC1][4];
#pragma unroll
      for (int kc = 0; kc < KC1; ++kc)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int k = 16 * kc + 4 * qd + i;
          const int a = k < 1 ? 0 : (k > M ? M - 1 : k - 1);
          const int64_t at = (k >= 1 && k <= M) ? neighbour_rt<D, W>(c, logn, a) : ptc;
          raw[kc][i] = v[at];
        }
      const double sj = sv[16 * g + r16];
#pragma unroll
      for (int kc = 0; kc < KC1; ++kc) {
        f32x4 xf;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int k = 16 * kc + 4 * qd + i;
          const double val = (k <= M) ? raw[kc][i] : sj;
          const float xs = ((float)(h2 * val) - mxs[k]) * sxs[k];
          xf[i] = (pvalid && k < NI) ? xs : 0.f;
        }
        xb[g][kc] = to_bf16x4(xf);
      }
    }
    // the check's gathers v[mu_j] (lane pl: point j), issued here so that the
    // network hides their latency
    int c[D];
    coords<D>(valid ? j : 0, logn, c);
    double vq[M];
#pragma unroll
    for (int a = 0; a < M; ++a) vq[a] = v[neighbour_ct<D, W>(c, logn, a)];
    bf16x4 a1[kGroups][KC];
#pragma unroll
    for (int ht = 0; ht < KC; ++ht) {
      f32x4 acc[kGroups];
#pragma unroll
      for (int g = 0; g < kGroups; ++g) acc[g] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kc = 0; kc + 1 < KC1; kc += 2) {
        const unsigned short* wr = W1s + (16 * ht + r16) * F::W1S + 16 * kc + 4 * qd;
        const bf16x8 A = cat8(*reinterpret_cast<const bf16x4*>(wr),
                              *reinterpret_cast<const bf16x4*>(wr + 16));
#pragma unroll
        for (int g = 0; g < kGroups; ++g)
          acc[g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, cat8(xb[g][kc], xb[g][kc + 1]),
                                                           acc[g], 0, 0, 0);
      }
      if constexpr (KC1 % 2 == 1) {
        const bf16x4 A = *reinterpret_cast<const bf16x4*>(W1s + (16 * ht + r16) * F::W1S +
                                                          16 * (KC1 - 1) + 4 * qd);
#pragma unroll
        for (int g = 0; g < kGroups; ++g)
          acc[g] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, xb[g][KC1 - 1], acc[g], 0, 0, 0);
      }
#pragma unroll
      for (int g = 0; g < kGroups; ++g) {
        f32x4 z;
#pragma unroll
        for (int i = 0; i < 4; ++i) z[i] = silu(acc[g][i] + b1s[16 * ht + 4 * qd + i]);
        a1[g][ht] = to_bf16x4(z);
      }
    }
    // second hidden layer tile by tile; each finished tile (16 hidden units)
    // is at once the next K chunk of the output layer
    f32x4 acc3[kGroups][OT];
#pragma unroll
    for (int g = 0; g < kGroups; ++g)
#pragma unroll
      for (int ot = 0; ot < OT; ++ot) acc3[g][ot] = f32x4{0.f, 0.f, 0.f, 0.f};
    static_assert(KC % 2 == 0, "hidden width: whole pairs of 16-wide tiles");
    // second-layer tiles in pairs: tile ht of z2 = W2 a1, SiLU, and the pair
    // (ht, ht+1) is the next 32-wide K block of the output layer
#pragma unroll
    for (int hp = 0; hp < KC; hp += 2) {
      bf16x4 a2[2][kGroups];
#pragma unroll
      for (int h2i = 0; h2i < 2; ++h2i) {
        const int ht = hp + h2i;
        f32x4 acc[kGroups];
#pragma unroll
        for (int g = 0; g < kGroups; ++g) acc[g] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kc = 0; kc < KC; kc += 2) {
          const unsigned short* wr = W2s + (16 * ht + r16) * kWStride + 16 * kc + 4 * qd;
          const bf16x8 A = cat8(*reinterpret_cast<const bf16x4*>(wr),
                                *reinterpret_cast<const bf16x4*>(wr + 16));
#pragma unroll
          for (int g = 0; g < kGroups; ++g)
            acc[g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, cat8(a1[g][kc], a1[g][kc + 1]),
                                                             acc[g], 0, 0, 0);
        }
#pragma unroll
        for (int g = 0; g < kGroups; ++g) {
          f32x4 z;
#pragma unroll
          for (int i = 0; i < 4; ++i) z[i] = silu(acc[g][i] + b2s[16 * ht + 4 * qd + i]);
          a2[h2i][g] = to_bf16x4(z);
        }
      }
#pragma unroll
      for (int ot = 0; ot < OT; ++ot) {
        const unsigned short* wr = W3s + (16 * ot + r16) * kWStride + 16 * hp + 4 * qd;
        const bf16x8 A = cat8(*reinterpret_cast<const bf16x4*>(wr),
                              *reinterpret_cast<const bf16x4*>(wr + 16));
#pragma unroll
        for (int g = 0; g < kGroups; ++g)
          acc3[g][ot] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, cat8(a2[0][g], a2[1][g]),
                                                               acc3[g][ot], 0, 0, 0);
      }
    }
    // de-standardised outputs y_o to the staging row of their point
    // (o < m: P entries, m <= o < 2m: C entries before the 1/|s| scaling)
#pragma unroll
    for (int g = 0; g < kGroups; ++g)
#pragma unroll
      for (int ot = 0; ot < OT; ++ot) {
        const int o0 = 16 * ot + 4 * qd;
        if (o0 < NO) {
          f32x4 y;
#pragma unroll
          for (int i = 0; i < 4; ++i)
            y[i] = mys[o0 + i] + sys[o0 + i] * (acc3[g][ot][i] + b3s[o0 + i]);
          *reinterpret_cast<f32x4*>(stg + (16 * g + r16) * SST + o0) = y;
        }
      }
    wave_sync();

    // ---- check, one lane per point (lanes pl and pl + 32 alike) ----
    const double inv = iv[pl];
    double q[M];
    {
      const float* row = stg + pl * SST;
      f32x4 yr[F::NR];
#pragma unroll
      for (int u = 0; u < F::NR; ++u) yr[u] = *reinterpret_cast<const f32x4*>(row + 4 * u);
#pragma unroll
      for (int a = 0; a < M; ++a) {
        const double vm = vq[a] - s;
        const double pa = (double)yr[a / 4][a % 4];
        const double ca = (double)yr[(M + a) / 4][(M + a) % 4] * inv;
        q[a] = pa - ca * vm;
      }
    }
    // rho = sqrt(q^T M q / q^T A1 q) of eq. (A) in the parity basis: u are
    // q's unnormalised parity coordinates; lane pl accumulates u^T A1' u, lane
    // pl + 32 u^T M' u from the point's shift triangles
    double u[M];
#pragma unroll
    for (int k = 0; k < M; ++k) u[k] = 0.0;
    parity_coords<D, W>(q, u, std::make_integer_sequence<int, M * PF::NC>{});
    double qaq, qmq;
    {
      const double* tb = reinterpret_cast<const double*>(Tb + id * PF::TRIP) + (half ? 1 : 0);
      const double acc = parity_form<D, W>(tb, u, std::make_integer_sequence<int, PF::TRI>{});
      const double other = __shfl_xor(acc, 32);
      qaq = half ? other : acc;
      qmq = half ? acc : other;
    }
    const double lim = rs[id] + thr;
    const bool ok = valid && (qaq > 0.0) && isfinite(qmq) && (qmq <= lim * lim * qaq);
    if (half == 0 && valid) fallback[j] = ok ? 0 : 1;
    nf_local += __popcll(__ballot(half == 0 && valid && !ok));

    // ---- the point's rows. The network only proposes the stencil q (the
    // row of Q); a kept point takes the rows that stencil defines:
    // C = (Q G)[j, mu_j] = G_mu,mu q and P = q + C (v[mu_j] - s_j) (Sec. 4.1,
    // eq. PC), so its row of C A - P differs from zero only by the truncated
    // part that rho measures. A failed point takes its shift's exact rows
    // alpha + C (v[mu_j] - s_j) and C. ----
    double cr[M];
#pragma unroll
    for (int a = 0; a < M; ++a) cr[a] = 0.0;
    g_times<D, W>(Gt + id * PF::TRIP, u, cr, std::make_integer_sequence<int, PF::NC>{});
    if (!ok) {
#pragma unroll
      for (int a = 0; a < M; ++a) {
        const double2 ac = actab[(int64_t)id * M + a];
        q[a] = ac.x;
        cr[a] = ac.y;
      }
    }
    // both halves hold the same rows; each stages half of every row (FP64)
    // in the wave's staging area, whose FP32 outputs every lane has read, and
    // the wave's 32 x m block then leaves as contiguous stores
    double* stgd = reinterpret_cast<double*>(stg);
    constexpr int HM = (M + 1) / 2;
    const int64_t rbase = wbase * M;
    const int rend = (int)((N - wbase < kPW ? N - wbase : kPW) * M);  // entries of valid points
    wave_sync();
#pragma unroll
    for (int i = 0; i < HM; ++i) {
      const double hi = (HM + i < M) ? cr[(HM + i < M) ? HM + i : 0] : 0.0;
      if (half == 0) stgd[pl * M + i] = cr[i];
      else if (HM + i < M) stgd[pl * M + HM + i] = hi;
    }
    wave_sync();
#pragma unroll
    for (int w = 0; w < (kPW * M + 63) / 64; ++w) {
      const int e = lane + 64 * w;
      if (e < rend) Crows[rbase + e] = stgd[e];
    }
    // P entries with the rounding of the exact assembly (product and sum
    // rounded separately)
#pragma unroll
    for (int a = 0; a < M; ++a) q[a] = exact_entry(q[a], cr[a], vq[a] - s);
    wave_sync();
#pragma unroll
    for (int i = 0; i < HM; ++i) {
      const double hi = (HM + i < M) ? q[(HM + i < M) ? HM + i : 0] : 0.0;
      if (half == 0) stgd[pl * M + i] = q[i];
      else if (HM + i < M) stgd[pl * M + HM + i] = hi;
    }
    wave_sync();
#pragma unroll
    for (int w = 0; w < (kPW * M + 63) / 64; ++w) {
      const int e = lane + 64 * w;
      if (e < rend) P[rbase + e] = stgd[e];
    }
    wave_sync();  // the wave's LDS area is rewritten by its next chunk
  }
  if (lane == 0 && nf_local) atomicAdd(nfall, nf_local);
}

template <int D, int W>
hipError_t launch_fused_dw(const lsp_problem* p, const lsp::MlpView& mv, double thr,
                           const double* rho_star, double* P, double* Crows, int32_t* fallback,
                           int* nfall) {
  using F = Fused<D, W>;
  const size_t lds = F::bytes(p->num_shifts);
  if (lds > kLdsLimit) return hipErrorInvalidValue;  // excluded by learned_fused_supported
  // The kernel's dynamic-LDS attribute and its occupancy are properties of
  // the function on one device, shared by every problem object that launches
  // it there: keep them per device and update them under a lock, so problems
  // used from different threads do not race on them.
  struct Attr {
    size_t bytes = 0;
    int per_cu = 1;
  };
  static std::mutex mu;
  static std::map<int, Attr> attrs;
  int per_cu = 1;
  {
    std::lock_guard<std::mutex> lock(mu);
    Attr& at = attrs[p->device];
    if (at.bytes < lds) {
      hipError_t e =
          hipFuncSetAttribute(reinterpret_cast<const void*>(&learned_fused_kernel<D, W>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
      int nb = 0;
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &nb, reinterpret_cast<const void*>(&learned_fused_kernel<D, W>), kThreads, lds);
      if (e != hipSuccess) return e;
      if (nb < 1) return hipErrorInvalidConfiguration;
      at.bytes = lds;
      at.per_cu = nb;
    }
    per_cu = at.per_cu;
  }
  int cus = 0;
  hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device);
  if (e != hipSuccess) return e;
  const int64_t nchunks = (p->N + kPW - 1) / kPW;
  const int64_t want = (nchunks + kWaves - 1) / kWaves;
  const int blocks = (int)std::min<int64_t>(want, (int64_t)per_cu * cus);
  int logn = 0;
  while ((1 << logn) < p->n) ++logn;
  NetPtrs net{mv.W1, mv.W2, mv.W3, mv.b1, mv.b2, mv.b3, mv.norm};
  hipLaunchKernelGGL((learned_fused_kernel<D, W>), dim3(blocks), dim3(kThreads), lds,
                     p->stream, p->v, logn, p->N, 1.0 / ((double)p->n * p->n), p->ws.S, p->ws.nS,
                     p->ws.Mtab, reinterpret_cast<const double2*>(p->ws.actab), rho_star, thr,
                     net, nchunks, P, Crows, fallback, nfall);
  return hipGetLastError();
}

}  // namespace

namespace lsp {

bool learned_fused_supported(const lsp_problem* p, const MlpView& mv) {
  const int W = 2 * p->t + 1;
  const bool shape = (p->d == 2 && (W == 3 || W == 5)) || (p->d == 3 && W == 3);
  if (!shape || mv.n_hidden != kH) return false;
  size_t lds = 0;
  if (p->d == 2) lds = (W == 3) ? Fused<2, 3>::bytes(p->num_shifts) : Fused<2, 5>::bytes(p->num_shifts);
  else lds = Fused<3, 3>::bytes(p->num_shifts);
  return lds <= kLdsLimit;
}

hipError_t launch_learned_fused(const lsp_problem* p, const MlpView& mv, double thr,
                                const double* rho_star, double* P, double* Crows,
                                int32_t* fallback, int* nfall) {
  const int W = 2 * p->t + 1;
  if (p->d == 2 && W == 3)
    return launch_fused_dw<2, 3>(p, mv, thr, rho_star, P, Crows, fallback, nfall);
  if (p->d == 2 && W == 5)
    return launch_fused_dw<2, 5>(p, mv, thr, rho_star, P, Crows, fallback, nfall);
  if (p->d == 3 && W == 3)
    return launch_fused_dw<3, 3>(p, mv, thr, rho_star, P, Crows, fallback, nfall);
  return hipErrorInvalidValue;
}

}  // namespace lsp
