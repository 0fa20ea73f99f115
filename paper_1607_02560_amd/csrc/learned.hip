// Fused learned setup: for every grid point, the surrogate network's P and C
// rows, the check of the predicted stencil against the exact Gram matrices of
// eq. (A), and the exact row where the check fails, in one pass over the grid.
//
// Per block of 4 waves (persistent over chunks of 256 points, two blocks per
// CU):
//   * the network's BF16 weights, biases, standardisation and the shift list
//     sit in LDS; one lane per point first finds its shift s_j (also the
//     network's last input);
//   * each wave evaluates 64 points as 4 groups of 16 with
//     v_mfma_f32_16x16x16bf16 in the transposed form Z^T = W X^T, so that the
//     accumulator layout of one layer (lane l holds rows 4(l/16)+i, column
//     l%16) is exactly the B-operand layout of the next: activations never
//     leave registers, and the output layer accumulates while the second
//     hidden layer is produced;
//   * the de-standardised outputs are written straight to the P and C rows;
//     one lane per point reads its rows back (L2), forms q = p - c (v[mu_j] -
//     s_j) and decides with one quadratic form q^T K_s q <= 0, K_s = M_s -
//     (rho*(s) + threshold)^2 A1_s (eq. A), whose packed upper triangle is
//     staged in LDS once per distinct shift of the wave and read as
//     broadcasts; rows that fail are overwritten with the exact rows.
// Numerics equal the unfused path: the same BF16 roundings, FP32 bias and
// SiLU, FP32 de-standardisation, FP64 check and rows.
#include "setup_common.h"

namespace {

using lsp::nearest_shift;
using lsp::Nbhd;
using lsp::Pow;

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 hbf16x4 __attribute__((ext_vector_type(4)));

constexpr int kH = 128;           // hidden width of the fused kernel
constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;
constexpr int kPts = kThreads;    // points per block pass (one per lane)
constexpr int kWStride = kH + 8;  // LDS row stride (bf16) of W2 and W3: 68 dwords

// four FP32 values -> BF16 bits, round to nearest even (v_cvt_pk_bf16_f32),
// the rounding of the unfused kernels
__device__ __forceinline__ bf16x4 to_bf16x4(f32x4 x) {
  return __builtin_bit_cast(bf16x4, __builtin_convertvector(x, hbf16x4));
}

// SiLU with the logistic function of the unfused kernels (hardware reciprocal)
__device__ __forceinline__ float silu(float z) {
  return z * __builtin_amdgcn_rcpf(1.0f + __expf(-z));
}

// Compile-time geometry of the fused kernel for neighbourhood mu_0^t in D dims.
template <int D, int W>
struct Fused {
  static constexpr int M = Pow<D, W>::v;
  static constexpr int NI = M + 2, NO = 2 * M;
  static constexpr int IP = (NI + 15) / 16 * 16, OP = (NO + 15) / 16 * 16;
  static constexpr int W1S = IP + 8;     // LDS row stride of W1 (bf16): 12 or 20 dwords
  static constexpr int MM = M * (M + 1) / 2;
  static constexpr int KS = (MM + 15) / 16 * 16;  // doubles per shift of packed K
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
  static constexpr size_t oSV = (oSY + 4 * OP + 15) / 16 * 16;      // s_j, 64 per wave
  static constexpr size_t oK = oSV + 8 * 64 * (size_t)kWaves;        // K_s, one per wave
  static constexpr size_t oS = oK + 8 * (size_t)KS * kWaves;         // shift list
  // LDS bytes for a shift list of up to `shifts` entries
  static constexpr size_t bytes(int shifts) { return oS + 8 * (size_t)shifts; }
  static_assert(IP <= 32 && OP <= 64, "fused kernel sizes");
};

// the same entry as the exact setup's assembly: product and sum rounded separately
__device__ __forceinline__ double exact_entry(double alpha, double c, double v_minus_s) {
#pragma clang fp contract(off)
  return alpha + c * v_minus_s;
}

// Packed K_s of every shift: for a <= b, K'[a][b] = (a == b ? 1 : 2) *
// (M_ab - lim^2 A1_ab), lim = rho*(s) + thr, with A1_ab = gam[|a - b|],
// M = A1 - G G (G_ab = g[|a - b|]; eq. A) and rho*(s) of the shift's exact
// stencil alpha_s. One block of 256 threads per shift (tables staged in LDS);
// block 0 also clears the fallback counter.
template <int D, int W>
__global__ __launch_bounds__(256) void kform_kernel(const double* __restrict__ gtab,
                                                    const double* __restrict__ gamtab,
                                                    const double2* __restrict__ actab,
                                                    const int* __restrict__ nS_ptr, double thr,
                                                    double* rho_star, double* Kf, int* nfall) {
  using Nb = Nbhd<D, W>;
  using F = Fused<D, W>;
  constexpr int M = F::M;
  const int si = blockIdx.x;
  const int tid = threadIdx.x;
  if (si == 0 && tid == 0) *nfall = 0;  // fallback count of the pass that follows
  if (si >= *nS_ptr) return;            // uniform over the block
  __shared__ double g[M], gm[M], al[M];
  __shared__ int dix[M][M];             // table index of |a - b|
  __shared__ double red[2][256];
  if (tid < M) {
    g[tid] = gtab[(int64_t)si * M + tid];
    gm[tid] = gamtab[(int64_t)si * M + tid];
    al[tid] = actab[(int64_t)si * M + tid].x;
  }
  for (int e = tid; e < M * M; e += 256) dix[e / M][e % M] = Nb::diff_index(e / M, e % M);
  __syncthreads();
  double u = 0.0, w = 0.0;
  if (tid < M) {
    for (int b = 0; b < M; ++b) {
      u = fma(g[dix[tid][b]], al[b], u);
      w = fma(gm[dix[tid][b]], al[b], w);
    }
    w *= al[tid];
    u *= u;
  }
  red[0][tid] = u;
  red[1][tid] = w;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) {
      red[0][tid] += red[0][tid + o];
      red[1][tid] += red[1][tid + o];
    }
    __syncthreads();
  }
  const double qaq = red[1][0], qmq = qaq - red[0][0];
  const double rs = sqrt(fmax(qmq, 0.0) / qaq);
  if (tid == 0) rho_star[si] = rs;
  const double lim = rs + thr, lim2 = lim * lim;
  for (int e = tid; e < F::MM; e += 256) {
    int r = 0, start = 0;
    while (start + (M - r) <= e) {
      start += M - r;
      ++r;
    }
    const int c = r + (e - start);
    double gg = 0.0;
    for (int k = 0; k < M; ++k) gg = fma(g[dix[r][k]], g[dix[k][c]], gg);
    const double a1 = gm[dix[r][c]];
    const double kv = (a1 - gg) - lim2 * a1;
    Kf[(int64_t)si * F::KS + e] = (r == c) ? kv : 2.0 * kv;
  }
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

template <int D, int W>
__global__ __launch_bounds__(kThreads, 2) void learned_fused_kernel(
    const double* __restrict__ v, int logn, int64_t N, double h2, const double* __restrict__ S,
    const int* __restrict__ nS_ptr, const double2* __restrict__ actab,
    const double* __restrict__ Kf, NetPtrs net, int nchunks, double* P, double* Crows,
    int32_t* __restrict__ fallback, int* __restrict__ nfall) {
  using F = Fused<D, W>;
  constexpr int M = F::M, NI = F::NI, NO = F::NO, IP = F::IP, OP = F::OP;
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
  double* sw = reinterpret_cast<double*>(lds + F::oSV) + wave * 64;
  double* Kw = reinterpret_cast<double*>(lds + F::oK) + wave * F::KS;

  // ---- network and shift list into LDS (once per block) ----
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
  for (int e = tid; e < nS; e += kThreads) Ss[e] = S[e];
  __syncthreads();

  const int r16 = lane & 15, qd = lane >> 4;
  int nf_local = 0;
  for (int chunk = blockIdx.x; chunk < nchunks; chunk += gridDim.x) {
    const int64_t wbase = (int64_t)chunk * kPts + wave * 64;
    // ---- the shift of each point (one lane per point) ----
    const int64_t j = wbase + lane;
    const bool valid = j < N;
    int id = 0;
    if (valid) id = nearest_shift(Ss, nS, v[j]);
    const double s = Ss[id];
    sw[lane] = s;
    __syncthreads();

    // ---- network: 4 groups of 16 points per wave ----
    // inputs: h^2 v_j, the patch h^2 v[j + a], h^2 s_j; every lane loads its
    // 4 KC1 values unconditionally (clamped addresses) so the loads overlap
    bf16x4 xb[4][KC1];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
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
      const double sj = sw[16 * g + r16];
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
    bf16x4 a1[4][KC];
#pragma unroll
    for (int ht = 0; ht < KC; ++ht) {
      f32x4 acc[4];
#pragma unroll
      for (int g = 0; g < 4; ++g) acc[g] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kc = 0; kc < KC1; ++kc) {
        const bf16x4 A =
            *reinterpret_cast<const bf16x4*>(W1s + (16 * ht + r16) * F::W1S + 16 * kc + 4 * qd);
#pragma unroll
        for (int g = 0; g < 4; ++g)
          acc[g] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, xb[g][kc], acc[g], 0, 0, 0);
      }
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        f32x4 z;
#pragma unroll
        for (int i = 0; i < 4; ++i) z[i] = silu(acc[g][i] + b1s[16 * ht + 4 * qd + i]);
        a1[g][ht] = to_bf16x4(z);
      }
    }
    // second hidden layer tile by tile; each finished tile (16 hidden units)
    // is at once the next K chunk of the output layer
    f32x4 acc3[4][OT];
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
      for (int ot = 0; ot < OT; ++ot) acc3[g][ot] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ht = 0; ht < KC; ++ht) {
      f32x4 acc[4];
#pragma unroll
      for (int g = 0; g < 4; ++g) acc[g] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kc = 0; kc < KC; ++kc) {
        const bf16x4 A =
            *reinterpret_cast<const bf16x4*>(W2s + (16 * ht + r16) * kWStride + 16 * kc + 4 * qd);
#pragma unroll
        for (int g = 0; g < 4; ++g)
          acc[g] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, a1[g][kc], acc[g], 0, 0, 0);
      }
      bf16x4 a2[4];
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        f32x4 z;
#pragma unroll
        for (int i = 0; i < 4; ++i) z[i] = silu(acc[g][i] + b2s[16 * ht + 4 * qd + i]);
        a2[g] = to_bf16x4(z);
      }
#pragma unroll
      for (int ot = 0; ot < OT; ++ot) {
        const bf16x4 A =
            *reinterpret_cast<const bf16x4*>(W3s + (16 * ot + r16) * kWStride + 16 * ht + 4 * qd);
#pragma unroll
        for (int g = 0; g < 4; ++g)
          acc3[g][ot] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, a2[g], acc3[g][ot], 0, 0, 0);
      }
    }
    // de-standardised outputs straight into the rows: P[pt][o] = y_o and
    // C[pt][o - M] = y_o / |s_pt| (the kept rows)
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int64_t pt = wbase + 16 * g + r16;
      if (pt < N) {
        const double inv = 1.0 / fabs(sw[16 * g + r16]);
#pragma unroll
        for (int ot = 0; ot < OT; ++ot)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int o = 16 * ot + 4 * qd + i;
            const float y = mys[o] + sys[o] * (acc3[g][ot][i] + b3s[o]);
            if (o < M) P[pt * M + o] = (double)y;
            else if (o < NO) Crows[pt * M + (o - M)] = (double)y * inv;
          }
      }
    }
    __syncthreads();  // the rows of the block's points are written

    // ---- check, one lane per point ----
    double vm[M], q[M];
    if (valid) {
      int c[D];
      coords<D>(j, logn, c);
#pragma unroll
      for (int a = 0; a < M; ++a) {
        vm[a] = v[neighbour_ct<D, W>(c, logn, a)] - s;
        q[a] = P[j * M + a] - Crows[j * M + a] * vm[a];
      }
    } else {
#pragma unroll
      for (int a = 0; a < M; ++a) {
        vm[a] = 0.0;
        q[a] = 0.0;
      }
    }
    // q^T K_s q, one pass per distinct shift of the wave: the wave copies the
    // packed K_s into its LDS area, then the lanes of that shift read it as
    // broadcasts
    double form = 0.0;
    bool todo = valid;
    unsigned long long pending = __ballot(todo);
    while (pending) {
      const int sid = __builtin_amdgcn_readlane(id, __builtin_ctzll(pending));
      const double2* Kg = reinterpret_cast<const double2*>(Kf + (int64_t)sid * F::KS);
      double2* Kw2 = reinterpret_cast<double2*>(Kw);
      constexpr int KV = (F::KS / 2 + 63) / 64;  // double2 per lane
      double2 kv[KV];
#pragma unroll
      for (int u = 0; u < KV; ++u)
        if (lane + 64 * u < F::KS / 2) kv[u] = Kg[lane + 64 * u];
#pragma unroll
      for (int u = 0; u < KV; ++u)
        if (lane + 64 * u < F::KS / 2) Kw2[lane + 64 * u] = kv[u];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (todo && id == sid) {
        double f = 0.0;
        int e = 0;
#pragma unroll
        for (int a = 0; a < M; ++a) {
          double rsum = 0.0;
#pragma unroll
          for (int b = a; b < M; ++b) rsum = fma(Kw[e++], q[b], rsum);
          f = fma(q[a], rsum, f);
        }
        form = f;
        todo = false;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      pending = __ballot(todo);
    }
    double qq = 0.0;
#pragma unroll
    for (int a = 0; a < M; ++a) qq = fma(q[a], q[a], qq);
    const bool ok = valid && isfinite(form) && (qq > 0.0) && (form <= 0.0);
    if (valid && !ok) {  // the exact rows alpha + C (v[mu_j] - s_j) and C
      const double2* act = actab + (int64_t)id * M;
#pragma unroll
      for (int a = 0; a < M; ++a) {
        const double2 ac = act[a];
        P[j * M + a] = exact_entry(ac.x, ac.y, vm[a]);
        Crows[j * M + a] = ac.y;
      }
    }
    if (valid) fallback[j] = ok ? 0 : 1;
    nf_local += __popcll(__ballot(valid && !ok));
    __syncthreads();  // sw and the rows are reused by the next chunk
  }
  if (lane == 0 && nf_local) atomicAdd(nfall, nf_local);
}

template <int D, int W>
hipError_t launch_fused_dw(const lsp_problem* p, const lsp::MlpView& mv, double thr,
                           double* rho_star, double* Kf, double* P, double* Crows,
                           int32_t* fallback, int* nfall) {
  using F = Fused<D, W>;
  hipLaunchKernelGGL((kform_kernel<D, W>), dim3(p->num_shifts), dim3(256), 0, p->stream,
                     p->ws.gtab, p->ws.gamtab, reinterpret_cast<const double2*>(p->ws.actab),
                     p->ws.nS, thr, rho_star, Kf, nfall);
  const size_t lds = F::bytes(p->num_shifts);
  static size_t attr_bytes = 0;
  if (attr_bytes < lds) {
    const hipError_t e =
        hipFuncSetAttribute(reinterpret_cast<const void*>(&learned_fused_kernel<D, W>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr_bytes = lds;
  }
  int cus = 0;
  hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device);
  if (e != hipSuccess) return e;
  const int64_t nchunks = (p->N + kPts - 1) / kPts;
  const int blocks = (int)std::min<int64_t>(nchunks, 2 * (int64_t)cus);
  int logn = 0;
  while ((1 << logn) < p->n) ++logn;
  NetPtrs net{mv.W1, mv.W2, mv.W3, mv.b1, mv.b2, mv.b3, mv.norm};
  hipLaunchKernelGGL((learned_fused_kernel<D, W>), dim3(blocks), dim3(kThreads), lds,
                     p->stream, p->v, logn, p->N, 1.0 / ((double)p->n * p->n), p->ws.S, p->ws.nS,
                     reinterpret_cast<const double2*>(p->ws.actab), Kf, net, (int)nchunks, P,
                     Crows, fallback, nfall);
  return hipGetLastError();
}

}  // namespace

namespace lsp {

bool learned_fused_supported(const lsp_problem* p, const MlpView& mv) {
  const int W = 2 * p->t + 1;
  const bool shape = (p->d == 2 && (W == 3 || W == 5)) || (p->d == 3 && W == 3);
  return shape && mv.n_hidden == kH;
}

size_t learned_kform_doubles(int d, int t) {
  const int W = 2 * t + 1;
  int M = 1;
  for (int i = 0; i < d; ++i) M *= W;
  const int MM = M * (M + 1) / 2;
  return (size_t)(MM + 15) / 16 * 16;
}

hipError_t launch_learned_fused(const lsp_problem* p, const MlpView& mv, double thr,
                                double* rho_star, double* Kf, double* P, double* Crows,
                                int32_t* fallback, int* nfall) {
  const int W = 2 * p->t + 1;
  if (p->d == 2 && W == 3)
    return launch_fused_dw<2, 3>(p, mv, thr, rho_star, Kf, P, Crows, fallback, nfall);
  if (p->d == 2 && W == 5)
    return launch_fused_dw<2, 5>(p, mv, thr, rho_star, Kf, P, Crows, fallback, nfall);
  if (p->d == 3 && W == 3)
    return launch_fused_dw<3, 3>(p, mv, thr, rho_star, Kf, P, Crows, fallback, nfall);
  return hipErrorInvalidValue;
}

}  // namespace lsp
