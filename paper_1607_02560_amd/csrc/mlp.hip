// Learned-stencil surrogate: a 2-hidden-layer SiLU network mapping the local
// potential patch of a grid point to its P and C rows, trained and evaluated
// with hand-written BF16 MFMA kernels (FP32 accumulation, FP32 master weights
// and Adam state), and the learned setup that checks every predicted row with
// the exact Gram matrices of eq. (A) and falls back to the exact row where the
// check fails. The surrogate is not part of the paper; its rows feed the same
// preconditioner P^-1 C of eq. (PC).
//
// Network (per point): x (n_in raw features) -> standardise -> z1 = W1 x + b1,
// a1 = silu(z1) -> z2 = W2 a1 + b2, a2 = silu(z2) -> y = W3 a2 + b3 ->
// de-standardise. Loss: mean squared error of y against standardised targets.
//
// Device layouts (row-major, padded so that every GEMM dimension is a
// multiple of 16; padded weights and biases stay zero because their
// gradients are zero):
//   W1 [H][Ip], b1 [H], W2 [H][H], b2 [H], W3 [Op][H], b3 [Op]
//   activations [rows][H] (FP32 pre-activations, BF16 post-activations),
//   inputs [rows][Ip] BF16, outputs [rows][Op] FP32.
#include <type_traits>

#include "setup_common.h"

#include <cstdio>
#include <cstring>

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef short s16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kT = 256;

// FP32 -> BF16 bits, round to nearest even (v_cvt_pk_bf16_f32)
__device__ __forceinline__ unsigned short to_bf16(float x) {
  return __builtin_bit_cast(unsigned short, (__bf16)x);
}

// logistic function with the hardware reciprocal (v_rcp_f32, about 1 ulp);
// exp(-z) = inf for very negative z gives 0
__device__ __forceinline__ float sigmoidf_(float z) {
  return __builtin_amdgcn_rcpf(1.0f + __expf(-z));
}

// C[m][n] = sum_k A(m,k) B(k,n) (+ bias[n]) (+ C[m][n] if accumulate), with
// A(m,k) = A[m sam + k sak], B(k,n) = B[k sbk + n sbn] in BF16 and C in FP32.
// M, N, K are multiples of 16. Four waves per block, one 16x16 tile each
// (2 x 2 tiles per block). k runs in blocks of 32 from the start of the
// block's range, one v_mfma_f32_16x16x32_bf16 each, with lane group q
// holding k = 4q .. 4q+3 and 16 + 4q .. 16 + 4q + 3 of the block (the
// placement the fused learned kernel uses for its tile pairs, so both sum in
// the same order); a last odd 16 of k takes one v_mfma_f32_16x16x16bf16.
// Operands of two k-blocks are loaded together.
// With gridDim.z > 1 block z sums k in [z kchunk, (z+1) kchunk) and writes
// its raw partial tile to C + z M ldc (split_reduce_kernel adds them).
// MFMA operand layout: lane l holds A[l%16][4(l/16)+i], B[4(l/16)+i][l%16]
// and D[4(l/16)+i][l%16], i = 0..3.
// AK1 / BK1: the operand is contiguous in k (sak = 1 / sbk = 1, rows 8-byte
// aligned), so the four k values a lane needs per 16 come in one 8-byte load
// instead of four 2-byte loads (the same values, the same sums).
// EPI (no k split): the elementwise step that follows the product, fused
// into its store, with the operations of the separate kernels it replaces:
//   kEpiSilu      C as usual, and Ab = bf16(silu(C)) (same ld);
//   kEpiSiluBack  the product is dA; C = dZ = dA silu'(Z) (Z the same
//                 shape, rows >= valid_rows zero) and Ab = bf16(dZ).
enum { kEpiNone = 0, kEpiSilu = 1, kEpiSiluBack = 2 };

template <bool AK1, bool BK1, int EPI>
__global__ __launch_bounds__(kT) void gemm_bf16_kernel(
    const unsigned short* __restrict__ A, int64_t sam, int64_t sak,
    const unsigned short* __restrict__ B, int64_t sbk, int64_t sbn, float* C, int64_t ldc, int M,
    int N, int K, const float* __restrict__ bias, int accumulate, int kchunk,
    unsigned short* __restrict__ Ab, const float* __restrict__ Zin, int valid_rows) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int m0 = (blockIdx.y * 2 + (wave >> 1)) * 16;
  const int n0 = (blockIdx.x * 2 + (wave & 1)) * 16;
  if (m0 >= M || n0 >= N) return;  // uniform over the wave; no barrier below
  const int r = lane & 15, kq = (lane >> 4) * 4;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  const unsigned short* ap = A + (int64_t)(m0 + r) * sam;
  const unsigned short* bp = B + (int64_t)(n0 + r) * sbn;
  const int kb = blockIdx.z * kchunk;
  const int ke = min(K, kb + kchunk);
  const bool split = gridDim.z > 1;
  if (split) {
    C += (int64_t)blockIdx.z * M * ldc;
    bias = nullptr;
    accumulate = 0;
  }
  // two 32-blocks of operands are loaded before their two MFMAs (one memory
  // round trip per 64 values of k); the MFMAs run in k order either way
  auto load8 = [&](const unsigned short* p, int64_t stride, int kbase, auto unit) {
    if constexpr (decltype(unit)::value) {
      const uint2 lo = *reinterpret_cast<const uint2*>(p + kbase + kq);
      const uint2 hi = *reinterpret_cast<const uint2*>(p + kbase + 16 + kq);
      return __builtin_bit_cast(bf16x8, make_uint4(lo.x, lo.y, hi.x, hi.y));
    } else {
      s16x8 v;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        v[i] = (short)p[(int64_t)(kbase + kq + i) * stride];
        v[4 + i] = (short)p[(int64_t)(kbase + 16 + kq + i) * stride];
      }
      return __builtin_bit_cast(bf16x8, v);
    }
  };
  auto load4 = [&](const unsigned short* p, int64_t stride, int kbase, auto unit) {
    if constexpr (decltype(unit)::value) {
      return __builtin_bit_cast(bf16x4, *reinterpret_cast<const uint2*>(p + kbase + kq));
    } else {
      bf16x4 v;
#pragma unroll
      for (int i = 0; i < 4; ++i) v[i] = (short)p[(int64_t)(kbase + kq + i) * stride];
      return v;
    }
  };
  const std::integral_constant<bool, AK1> ua{};
  const std::integral_constant<bool, BK1> ub{};
  int k0 = kb;
  for (; k0 + 64 <= ke; k0 += 64) {
    const bf16x8 a0 = load8(ap, sak, k0, ua), b0 = load8(bp, sbk, k0, ub);
    const bf16x8 a1 = load8(ap, sak, k0 + 32, ua), b1 = load8(bp, sbk, k0 + 32, ub);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b0, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1, acc, 0, 0, 0);
  }
  if (k0 + 32 <= ke) {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(load8(ap, sak, k0, ua), load8(bp, sbk, k0, ub),
                                                  acc, 0, 0, 0);
    k0 += 32;
  }
  if (k0 < ke) {  // the last 16 values of k
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(load4(ap, sak, k0, ua), load4(bp, sbk, k0, ub),
                                                    acc, 0, 0, 0);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int row = m0 + kq + i, col = n0 + r;
    float val = acc[i];
    if (bias) val += bias[col];
    const int64_t at = (int64_t)row * ldc + col;
    float* cp = C + at;
    if (accumulate) val += *cp;
    if constexpr (EPI == kEpiSiluBack) {
      float gz = 0.f;
      if (row < valid_rows) {
        const float z = Zin[at];
        const float sg = sigmoidf_(z);
        gz = val * (sg * (1.f + z * (1.f - sg)));
      }
      *cp = gz;
      Ab[at] = to_bf16(gz);
    } else {
      *cp = val;
      if constexpr (EPI == kEpiSilu) Ab[at] = to_bf16(val * sigmoidf_(val));
    }
  }
}

// The same product for operands that are strided in k and contiguous in m
// and n (sam = 1, sbn = 1: the weight gradients, which reduce over the batch
// rows): per 32 values of k the block copies its 32 x 32 tiles of A and B
// into LDS with 16-byte loads (8 values of m or n for one k per thread) and
// stores them transposed, so that every lane reads its MFMA operands as two
// 8-byte LDS reads; k beyond the block's range is read as zero, so a last 16
// of k takes the 32-wide product too. Rows or columns past M or N load zeros
// and are not stored. Output as gemm_bf16_kernel (split in k: raw partials).
constexpr int kLdsK = 32 + 8;  // LDS row of one m (or n): 32 values of k, padded

__global__ __launch_bounds__(kT) void gemm_bf16_kt_kernel(
    const unsigned short* __restrict__ A, int64_t sak, const unsigned short* __restrict__ B,
    int64_t sbk, float* C, int64_t ldc, int M, int N, int K, int kchunk) {
  __shared__ __align__(16) unsigned short sA[32 * kLdsK];
  __shared__ __align__(16) unsigned short sB[32 * kLdsK];
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int mb = blockIdx.y * 32, nb = blockIdx.x * 32;
  const int r = lane & 15, kq = (lane >> 4) * 4;
  const int mw = (wave >> 1) * 16, nw = (wave & 1) * 16;  // the wave's tile in the block
  const int kb = blockIdx.z * kchunk;
  const int ke = min(K, kb + kchunk);
  if (gridDim.z > 1) C += (int64_t)blockIdx.z * M * ldc;
  // copy roles: threads 0..127 take A, 128..255 take B; one k and 8 of m (n)
  const bool isA = tid < 128;
  const int t = tid & 127;
  const int kk = t >> 2, seg = (t & 3) * 8;
  const int lim = isA ? M - mb : N - nb;
  const unsigned short* src = isA ? A + mb + seg : B + nb + seg;
  const int64_t sk = isA ? sak : sbk;
  unsigned short* dst = (isA ? sA : sB) + seg * kLdsK + kk;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = kb; k0 < ke; k0 += 32) {
    uint4 v = make_uint4(0u, 0u, 0u, 0u);
    if (k0 + kk < ke && seg < lim) v = *reinterpret_cast<const uint4*>(src + (int64_t)(k0 + kk) * sk);
    const unsigned int w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      dst[(2 * j) * kLdsK] = (unsigned short)(w[j] & 0xffffu);
      dst[(2 * j + 1) * kLdsK] = (unsigned short)(w[j] >> 16);
    }
    __syncthreads();
    const unsigned short* pa = sA + (mw + r) * kLdsK + kq;
    const unsigned short* pb = sB + (nw + r) * kLdsK + kq;
    const uint2 a0 = *reinterpret_cast<const uint2*>(pa), a1 = *reinterpret_cast<const uint2*>(pa + 16);
    const uint2 b0 = *reinterpret_cast<const uint2*>(pb), b1 = *reinterpret_cast<const uint2*>(pb + 16);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
        __builtin_bit_cast(bf16x8, make_uint4(a0.x, a0.y, a1.x, a1.y)),
        __builtin_bit_cast(bf16x8, make_uint4(b0.x, b0.y, b1.x, b1.y)), acc, 0, 0, 0);
    __syncthreads();
  }
  const int col = nb + nw + r;
  if (col >= N) return;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int row = mb + mw + kq + i;
    if (row < M) C[(int64_t)row * ldc + col] = acc[i];
  }
}

// C[m][n] = sum over z of part[z][m][n] (fixed order) (+ bias[n]) (+ C[m][n])
__global__ void split_reduce_kernel(const float* __restrict__ part, int splits, int M, int N,
                                    float* C, int64_t ldc, const float* __restrict__ bias,
                                    int accumulate) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)M * N) return;
  const int m = (int)(e / N), n = (int)(e % N);
  float s = 0.f;
  int z = 0;
  for (; z + 8 <= splits; z += 8) {  // eight loads in flight, added in order
    float x[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) x[u] = part[(int64_t)(z + u) * M * N + e];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += x[u];
  }
  for (; z < splits; ++z) s += part[(int64_t)z * M * N + e];
  if (bias) s += bias[n];
  float* cp = C + (int64_t)m * ldc + n;
  if (accumulate) s += *cp;
  *cp = s;
}

// Xb[r][c] = bf16((X[r][c] - mu[c]) * (1 / sd[c])) for r < rows, c < cols; 0 in
// the padding (rows .. rows_pad, cols .. ld).
__global__ void standardise_kernel(const float* __restrict__ X, int rows, int rows_pad, int cols,
                                   int ld, const float* __restrict__ mu,
                                   const float* __restrict__ sd, unsigned short* Xb) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)rows_pad * ld) return;
  const int r = (int)(e / ld), c = (int)(e % ld);
  float v = 0.f;
  if (r < rows && c < cols) v = (X[(int64_t)r * cols + c] - mu[c]) * (1.0f / sd[c]);
  Xb[e] = to_bf16(v);
}

// R = Y - (T - mu)/sd on the valid block [rows][cols] of Y [rows_pad][ld];
// dY = scale R (FP32 and BF16; zero in the padding); per-block sums of R^2.
__global__ void mse_grad_kernel(const float* __restrict__ Y, const float* __restrict__ T,
                                int rows, int rows_pad, int cols, int ld,
                                const float* __restrict__ mu, const float* __restrict__ sd,
                                float scale, float* dY, unsigned short* dYb, double* loss_part) {
  __shared__ double red[kT];
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double r2 = 0.0;
  if (e < (int64_t)rows_pad * ld) {
    const int r = (int)(e / ld), c = (int)(e % ld);
    float g = 0.f;
    if (r < rows && c < cols) {
      const float res = Y[e] - (T[(int64_t)r * cols + c] - mu[c]) / sd[c];
      r2 = (double)res * res;
      g = scale * res;
    }
    dY[e] = g;
    dYb[e] = to_bf16(g);
  }
  red[threadIdx.x] = r2;
  __syncthreads();
  for (int o = kT / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss_part[blockIdx.x] = red[0];
}

// Column sums out[c] = sum over rows of D[r][c] in two fixed-order stages.
// Stage 1: block (cb, rb) sums columns 64 cb .. 64 cb + 63 over the rows of
// row block rb (kColRows rows): thread (g, c) takes rows g, g + 4, ... with
// eight loads in flight (a wave reads 64 consecutive columns of one row), and
// the four row groups meet in LDS; part[rb][c] holds the block's sums.
constexpr int kColRows = 128;

__global__ __launch_bounds__(kT) void colsum_partial_kernel(const float* __restrict__ D, int rows,
                                                            int ld, int ncol, float* part) {
  __shared__ float red[kT];
  const int c = blockIdx.x * 64 + (threadIdx.x & 63);
  const int g = threadIdx.x >> 6;
  const int r0 = blockIdx.y * kColRows;
  const int r1 = min(rows, r0 + kColRows);
  float s = 0.f;
  if (c < ncol) {
    int r = r0 + g;
    for (; r + 28 < r1; r += 32) {
      float x[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) x[u] = D[(int64_t)(r + 4 * u) * ld + c];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += x[u];
    }
    for (; r < r1; r += 4) s += D[(int64_t)r * ld + c];
  }
  red[threadIdx.x] = s;
  __syncthreads();
  if (g == 0 && c < ncol)
    part[(int64_t)blockIdx.y * ncol + c] =
        ((red[threadIdx.x] + red[threadIdx.x + 64]) + red[threadIdx.x + 128]) +
        red[threadIdx.x + 192];
}

// Stage 2: out[c] = sum over row blocks of part[rb][c], in row-block order
// (eight loads in flight, added in order)
__global__ void colsum_final_kernel(const float* __restrict__ part, int nrb, int ncol,
                                    float* out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncol) return;
  float s = 0.f;
  int rb = 0;
  for (; rb + 8 <= nrb; rb += 8) {
    float x[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) x[u] = part[(int64_t)(rb + u) * ncol + c];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += x[u];
  }
  for (; rb < nrb; ++rb) s += part[(int64_t)rb * ncol + c];
  out[c] = s;
}

// Adam (Kingma and Ba) with bias correction on every parameter; the BF16
// copy of each weight is refreshed from the updated FP32 value.
__global__ void adam_kernel(float* p, const float* __restrict__ g, float* m, float* v, int count,
                            float lr, float b1, float b2, float eps, float c1, float c2,
                            unsigned short* pb) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  const float gi = g[e];
  const float mi = b1 * m[e] + (1.f - b1) * gi;
  const float vi = b2 * v[e] + (1.f - b2) * gi * gi;
  m[e] = mi;
  v[e] = vi;
  const float mh = mi / c1, vh = vi / c2;
  const float pn = p[e] - lr * mh / (sqrtf(vh) + eps);
  p[e] = pn;
  pb[e] = to_bf16(pn);
}

__global__ void to_bf16_kernel(const float* __restrict__ x, int count, unsigned short* y) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) y[e] = to_bf16(x[e]);
}

// per-column mean and deviation of X [rows][cols] (FP64 sums, fixed order)
__global__ void moments_kernel(const float* __restrict__ X, int rows, int cols, float* mu,
                               float* sd) {
  __shared__ double s1[kT], s2[kT];
  const int c = blockIdx.x;
  double a = 0.0, b = 0.0;
  for (int r = threadIdx.x; r < rows; r += kT) {
    const double x = X[(int64_t)r * cols + c];
    a += x;
    b += x * x;
  }
  s1[threadIdx.x] = a;
  s2[threadIdx.x] = b;
  __syncthreads();
  for (int o = kT / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      s1[threadIdx.x] += s1[threadIdx.x + o];
      s2[threadIdx.x] += s2[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double mean = s1[0] / rows;
    const double var = s2[0] / rows - mean * mean;
    mu[c] = (float)mean;
    sd[c] = (var > 0.0) ? (float)sqrt(var) : 1.0f;
  }
}

// Y [rows][cols] = mu + sd * Ys[r][c] (de-standardise the network outputs)
__global__ void destandardise_kernel(const float* __restrict__ Ys, int rows, int cols, int ld,
                                     const float* __restrict__ mu, const float* __restrict__ sd,
                                     float* Y) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)rows * cols) return;
  const int r = (int)(e / cols), c = (int)(e % cols);
  Y[e] = mu[c] + sd[c] * Ys[(int64_t)r * ld + c];
}

}  // namespace

// ----------------------------------------------------------------------------
// The network object
// ----------------------------------------------------------------------------
struct lsp_mlp {
  int n_in = 0, n_hidden = 0, n_out = 0;
  int Ip = 0, Op = 0;  // padded input and output widths
  int bmax = 0;        // rows per batch (multiple of 16)
  hipStream_t stream = nullptr;
  size_t nparam = 0;   // padded parameter count
  size_t off_W1 = 0, off_b1 = 0, off_W2 = 0, off_b2 = 0, off_W3 = 0, off_b3 = 0;
  float* param = nullptr;  // FP32 master (padded layout)
  float* grad = nullptr;
  float* adam_m = nullptr;
  float* adam_v = nullptr;
  unsigned short* pbf = nullptr;  // BF16 copy of param
  int adam_t = 0;
  float* norm = nullptr;  // mu_x [n_in], sd_x [n_in], mu_y [n_out], sd_y [n_out]
  // activations for bmax rows
  unsigned short* Xb = nullptr;
  float* Z1 = nullptr;
  float* Z2 = nullptr;
  unsigned short* A1b = nullptr;
  unsigned short* A2b = nullptr;
  float* Y = nullptr;
  float* dY = nullptr;
  unsigned short* dYb = nullptr;
  float* dA = nullptr;
  float* dZ = nullptr;
  unsigned short* dZb = nullptr;
  double* loss_part = nullptr;
  double* loss_host = nullptr;  // pinned
  float* gsplit = nullptr;      // k-split partial tiles of the weight gradients
  size_t gsplit_cap = 0;
  float* colpart = nullptr;     // column-sum partials of the bias gradients
};

namespace {

template <typename T>
int dalloc_(T** p, size_t n) {
  if (hipMalloc((void**)p, sizeof(T) * (n ? n : 1)) != hipSuccess)
    return lsp::set_error(LSP_ENOMEM, "device allocation for the surrogate failed");
  return LSP_OK;
}

template <typename T>
void dfree_(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

inline int round16(int x) { return (x + 15) / 16 * 16; }

inline unsigned blocks_for(int64_t n, int t = kT) { return (unsigned)((n + t - 1) / t); }

// One GEMM; reductions long against the number of output tiles (weight
// gradients over the batch rows) are split over k into partial tiles in
// split_buf (split_cap floats) and summed by a second kernel in a fixed order.
using GemmKernel = void (*)(const unsigned short*, int64_t, int64_t, const unsigned short*,
                           int64_t, int64_t, float*, int64_t, int, int, int, const float*, int, int,
                           unsigned short*, const float*, int);

template <int EPI>
GemmKernel gemm_kernel_for(bool ak1, bool bk1) {
  return ak1 ? (bk1 ? gemm_bf16_kernel<true, true, EPI> : gemm_bf16_kernel<true, false, EPI>)
             : (bk1 ? gemm_bf16_kernel<false, true, EPI> : gemm_bf16_kernel<false, false, EPI>);
}

// epi: the elementwise step fused into the store (gemm_bf16_kernel), with its
// BF16 output Ab, and for kEpiSiluBack the pre-activations Zin and the valid
// rows; an epilogue is only taken without a k split, bias or accumulation
// of kEpiSiluBack
hipError_t gemm(hipStream_t s, const unsigned short* A, int64_t sam, int64_t sak,
                const unsigned short* B, int64_t sbk, int64_t sbn, float* C, int64_t ldc, int M,
                int N, int K, const float* bias, bool accumulate, float* split_buf = nullptr,
                size_t split_cap = 0, int epi = kEpiNone, unsigned short* Ab = nullptr,
                const float* Zin = nullptr, int valid_rows = 0) {
  dim3 grid((N + 31) / 32, (M + 31) / 32);
  // operands contiguous in k with 8-byte aligned rows take the vector loads
  const bool ak1 = sak == 1 && sam % 4 == 0 && ((uintptr_t)A & 7) == 0;
  const bool bk1 = sbk == 1 && sbn % 4 == 0 && ((uintptr_t)B & 7) == 0;
  int splits = 1;
  if (split_buf && K >= 1024 && (int)(grid.x * grid.y) < 128) {
    splits = std::min(64, K / 256);
    while (splits > 1 && (size_t)splits * M * N > split_cap) splits /= 2;
  }
  if (epi != kEpiNone &&
      (splits > 1 || !Ab || (epi == kEpiSiluBack && (!Zin || bias || accumulate))))
    return hipErrorInvalidValue;
  // both operands strided in k, contiguous in m and n, 16-byte aligned rows:
  // the LDS-transposing kernel (no bias, no accumulation, no epilogue)
  const bool kt = !ak1 && !bk1 && sam == 1 && sbn == 1 && sak % 8 == 0 && sbk % 8 == 0 &&
                  ((uintptr_t)A & 15) == 0 && ((uintptr_t)B & 15) == 0 && !bias && !accumulate &&
                  epi == kEpiNone;
  const GemmKernel kern = epi == kEpiSilu       ? gemm_kernel_for<kEpiSilu>(ak1, bk1)
                          : epi == kEpiSiluBack ? gemm_kernel_for<kEpiSiluBack>(ak1, bk1)
                                                : gemm_kernel_for<kEpiNone>(ak1, bk1);
  if (splits <= 1) {
    if (kt)
      hipLaunchKernelGGL(gemm_bf16_kt_kernel, grid, dim3(kT), 0, s, A, sak, B, sbk, C, ldc, M, N,
                         K, K);
    else
      hipLaunchKernelGGL(kern, grid, dim3(kT), 0, s, A, sam, sak, B, sbk, sbn, C, ldc, M, N, K,
                         bias, accumulate ? 1 : 0, K, Ab, Zin, valid_rows);
    return hipGetLastError();
  }
  // whole 32-blocks per split (the k placement starts at each split's start)
  const int kchunk = ((K + splits - 1) / splits + 31) / 32 * 32;
  splits = (K + kchunk - 1) / kchunk;
  grid.z = splits;
  if (kt)
    hipLaunchKernelGGL(gemm_bf16_kt_kernel, grid, dim3(kT), 0, s, A, sak, B, sbk, split_buf,
                       (int64_t)N, M, N, K, kchunk);
  else
    hipLaunchKernelGGL(kern, grid, dim3(kT), 0, s, A, sam, sak, B, sbk, sbn, split_buf,
                       (int64_t)N, M, N, K, nullptr, 0, kchunk, nullptr, nullptr, 0);
  hipLaunchKernelGGL(split_reduce_kernel, dim3((unsigned)(((int64_t)M * N + kT - 1) / kT)),
                     dim3(kT), 0, s, split_buf, splits, M, N, C, ldc, bias, accumulate ? 1 : 0);
  return hipGetLastError();
}

// out[c] = column sums of D [rows][ld] (ncol columns), two launches; part
// holds ceil(rows / kColRows) * ncol floats
hipError_t colsum(hipStream_t s, const float* D, int rows, int ld, int ncol, float* part,
                  float* out) {
  const int nrb = (rows + kColRows - 1) / kColRows;
  hipLaunchKernelGGL(colsum_partial_kernel, dim3((unsigned)((ncol + 63) / 64), (unsigned)nrb),
                     dim3(kT), 0, s, D, rows, ld, ncol, part);
  hipLaunchKernelGGL(colsum_final_kernel, dim3(blocks_for(ncol)), dim3(kT), 0, s, part, nrb,
                     ncol, out);
  return hipGetLastError();
}

// forward pass of rows_pad rows of raw inputs X (rows valid) on stream s;
// leaves Z1, A1b, Z2, A2b and the standardised outputs Y [rows_pad][Op]
hipError_t forward(lsp_mlp* q, const float* X, int rows, int rows_pad, hipStream_t s) {
  const int H = q->n_hidden;
  const float* mu_x = q->norm;
  const float* sd_x = q->norm + q->n_in;
  hipLaunchKernelGGL(standardise_kernel, dim3(blocks_for((int64_t)rows_pad * q->Ip)), dim3(kT), 0,
                     s, X, rows, rows_pad, q->n_in, q->Ip, mu_x, sd_x, q->Xb);
  const unsigned short* W1 = q->pbf + q->off_W1;
  const unsigned short* W2 = q->pbf + q->off_W2;
  const unsigned short* W3 = q->pbf + q->off_W3;
  hipError_t e;
  // z1 = W1 x + b1: A(b, i) = Xb[b Ip + i], B(i, h) = W1[h Ip + i]
  if ((e = gemm(s, q->Xb, q->Ip, 1, W1, 1, q->Ip, q->Z1, H, rows_pad, H, q->Ip,
                q->param + q->off_b1, false, nullptr, 0, kEpiSilu, q->A1b)))
    return e;
  // (a1 = bf16(silu(z1)) in the same launch)
  if ((e = gemm(s, q->A1b, H, 1, W2, 1, H, q->Z2, H, rows_pad, H, H, q->param + q->off_b2, false,
                nullptr, 0, kEpiSilu, q->A2b)))
    return e;
  if ((e = gemm(s, q->A2b, H, 1, W3, 1, H, q->Y, q->Op, rows_pad, q->Op, H, q->param + q->off_b3,
                false)))
    return e;
  return hipGetLastError();
}

// loss and gradients of one batch (grad buffer overwritten); loss sums to loss_part
hipError_t backward(lsp_mlp* q, const float* T, int rows, int rows_pad, int* nblk_loss) {
  const int H = q->n_hidden;
  hipStream_t s = q->stream;
  const float* mu_y = q->norm + 2 * q->n_in;
  const float* sd_y = mu_y + q->n_out;
  const float scale = 2.0f / ((float)rows * (float)q->n_out);
  const unsigned nb = blocks_for((int64_t)rows_pad * q->Op);
  *nblk_loss = (int)nb;
  hipLaunchKernelGGL(mse_grad_kernel, dim3(nb), dim3(kT), 0, s, q->Y, T, rows, rows_pad, q->n_out,
                     q->Op, mu_y, sd_y, scale, q->dY, q->dYb, q->loss_part);
  float* g = q->grad;
  const unsigned short* W2 = q->pbf + q->off_W2;
  const unsigned short* W3 = q->pbf + q->off_W3;
  hipError_t e;
  // gW3 [Op][H] = dY^T A2: A(o, b) = dYb[b Op + o], B(b, h) = A2b[b H + h]
  if ((e = gemm(s, q->dYb, 1, q->Op, q->A2b, H, 1, g + q->off_W3, H, q->Op, H, rows_pad, nullptr,
                false, q->gsplit, q->gsplit_cap)))
    return e;
  if ((e = colsum(s, q->dY, rows_pad, q->Op, q->Op, q->colpart, g + q->off_b3))) return e;
  // dA2 = dY W3: A(b, o) = dYb[b Op + o], B(o, h) = W3[o H + h]; the same
  // launch stores dZ2 = dA2 silu'(Z2) (FP32 in dZ, BF16 in dZb)
  if ((e = gemm(s, q->dYb, q->Op, 1, W3, H, 1, q->dZ, H, rows_pad, H, q->Op, nullptr, false,
                nullptr, 0, kEpiSiluBack, q->dZb, q->Z2, rows)))
    return e;
  // gW2 [H][H] = dZ2^T A1
  if ((e = gemm(s, q->dZb, 1, H, q->A1b, H, 1, g + q->off_W2, H, H, H, rows_pad, nullptr, false,
                q->gsplit, q->gsplit_cap)))
    return e;
  if ((e = colsum(s, q->dZ, rows_pad, H, H, q->colpart, g + q->off_b2))) return e;
  // dA1 = dZ2 W2: B(h2, h1) = W2[h2 H + h1]; the same launch stores
  // dZ1 = dA1 silu'(Z1), FP32 in dA and BF16 in A1b (a1 is not read again;
  // dZb is this product's operand)
  if ((e = gemm(s, q->dZb, H, 1, W2, H, 1, q->dA, H, rows_pad, H, H, nullptr, false, nullptr, 0,
                kEpiSiluBack, q->A1b, q->Z1, rows)))
    return e;
  // gW1 [H][Ip] = dZ1^T Xb
  if ((e = gemm(s, q->A1b, 1, H, q->Xb, q->Ip, 1, g + q->off_W1, q->Ip, H, q->Ip, rows_pad,
                nullptr, false, q->gsplit, q->gsplit_cap)))
    return e;
  if ((e = colsum(s, q->dA, rows_pad, H, H, q->colpart, g + q->off_b1))) return e;
  return hipGetLastError();
}

int check_rows(const lsp_mlp* q, int rows) {
  if (rows < 1 || rows > q->bmax)
    return lsp::set_error(LSP_EINVAL, "rows must be in 1.." + std::to_string(q->bmax));
  return LSP_OK;
}

double sum_loss(lsp_mlp* q, int nblk, int rows) {
  (void)hipMemcpyAsync(q->loss_host, q->loss_part, sizeof(double) * nblk, hipMemcpyDeviceToHost,
                       q->stream);
  (void)hipStreamSynchronize(q->stream);
  double s = 0.0;
  for (int i = 0; i < nblk; ++i) s += q->loss_host[i];
  return s / ((double)rows * q->n_out);
}

// host FP32 parameters in the unpadded order W1, b1, W2, b2, W3, b3 <-> padded device layout
void pad_params(const lsp_mlp* q, const float* in, std::vector<float>& out) {
  const int I = q->n_in, H = q->n_hidden, O = q->n_out;
  out.assign(q->nparam, 0.f);
  size_t k = 0;
  for (int h = 0; h < H; ++h)
    for (int i = 0; i < I; ++i) out[q->off_W1 + (size_t)h * q->Ip + i] = in[k++];
  for (int h = 0; h < H; ++h) out[q->off_b1 + h] = in[k++];
  for (int h = 0; h < H; ++h)
    for (int i = 0; i < H; ++i) out[q->off_W2 + (size_t)h * H + i] = in[k++];
  for (int h = 0; h < H; ++h) out[q->off_b2 + h] = in[k++];
  for (int o = 0; o < O; ++o)
    for (int h = 0; h < H; ++h) out[q->off_W3 + (size_t)o * H + h] = in[k++];
  for (int o = 0; o < O; ++o) out[q->off_b3 + o] = in[k++];
}

void unpad_params(const lsp_mlp* q, const std::vector<float>& in, float* out) {
  const int I = q->n_in, H = q->n_hidden, O = q->n_out;
  size_t k = 0;
  for (int h = 0; h < H; ++h)
    for (int i = 0; i < I; ++i) out[k++] = in[q->off_W1 + (size_t)h * q->Ip + i];
  for (int h = 0; h < H; ++h) out[k++] = in[q->off_b1 + h];
  for (int h = 0; h < H; ++h)
    for (int i = 0; i < H; ++i) out[k++] = in[q->off_W2 + (size_t)h * H + i];
  for (int h = 0; h < H; ++h) out[k++] = in[q->off_b2 + h];
  for (int o = 0; o < O; ++o)
    for (int h = 0; h < H; ++h) out[k++] = in[q->off_W3 + (size_t)o * H + h];
  for (int o = 0; o < O; ++o) out[k++] = in[q->off_b3 + o];
}

}  // namespace

namespace lsp {

hipError_t mlp_forward_raw(lsp_mlp* q, const float* X, int rows, float* Y, hipStream_t s) {
  const int rp = round16(rows);
  hipError_t e = forward(q, X, rows, rp, s);
  if (e != hipSuccess) return e;
  const float* mu_y = q->norm + 2 * q->n_in;
  hipLaunchKernelGGL(destandardise_kernel, dim3(blocks_for((int64_t)rows * q->n_out)), dim3(kT), 0,
                     s, q->Y, rows, q->n_out, q->Op, mu_y, mu_y + q->n_out, Y);
  return hipGetLastError();
}

hipStream_t mlp_stream(const lsp_mlp* q) { return q->stream; }

MlpView mlp_view(const lsp_mlp* q) {
  return MlpView{q->n_in,           q->n_hidden,           q->n_out,
                 q->pbf + q->off_W1, q->pbf + q->off_W2,     q->pbf + q->off_W3,
                 q->param + q->off_b1, q->param + q->off_b2, q->param + q->off_b3,
                 q->norm};
}

int mlp_batch_rows(const lsp_mlp* q) { return q->bmax; }
int mlp_inputs(const lsp_mlp* q) { return q->n_in; }
int mlp_outputs(const lsp_mlp* q) { return q->n_out; }

}  // namespace lsp

// ----------------------------------------------------------------------------
// C ABI
// ----------------------------------------------------------------------------
extern "C" {

int lsp_mlp_create(int n_in, int n_hidden, int n_out, int batch_rows, void* stream,
                   lsp_mlp** out) {
  if (!out) return lsp::set_error(LSP_EINVAL, "out is NULL");
  *out = nullptr;
  if (n_in < 1 || n_hidden < 16 || n_hidden % 16 || n_out < 1 || batch_rows < 16)
    return lsp::set_error(LSP_EINVAL, "sizes: n_in, n_out >= 1, n_hidden a multiple of 16, "
                                      "batch_rows >= 16");
  lsp_mlp* q = new lsp_mlp();
  q->n_in = n_in;
  q->n_hidden = n_hidden;
  q->n_out = n_out;
  q->Ip = round16(n_in);
  q->Op = round16(n_out);
  q->bmax = round16(batch_rows);
  q->stream = static_cast<hipStream_t>(stream);
  const int H = n_hidden;
  size_t o = 0;
  q->off_W1 = o; o += (size_t)H * q->Ip;
  q->off_b1 = o; o += H;
  q->off_W2 = o; o += (size_t)H * H;
  q->off_b2 = o; o += H;
  q->off_W3 = o; o += (size_t)q->Op * H;
  q->off_b3 = o; o += q->Op;
  q->nparam = o;
  q->gsplit_cap = (size_t)64 * H * std::max(H, std::max(q->Ip, q->Op));
  const size_t B = q->bmax;
  int rc = LSP_OK;
  if ((rc = dalloc_(&q->param, o)) || (rc = dalloc_(&q->grad, o)) ||
      (rc = dalloc_(&q->adam_m, o)) || (rc = dalloc_(&q->adam_v, o)) ||
      (rc = dalloc_(&q->pbf, o)) || (rc = dalloc_(&q->norm, 2 * (size_t)(n_in + n_out))) ||
      (rc = dalloc_(&q->Xb, B * q->Ip)) || (rc = dalloc_(&q->Z1, B * H)) ||
      (rc = dalloc_(&q->Z2, B * H)) || (rc = dalloc_(&q->A1b, B * H)) ||
      (rc = dalloc_(&q->A2b, B * H)) || (rc = dalloc_(&q->Y, B * q->Op)) ||
      (rc = dalloc_(&q->dY, B * q->Op)) || (rc = dalloc_(&q->dYb, B * q->Op)) ||
      (rc = dalloc_(&q->dA, B * H)) || (rc = dalloc_(&q->dZ, B * H)) ||
      (rc = dalloc_(&q->dZb, B * H)) ||
      (rc = dalloc_(&q->loss_part, B * q->Op / kT + 1)) ||
      (rc = dalloc_(&q->gsplit, (size_t)64 * H * std::max(H, std::max(q->Ip, q->Op)))) ||
      (rc = dalloc_(&q->colpart,
                    (B + kColRows - 1) / kColRows * (size_t)std::max(H, q->Op)))) {
    lsp_mlp_destroy(q);
    return rc;
  }
  if (hipHostMalloc((void**)&q->loss_host, sizeof(double) * (B * q->Op / kT + 1)) != hipSuccess) {
    lsp_mlp_destroy(q);
    return lsp::set_error(LSP_ENOMEM, "pinned host allocation failed");
  }
  (void)hipMemsetAsync(q->param, 0, sizeof(float) * o, q->stream);
  (void)hipMemsetAsync(q->adam_m, 0, sizeof(float) * o, q->stream);
  (void)hipMemsetAsync(q->adam_v, 0, sizeof(float) * o, q->stream);
  (void)hipMemsetAsync(q->pbf, 0, sizeof(unsigned short) * o, q->stream);
  std::vector<float> nrm(2 * (size_t)(n_in + n_out), 0.f);
  for (int i = 0; i < n_in; ++i) nrm[n_in + i] = 1.f;
  for (int i = 0; i < n_out; ++i) nrm[2 * n_in + n_out + i] = 1.f;
  if (hipMemcpy(q->norm, nrm.data(), sizeof(float) * nrm.size(), hipMemcpyHostToDevice) !=
      hipSuccess) {
    lsp_mlp_destroy(q);
    return lsp::set_error(LSP_EHIP, "upload of the standardisation failed");
  }
  *out = q;
  return LSP_OK;
}

void lsp_mlp_destroy(lsp_mlp* q) {
  if (!q) return;
  (void)hipStreamSynchronize(q->stream);
  dfree_(q->param); dfree_(q->grad); dfree_(q->adam_m); dfree_(q->adam_v); dfree_(q->pbf);
  dfree_(q->norm); dfree_(q->Xb); dfree_(q->Z1); dfree_(q->Z2); dfree_(q->A1b); dfree_(q->A2b);
  dfree_(q->Y); dfree_(q->dY); dfree_(q->dYb); dfree_(q->dA); dfree_(q->dZ); dfree_(q->dZb);
  dfree_(q->loss_part);
  dfree_(q->gsplit);
  dfree_(q->colpart);
  if (q->loss_host) (void)hipHostFree(q->loss_host);
  delete q;
}

int lsp_mlp_num_params(const lsp_mlp* q) {
  if (!q) return 0;
  return q->n_in * q->n_hidden + q->n_hidden + q->n_hidden * q->n_hidden + q->n_hidden +
         q->n_out * q->n_hidden + q->n_out;
}

int lsp_mlp_set_params(lsp_mlp* q, const float* params_host) {
  if (!q || !params_host) return lsp::set_error(LSP_EINVAL, "NULL argument");
  std::vector<float> pad;
  pad_params(q, params_host, pad);
  if (hipMemcpy(q->param, pad.data(), sizeof(float) * pad.size(), hipMemcpyHostToDevice) !=
      hipSuccess)
    return lsp::set_error(LSP_EHIP, "parameter upload failed");
  hipLaunchKernelGGL(to_bf16_kernel, dim3(blocks_for((int64_t)q->nparam)), dim3(kT), 0, q->stream,
                     q->param, (int)q->nparam, q->pbf);
  (void)hipMemsetAsync(q->adam_m, 0, sizeof(float) * q->nparam, q->stream);
  (void)hipMemsetAsync(q->adam_v, 0, sizeof(float) * q->nparam, q->stream);
  q->adam_t = 0;
  return lsp::hip_check(hipStreamSynchronize(q->stream), "parameter upload");
}

int lsp_mlp_get_params(lsp_mlp* q, float* params_host) {
  if (!q || !params_host) return lsp::set_error(LSP_EINVAL, "NULL argument");
  std::vector<float> pad(q->nparam);
  (void)hipStreamSynchronize(q->stream);
  if (hipMemcpy(pad.data(), q->param, sizeof(float) * pad.size(), hipMemcpyDeviceToHost) !=
      hipSuccess)
    return lsp::set_error(LSP_EHIP, "parameter download failed");
  unpad_params(q, pad, params_host);
  return LSP_OK;
}

int lsp_mlp_set_normalisation(lsp_mlp* q, const float* norm_host) {
  if (!q || !norm_host) return lsp::set_error(LSP_EINVAL, "NULL argument");
  const size_t n = 2 * (size_t)(q->n_in + q->n_out);
  for (size_t i = 0; i < (size_t)q->n_in; ++i)
    if (!(norm_host[q->n_in + i] > 0.f)) return lsp::set_error(LSP_EINVAL, "deviation <= 0");
  for (size_t i = 0; i < (size_t)q->n_out; ++i)
    if (!(norm_host[2 * q->n_in + q->n_out + i] > 0.f))
      return lsp::set_error(LSP_EINVAL, "deviation <= 0");
  if (hipMemcpy(q->norm, norm_host, sizeof(float) * n, hipMemcpyHostToDevice) != hipSuccess)
    return lsp::set_error(LSP_EHIP, "standardisation upload failed");
  return LSP_OK;
}

int lsp_mlp_get_normalisation(lsp_mlp* q, float* norm_host) {
  if (!q || !norm_host) return lsp::set_error(LSP_EINVAL, "NULL argument");
  (void)hipStreamSynchronize(q->stream);
  if (hipMemcpy(norm_host, q->norm, sizeof(float) * 2 * (q->n_in + q->n_out),
                hipMemcpyDeviceToHost) != hipSuccess)
    return lsp::set_error(LSP_EHIP, "standardisation download failed");
  return LSP_OK;
}

int lsp_mlp_fit_normalisation(lsp_mlp* q, const float* X_dev, const float* T_dev, int rows) {
  if (!q || !X_dev || !T_dev || rows < 2) return lsp::set_error(LSP_EINVAL, "bad argument");
  hipLaunchKernelGGL(moments_kernel, dim3(q->n_in), dim3(kT), 0, q->stream, X_dev, rows, q->n_in,
                     q->norm, q->norm + q->n_in);
  hipLaunchKernelGGL(moments_kernel, dim3(q->n_out), dim3(kT), 0, q->stream, T_dev, rows,
                     q->n_out, q->norm + 2 * q->n_in, q->norm + 2 * q->n_in + q->n_out);
  return lsp::hip_check(hipGetLastError(), "normalisation fit");
}

int lsp_mlp_forward(lsp_mlp* q, const float* X_dev, int rows, float* Y_dev) {
  if (!q || !X_dev || !Y_dev) return lsp::set_error(LSP_EINVAL, "NULL argument");
  int rc = check_rows(q, rows);
  if (rc) return rc;
  return lsp::hip_check(lsp::mlp_forward_raw(q, X_dev, rows, Y_dev, q->stream),
                        "surrogate forward");
}

int lsp_mlp_loss_grad(lsp_mlp* q, const float* X_dev, const float* T_dev, int rows,
                      float* grad_host, double* loss_host) {
  if (!q || !X_dev || !T_dev) return lsp::set_error(LSP_EINVAL, "NULL argument");
  int rc = check_rows(q, rows);
  if (rc) return rc;
  const int rp = round16(rows);
  hipError_t e = forward(q, X_dev, rows, rp, q->stream);
  int nblk = 0;
  if (e == hipSuccess) e = backward(q, T_dev, rows, rp, &nblk);
  if (e != hipSuccess) return lsp::hip_check(e, "surrogate gradient");
  const double loss = sum_loss(q, nblk, rows);
  if (loss_host) *loss_host = loss;
  if (grad_host) {
    std::vector<float> pad(q->nparam);
    if (hipMemcpy(pad.data(), q->grad, sizeof(float) * pad.size(), hipMemcpyDeviceToHost) !=
        hipSuccess)
      return lsp::set_error(LSP_EHIP, "gradient download failed");
    unpad_params(q, pad, grad_host);
  }
  return LSP_OK;
}

int lsp_mlp_train_step(lsp_mlp* q, const float* X_dev, const float* T_dev, int rows, float lr,
                       double* loss_host) {
  if (!q || !X_dev || !T_dev) return lsp::set_error(LSP_EINVAL, "NULL argument");
  if (!(lr > 0.f)) return lsp::set_error(LSP_EINVAL, "lr must be > 0");
  int rc = check_rows(q, rows);
  if (rc) return rc;
  const int rp = round16(rows);
  hipError_t e = forward(q, X_dev, rows, rp, q->stream);
  int nblk = 0;
  if (e == hipSuccess) e = backward(q, T_dev, rows, rp, &nblk);
  if (e != hipSuccess) return lsp::hip_check(e, "surrogate training step");
  const float b1 = 0.9f, b2 = 0.999f;
  q->adam_t += 1;
  const float c1 = 1.f - powf(b1, (float)q->adam_t);
  const float c2 = 1.f - powf(b2, (float)q->adam_t);
  hipLaunchKernelGGL(adam_kernel, dim3(blocks_for((int64_t)q->nparam)), dim3(kT), 0, q->stream,
                     q->param, q->grad, q->adam_m, q->adam_v, (int)q->nparam, lr, b1, b2, 1e-8f,
                     c1, c2, q->pbf);
  if ((e = hipGetLastError()) != hipSuccess) return lsp::hip_check(e, "Adam step");
  if (loss_host) *loss_host = sum_loss(q, nblk, rows);
  return LSP_OK;
}

// ---- save / load: one flat little-endian file ----
// header (64 bytes): magic "LSPMLP01", version, n_in, n_hidden, n_out, Adam
// step count, parameter count, FNV-1a 64 checksum of the payload; payload
// (FP32): parameters (order of lsp_mlp_set_params), standardisation
// (mu_x, sd_x, mu_y, sd_y), Adam first and second moments (parameter order).
namespace {
struct MlpFileHeader {
  char magic[8];
  int32_t version, n_in, n_hidden, n_out, adam_t, reserved;
  uint64_t nparam, checksum;
  uint64_t pad[2];
};
static_assert(sizeof(MlpFileHeader) == 64, "file header layout");

uint64_t fnv1a(const void* data, size_t bytes, uint64_t h = 1469598103934665603ull) {
  const unsigned char* b = static_cast<const unsigned char*>(data);
  for (size_t i = 0; i < bytes; ++i) {
    h ^= b[i];
    h *= 1099511628211ull;
  }
  return h;
}
}  // namespace

int lsp_mlp_save(lsp_mlp* q, const char* path) {
  if (!q || !path) return lsp::set_error(LSP_EINVAL, "NULL argument");
  const size_t np = (size_t)lsp_mlp_num_params(q);
  const size_t nn = 2 * (size_t)(q->n_in + q->n_out);
  std::vector<float> payload(3 * np + nn);
  int rc = lsp_mlp_get_params(q, payload.data());
  if (rc) return rc;
  if ((rc = lsp_mlp_get_normalisation(q, payload.data() + np))) return rc;
  std::vector<float> pad(q->nparam);
  for (int k = 0; k < 2; ++k) {
    if (hipMemcpy(pad.data(), k == 0 ? q->adam_m : q->adam_v, sizeof(float) * q->nparam,
                  hipMemcpyDeviceToHost) != hipSuccess)
      return lsp::set_error(LSP_EHIP, "Adam state download failed");
    unpad_params(q, pad, payload.data() + np + nn + k * np);
  }
  MlpFileHeader h{};
  memcpy(h.magic, "LSPMLP01", 8);
  h.version = 1;
  h.n_in = q->n_in;
  h.n_hidden = q->n_hidden;
  h.n_out = q->n_out;
  h.adam_t = q->adam_t;
  h.nparam = np;
  h.checksum = fnv1a(payload.data(), sizeof(float) * payload.size());
  FILE* f = fopen(path, "wb");
  if (!f) return lsp::set_error(LSP_EINVAL, std::string("cannot open ") + path + " for writing");
  const bool ok = fwrite(&h, sizeof(h), 1, f) == 1 &&
                  fwrite(payload.data(), sizeof(float), payload.size(), f) == payload.size();
  if (fclose(f) != 0 || !ok) return lsp::set_error(LSP_EINVAL, std::string("write failed: ") + path);
  return LSP_OK;
}

int lsp_mlp_load(const char* path, int batch_rows, void* stream, lsp_mlp** out) {
  if (!path || !out) return lsp::set_error(LSP_EINVAL, "NULL argument");
  *out = nullptr;
  FILE* f = fopen(path, "rb");
  if (!f) return lsp::set_error(LSP_EINVAL, std::string("cannot open ") + path);
  MlpFileHeader h{};
  bool ok = fread(&h, sizeof(h), 1, f) == 1 && memcmp(h.magic, "LSPMLP01", 8) == 0 &&
            h.version == 1 && h.n_in >= 1 && h.n_out >= 1 && h.n_hidden >= 16 &&
            h.n_hidden % 16 == 0 && h.n_in <= 4096 && h.n_out <= 4096 && h.n_hidden <= 4096 &&
            h.adam_t >= 0;
  const uint64_t np = ok ? (uint64_t)h.n_hidden * (h.n_in + h.n_hidden + h.n_out + 2) + h.n_out : 0;
  ok = ok && h.nparam == np;
  std::vector<float> payload;
  if (ok) {
    payload.resize(3 * np + 2 * (size_t)(h.n_in + h.n_out));
    ok = fread(payload.data(), sizeof(float), payload.size(), f) == payload.size() &&
         fgetc(f) == EOF && fnv1a(payload.data(), sizeof(float) * payload.size()) == h.checksum;
  }
  fclose(f);
  if (!ok) return lsp::set_error(LSP_EINVAL, std::string("not a valid surrogate file: ") + path);
  lsp_mlp* q = nullptr;
  int rc = lsp_mlp_create(h.n_in, h.n_hidden, h.n_out, batch_rows, stream, &q);
  if (rc) return rc;
  const size_t nn = 2 * (size_t)(h.n_in + h.n_out);
  if ((rc = lsp_mlp_set_params(q, payload.data())) ||
      (rc = lsp_mlp_set_normalisation(q, payload.data() + np))) {
    lsp_mlp_destroy(q);
    return rc;
  }
  std::vector<float> pad;
  for (int k = 0; k < 2; ++k) {
    pad_params(q, payload.data() + np + nn + k * np, pad);
    if (hipMemcpy(k == 0 ? q->adam_m : q->adam_v, pad.data(), sizeof(float) * q->nparam,
                  hipMemcpyHostToDevice) != hipSuccess) {
      lsp_mlp_destroy(q);
      return lsp::set_error(LSP_EHIP, "Adam state upload failed");
    }
  }
  q->adam_t = h.adam_t;
  *out = q;
  return LSP_OK;
}

}  // extern "C"

// ----------------------------------------------------------------------------
// Rows of a problem: features, exact targets, learned rows with fallback
// ----------------------------------------------------------------------------
namespace {

using lsp::nearest_shift;
using lsp::Nbhd;
using lsp::Pow;

// flat index of the neighbour a of point j (periodic)
template <int D, int W>
__device__ __forceinline__ int64_t neighbour(int64_t j, int n, int a) {
  using Nb = Nbhd<D, W>;
  int64_t g = 0, rem = j, mul = 1;
  int c[D];
#pragma unroll
  for (int i = D - 1; i >= 0; --i) {
    c[i] = (int)(rem % n);
    rem /= n;
  }
#pragma unroll
  for (int i = 0; i < D; ++i) c[i] = (c[i] + Nb::comp(a, i) + n) & (n - 1);
#pragma unroll
  for (int i = D - 1; i >= 0; --i) {
    g += c[i] * mul;
    mul *= n;
  }
  return g;
}

// X[r] = (h^2 v_j, h^2 v[j + a] for a in mu_0^t, h^2 s_j), j = points[r] (or
// j0 + r), s_j the shift assigned to v_j (an index outside [0, N) gives a row
// of NaN and reads nothing)
template <int D, int W>
__global__ void features_kernel(const double* __restrict__ v, int n, int64_t N,
                                const double* __restrict__ S, const int* __restrict__ nS_ptr,
                                const int64_t* __restrict__ points, int64_t j0, int rows,
                                double h2, float* X) {
  constexpr int M = Pow<D, W>::v;
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  const int64_t j = points ? points[r] : j0 + r;
  float* x = X + (int64_t)r * (M + 2);
  if (j < 0 || j >= N) {
    for (int a = 0; a < M + 2; ++a) x[a] = __int_as_float(0x7fc00000);
    return;
  }
  x[0] = (float)(h2 * v[j]);
#pragma unroll
  for (int a = 0; a < M; ++a) x[1 + a] = (float)(h2 * v[neighbour<D, W>(j, n, a)]);
  x[M + 1] = (float)(h2 * S[nearest_shift(S, *nS_ptr, v[j])]);
}

// T[r] = (P[j, a] for a, C_{s_j}[a] |s_j| for a), j = points[r] (an index
// outside [0, N) gives a row of NaN and reads nothing)
template <int D, int W>
__global__ void targets_kernel(const double* __restrict__ P, const double* __restrict__ v,
                               int64_t N, const double* __restrict__ S,
                               const int* __restrict__ nS_ptr, const double* __restrict__ Ctab,
                               const int64_t* __restrict__ points, int rows, float* T) {
  constexpr int M = Pow<D, W>::v;
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  const int64_t j = points[r];
  float* t = T + (int64_t)r * 2 * M;
  if (j < 0 || j >= N) {
    for (int a = 0; a < 2 * M; ++a) t[a] = __int_as_float(0x7fc00000);
    return;
  }
  const int id = nearest_shift(S, *nS_ptr, v[j]);
  const double as = fabs(S[id]);
#pragma unroll
  for (int a = 0; a < M; ++a) {
    t[a] = (float)P[j * M + a];
    t[M + a] = (float)(Ctab[(int64_t)id * M + a] * as);
  }
}

// q^T A1 q, q^T M q = q^T A1 q - |G q|^2 and G q for a stencil q on mu_0^t,
// with G[a][b] = g[|a - b|] and A1[a][b] = gam[|a - b|] (eq. A; tables at the
// offsets [0, 2t]^d)
template <int D, int W>
__device__ __forceinline__ void gram_forms(const double* __restrict__ g,
                                           const double* __restrict__ gm, const double* q,
                                           double& qaq, double& qmq, double* gq) {
  using Nb = Nbhd<D, W>;
  constexpr int M = Pow<D, W>::v;
  double a1 = 0.0, gq2 = 0.0;
#pragma unroll
  for (int a = 0; a < M; ++a) {
    double u = 0.0, w = 0.0;
#pragma unroll
    for (int b = 0; b < M; ++b) {
      const int k = Nb::diff_index(a, b);
      u = fma(g[k], q[b], u);
      w = fma(gm[k], q[b], w);
    }
    gq[a] = u;
    gq2 = fma(u, u, gq2);
    a1 = fma(q[a], w, a1);
  }
  qaq = a1;
  qmq = a1 - gq2;
}

// an entry alpha + C (v - s) of an exact row, rounded exactly as the exact
// setup's assembly rounds it (product and sum rounded separately)
__device__ __forceinline__ double exact_entry(double alpha, double c, double v_minus_s) {
#pragma clang fp contract(off)
  return alpha + c * v_minus_s;
}

// Learned rows of points j0 .. j0+rows-1 from the de-standardised network
// outputs Y [rows][2m]: p = Y[:m], c = Y[m:] / |s_j|, stencil
// q = p - c (v[mu_j] - s_j) and rho = sqrt(q^T M q / q^T A1 q) (eq. A). A
// kept point takes the rows its stencil defines, C = (Q G)[j, mu_j] =
// G_mu,mu q and P = q + C (v[mu_j] - s_j) (Sec. 4.1, eq. PC). Rows with
// rho > rho*(s_j) + thr, where rho*(s_j) is the same quantity for the exact
// stencil of the shift (or with a non-finite value), take the exact row
// alpha + C (v[mu_j] - s_j) and C; fallback[j] records which.
template <int D, int W>
__global__ void learned_rows_kernel(const double* __restrict__ v, int n,
                                    const double* __restrict__ S, const int* __restrict__ nS_ptr,
                                    const double* __restrict__ gtab,
                                    const double* __restrict__ gamtab,
                                    const double2* __restrict__ actab,
                                    const double* __restrict__ rho_star,
                                    const float* __restrict__ Y, int64_t j0, int rows, double thr,
                                    double* P, double* Crows, int32_t* fallback, int* nfall) {
  constexpr int M = Pow<D, W>::v;
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  const int64_t j = j0 + r;
  const int id = nearest_shift(S, *nS_ptr, v[j]);
  const double s = S[id];
  const double inv_as = 1.0 / fabs(s);
  double vm[M], q[M], c[M];
#pragma unroll
  for (int a = 0; a < M; ++a) {
    vm[a] = v[neighbour<D, W>(j, n, a)] - s;
    c[a] = (double)Y[(int64_t)r * 2 * M + M + a] * inv_as;
    q[a] = (double)Y[(int64_t)r * 2 * M + a] - c[a] * vm[a];
  }
  double qaq, qmq, gq[M];
  gram_forms<D, W>(gtab + (int64_t)id * M, gamtab + (int64_t)id * M, q, qaq, qmq, gq);
  const double lim = rho_star[id] + thr;
  const bool ok = (qaq > 0.0) && isfinite(qmq) && (qmq <= lim * lim * qaq);
  const double2* act = actab + (int64_t)id * M;
#pragma unroll
  for (int a = 0; a < M; ++a) {
    double pr, cr;
    if (ok) {
      cr = gq[a];
      pr = exact_entry(q[a], gq[a], vm[a]);
    } else {
      const double2 ac = act[a];
      cr = ac.y;
      pr = exact_entry(ac.x, ac.y, vm[a]);
    }
    P[j * M + a] = pr;
    Crows[j * M + a] = cr;
  }
  fallback[j] = ok ? 0 : 1;
  if (!ok) atomicAdd(nfall, 1);
}

}  // namespace

namespace lsp {

#define LSP_DW_DISPATCH(FN, ...)                                              \
  do {                                                                        \
    const int W_ = 2 * p->t + 1;                                              \
    if (p->d == 2 && W_ == 3) { FN<2, 3><<<grid, blk, 0, p->stream>>>(__VA_ARGS__); } \
    else if (p->d == 2 && W_ == 5) { FN<2, 5><<<grid, blk, 0, p->stream>>>(__VA_ARGS__); } \
    else if (p->d == 2 && W_ == 7) { FN<2, 7><<<grid, blk, 0, p->stream>>>(__VA_ARGS__); } \
    else if (p->d == 3 && W_ == 3) { FN<3, 3><<<grid, blk, 0, p->stream>>>(__VA_ARGS__); } \
    else return hipErrorInvalidValue;                                         \
  } while (0)

hipError_t launch_features(const lsp_problem* p, const int64_t* points, int64_t j0, int rows,
                           float* X) {
  const dim3 grid(blocks_for(rows, 128)), blk(128);
  const double h2 = 1.0 / ((double)p->n * p->n);
  LSP_DW_DISPATCH(features_kernel, p->v, p->n, p->N, p->ws.S, p->ws.nS, points, j0, rows, h2,
                  X);
  return hipGetLastError();
}

hipError_t launch_targets(const lsp_problem* p, const double* P, const int64_t* points, int rows,
                          float* T) {
  const dim3 grid(blocks_for(rows, 128)), blk(128);
  LSP_DW_DISPATCH(targets_kernel, P, p->v, p->N, p->ws.S, p->ws.nS, p->ws.Ctab, points, rows,
                  T);
  return hipGetLastError();
}

hipError_t launch_learned_rows(const lsp_problem* p, const double* rho_star, const float* Y,
                               int64_t j0, int rows, double thr, double* P, double* Crows,
                               int32_t* fallback, int* nfall) {
  const dim3 grid(blocks_for(rows, 64)), blk(64);
  LSP_DW_DISPATCH(learned_rows_kernel, p->v, p->n, p->ws.S, p->ws.nS, p->ws.gtab, p->ws.gamtab,
                  reinterpret_cast<const double2*>(p->ws.actab), rho_star, Y, j0, rows, thr, P,
                  Crows, fallback, nfall);
  return hipGetLastError();
}

#undef LSP_DW_DISPATCH

}  // namespace lsp
