// Device kernels of the right-preconditioned GMRES (Sec. 5: GMRES with
// restart 40 and the preconditioner P^-1 C): BLAS-1 on complex128 vectors
// (interleaved) and the small Hessenberg-side steps of the device solve.
// Reductions are deterministic: each block reduces a fixed slice in a fixed
// order, then the block results are added in a fixed order (on the host by
// lsp_precond_solve, by reduce_parts_kernel on the device).
#include "lsp_internal.h"

namespace {

constexpr int kThreads = 256;

// part[i * nblk + b] = sum over block b's slice of conj(V_i) w, i < nv.
// Block b of row i (blockIdx.y) sums a fixed slice.
__global__ __launch_bounds__(kThreads) void multi_dot_kernel(const double2* __restrict__ V,
                                                             int64_t ldv,
                                                             const double2* __restrict__ w,
                                                             int64_t N, double2* part) {
  __shared__ double sr[kThreads], si[kThreads];
  const int tid = threadIdx.x;
  const int i = blockIdx.y;
  const double2* vi = V + (int64_t)i * ldv;
  double ar = 0.0, ai = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * kThreads + tid; e < N;
       e += (int64_t)gridDim.x * kThreads) {
    const double2 a = vi[e], b = w[e];
    // conj(a) * b
    ar = fma(a.x, b.x, ar);
    ar = fma(a.y, b.y, ar);
    ai = fma(a.x, b.y, ai);
    ai = fma(-a.y, b.x, ai);
  }
  sr[tid] = ar;
  si[tid] = ai;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if (tid < s) {
      sr[tid] += sr[tid + s];
      si[tid] += si[tid + s];
    }
    __syncthreads();
  }
  if (tid == 0) part[(int64_t)i * gridDim.x + blockIdx.x] = make_double2(sr[0], si[0]);
}

// Sum of the nblk (<= kThreads) partials of one block row, in tree order.
__device__ double2 block_sum(const double2* __restrict__ part, int nblk, double* sr, double* si) {
  const int tid = threadIdx.x;
  const double2 a = tid < nblk ? part[tid] : make_double2(0.0, 0.0);
  sr[tid] = a.x;
  si[tid] = a.y;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if (tid < s) {
      sr[tid] += sr[tid + s];
      si[tid] += si[tid + s];
    }
    __syncthreads();
  }
  return make_double2(sr[0], si[0]);
}

// out[i] = sum over b of part[i * nblk + b]: the second stage of the dots
__global__ __launch_bounds__(kThreads) void reduce_parts_kernel(const double2* __restrict__ part,
                                                                int nblk, double2* out) {
  __shared__ double sr[kThreads], si[kThreads];
  const double2 v = block_sum(part + (int64_t)blockIdx.x * nblk, nblk, sr, si);
  if (threadIdx.x == 0) out[blockIdx.x] = v;
}

// The norm of a vector from its dot partials <x, x>. mode 0: ||f||, kept in
// sc[kScFnorm]. mode 1: start of a restart cycle with r = x: beta = ||r||,
// g = (beta, 0, ..., 0), the estimate beta / ||f|| and the scale 1 / beta
// of the first basis vector.
__global__ __launch_bounds__(kThreads) void krylov_norm_kernel(const double2* __restrict__ part,
                                                               int nblk, int mode, int restart,
                                                               double* sc, double2* g) {
  __shared__ double sr[kThreads], si[kThreads];
  const double2 v = block_sum(part, nblk, sr, si);
  if (threadIdx.x != 0) return;
  const double nrm = sqrt(v.x);
  if (mode == 0) {
    sc[lsp::kScFnorm] = nrm;
    return;
  }
  sc[lsp::kScBeta] = nrm;
  sc[lsp::kScEst] = nrm / sc[lsp::kScFnorm];
  sc[lsp::kScInv] = nrm > 0.0 ? 1.0 / nrm : 0.0;
  sc[lsp::kScBreak] = 0.0;
  g[0] = make_double2(nrm, 0.0);
  for (int i = 1; i <= restart; ++i) g[i] = make_double2(0.0, 0.0);
}

__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 cconj(double2 a) { return make_double2(a.x, -a.y); }

// Column k of the Hessenberg matrix after classical Gram-Schmidt twice:
// h = hA + hB (the two passes' coefficients), h_{k+1,k} = ||w|| from the
// partials of <w, w>. The column is rotated by the earlier Givens rotations,
// a new rotation zeroes h_{k+1,k}, and the right-hand side g is rotated with
// it; |g_{k+1}| / ||f|| is the residual estimate. H is restart x restart,
// row-major; cs, sn, g as in the host loop of lsp_precond_solve.
__global__ __launch_bounds__(kThreads) void givens_kernel(
    const double2* __restrict__ part, int nblk, const double2* __restrict__ hA,
    const double2* __restrict__ hB, double2* H, double2* cs, double2* sn, double2* g, double* sc,
    int k, int restart) {
  __shared__ double sr[kThreads], si[kThreads];
  const double2 wn2 = block_sum(part, nblk, sr, si);
  if (threadIdx.x != 0) return;
  const double hk1 = sqrt(wn2.x);
  double2* col = H + k;  // entry i at col[i * restart]
  for (int i = 0; i <= k; ++i)
    col[(int64_t)i * restart] = make_double2(hA[i].x + hB[i].x, hA[i].y + hB[i].y);
  // earlier rotations: (h_i, h_{i+1}) <- (conj(c) h_i + conj(s) h_{i+1}, -s h_i + c h_{i+1})
  for (int i = 0; i < k; ++i) {
    const double2 hi = col[(int64_t)i * restart], hi1 = col[(int64_t)(i + 1) * restart];
    const double2 a = cmul(cconj(cs[i]), hi), b = cmul(cconj(sn[i]), hi1);
    const double2 c = cmul(sn[i], hi), d = cmul(cs[i], hi1);
    col[(int64_t)i * restart] = make_double2(a.x + b.x, a.y + b.y);
    col[(int64_t)(i + 1) * restart] = make_double2(d.x - c.x, d.y - c.y);
  }
  const double2 a = col[(int64_t)k * restart];
  const double rho = hypot(hypot(a.x, a.y), hk1);
  const double2 c = rho > 0.0 ? make_double2(a.x / rho, a.y / rho) : make_double2(1.0, 0.0);
  const double2 sv = rho > 0.0 ? make_double2(hk1 / rho, 0.0) : make_double2(0.0, 0.0);
  cs[k] = c;
  sn[k] = sv;
  col[(int64_t)k * restart] = make_double2(rho, 0.0);
  const double2 gk = g[k];
  const double2 gn = cmul(sv, gk);
  g[k + 1] = make_double2(-gn.x, -gn.y);
  g[k] = cmul(cconj(c), gk);
  sc[lsp::kScEst] = hypot(g[k + 1].x, g[k + 1].y) / sc[lsp::kScFnorm];
  sc[lsp::kScInv] = hk1 > 0.0 ? 1.0 / hk1 : 0.0;
  sc[lsp::kScBreak] = hk1 > 0.0 ? 0.0 : 1.0;
}

// y = H^-1 g for the leading k_used x k_used upper triangle (back substitution)
__global__ void trisolve_kernel(const double2* __restrict__ H, const double2* __restrict__ g,
                                int k_used, int restart, double2* y) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int i = k_used - 1; i >= 0; --i) {
    double2 acc = g[i];
    for (int j = i + 1; j < k_used; ++j) {
      const double2 t = cmul(H[(int64_t)i * restart + j], y[j]);
      acc.x -= t.x;
      acc.y -= t.y;
    }
    const double2 h = H[(int64_t)i * restart + i];
    const double den = h.x * h.x + h.y * h.y;
    y[i] = make_double2((acc.x * h.x + acc.y * h.y) / den, (acc.y * h.x - acc.x * h.y) / den);
  }
}

// y = a[0] * x with the scale read on the device
__global__ __launch_bounds__(kThreads) void scale_dev_kernel(const double2* __restrict__ x,
                                                             const double* __restrict__ a,
                                                             double2* y, int64_t N) {
  const double f = a[0];
  for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < N;
       e += (int64_t)gridDim.x * kThreads) {
    const double2 v = x[e];
    y[e] = make_double2(f * v.x, f * v.y);
  }
}

// w += sign * sum_i coef_i V_i
__global__ __launch_bounds__(kThreads) void multi_axpy_kernel(const double2* __restrict__ V,
                                                              int64_t ldv, int nv,
                                                              const double2* __restrict__ coef,
                                                              double sign, double2* w,
                                                              int64_t N) {
  for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < N;
       e += (int64_t)gridDim.x * kThreads) {
    double2 acc = w[e];
    for (int i = 0; i < nv; ++i) {
      const double2 c = coef[i];
      const double2 x = V[(int64_t)i * ldv + e];
      acc.x = fma(sign * c.x, x.x, acc.x);
      acc.x = fma(-sign * c.y, x.y, acc.x);
      acc.y = fma(sign * c.x, x.y, acc.y);
      acc.y = fma(sign * c.y, x.x, acc.y);
    }
    w[e] = acc;
  }
}

// y = a * x (real a), or y = b - x when sub is set
__global__ __launch_bounds__(kThreads) void scale_kernel(const double2* __restrict__ x, double a,
                                                         double2* y, int64_t N) {
  for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < N;
       e += (int64_t)gridDim.x * kThreads) {
    const double2 v = x[e];
    y[e] = make_double2(a * v.x, a * v.y);
  }
}

__global__ __launch_bounds__(kThreads) void sub_kernel(const double2* __restrict__ b,
                                                       const double2* __restrict__ x, double2* y,
                                                       int64_t N) {
  for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < N;
       e += (int64_t)gridDim.x * kThreads) {
    const double2 u = b[e], v = x[e];
    y[e] = make_double2(u.x - v.x, u.y - v.y);
  }
}

}  // namespace

namespace lsp {

int dot_blocks(int64_t N) {
  int64_t b = (N + kThreads - 1) / kThreads;
  if (b > 256) b = 256;
  return (int)(b < 1 ? 1 : b);
}

hipError_t launch_multi_dot(const double* V, int64_t ldv, int nv, const double* w, int64_t N,
                            double* part, hipStream_t s) {
  if (nv < 1) return hipSuccess;
  hipLaunchKernelGGL(multi_dot_kernel, dim3(dot_blocks(N), nv), dim3(kThreads), 0, s,
                     reinterpret_cast<const double2*>(V), ldv,
                     reinterpret_cast<const double2*>(w), N, reinterpret_cast<double2*>(part));
  return hipGetLastError();
}

hipError_t launch_reduce_parts(const double* part, int nblk, int nv, double* out,
                               hipStream_t s) {
  if (nv < 1) return hipSuccess;
  hipLaunchKernelGGL(reduce_parts_kernel, dim3(nv), dim3(kThreads), 0, s,
                     reinterpret_cast<const double2*>(part), nblk, reinterpret_cast<double2*>(out));
  return hipGetLastError();
}

hipError_t launch_krylov_norm(const double* part, int nblk, int mode, int restart, double* sc,
                              double* g, hipStream_t s) {
  hipLaunchKernelGGL(krylov_norm_kernel, dim3(1), dim3(kThreads), 0, s,
                     reinterpret_cast<const double2*>(part), nblk, mode, restart, sc,
                     reinterpret_cast<double2*>(g));
  return hipGetLastError();
}

hipError_t launch_givens(const double* part, int nblk, const double* hA, const double* hB,
                         double* H, double* cs, double* sn, double* g, double* sc, int k,
                         int restart, hipStream_t s) {
  hipLaunchKernelGGL(givens_kernel, dim3(1), dim3(kThreads), 0, s,
                     reinterpret_cast<const double2*>(part), nblk,
                     reinterpret_cast<const double2*>(hA), reinterpret_cast<const double2*>(hB),
                     reinterpret_cast<double2*>(H), reinterpret_cast<double2*>(cs),
                     reinterpret_cast<double2*>(sn), reinterpret_cast<double2*>(g), sc, k,
                     restart);
  return hipGetLastError();
}

hipError_t launch_trisolve(const double* H, const double* g, int k_used, int restart, double* y,
                           hipStream_t s) {
  hipLaunchKernelGGL(trisolve_kernel, dim3(1), dim3(64), 0, s,
                     reinterpret_cast<const double2*>(H), reinterpret_cast<const double2*>(g),
                     k_used, restart, reinterpret_cast<double2*>(y));
  return hipGetLastError();
}

hipError_t launch_scale_dev(const double* x, const double* a, double* y, int64_t N,
                            hipStream_t s) {
  int64_t b = (N + kThreads - 1) / kThreads;
  if (b > 4096) b = 4096;
  hipLaunchKernelGGL(scale_dev_kernel, dim3((unsigned)(b < 1 ? 1 : b)), dim3(kThreads), 0, s,
                     reinterpret_cast<const double2*>(x), a, reinterpret_cast<double2*>(y), N);
  return hipGetLastError();
}

hipError_t launch_multi_axpy(const double* V, int64_t ldv, int nv, const double* coef,
                             double sign, double* w, int64_t N, hipStream_t s) {
  int64_t b = (N + kThreads - 1) / kThreads;
  if (b > 4096) b = 4096;
  hipLaunchKernelGGL(multi_axpy_kernel, dim3((unsigned)(b < 1 ? 1 : b)), dim3(kThreads), 0, s,
                     reinterpret_cast<const double2*>(V), ldv, nv,
                     reinterpret_cast<const double2*>(coef), sign, reinterpret_cast<double2*>(w),
                     N);
  return hipGetLastError();
}

hipError_t launch_scale(const double* x, double a, double* y, int64_t N, hipStream_t s) {
  int64_t b = (N + kThreads - 1) / kThreads;
  if (b > 4096) b = 4096;
  hipLaunchKernelGGL(scale_kernel, dim3((unsigned)(b < 1 ? 1 : b)), dim3(kThreads), 0, s,
                     reinterpret_cast<const double2*>(x), a, reinterpret_cast<double2*>(y), N);
  return hipGetLastError();
}

hipError_t launch_sub(const double* b_, const double* x, double* y, int64_t N, hipStream_t s) {
  int64_t b = (N + kThreads - 1) / kThreads;
  if (b > 4096) b = 4096;
  hipLaunchKernelGGL(sub_kernel, dim3((unsigned)(b < 1 ? 1 : b)), dim3(kThreads), 0, s,
                     reinterpret_cast<const double2*>(b_), reinterpret_cast<const double2*>(x),
                     reinterpret_cast<double2*>(y), N);
  return hipGetLastError();
}

}  // namespace lsp
