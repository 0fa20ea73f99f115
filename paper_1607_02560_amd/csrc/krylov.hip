// Device BLAS-1 kernels for the right-preconditioned GMRES of lsp_precond_solve
// (Sec. 5: GMRES with restart 40 and the preconditioner P^-1 C).
// Vectors are complex128, interleaved. Reductions are deterministic: each
// block reduces a fixed slice in a fixed order and the host adds the block
// results in block order.
#include "lsp_internal.h"

namespace {

constexpr int kThreads = 256;

// part[i * nblk + b] = sum over block b's slice of conj(V_i) w, i < nv.
__global__ __launch_bounds__(kThreads) void multi_dot_kernel(const double2* __restrict__ V,
                                                             int64_t ldv, int nv,
                                                             const double2* __restrict__ w,
                                                             int64_t N, double2* part) {
  __shared__ double sr[kThreads], si[kThreads];
  const int tid = threadIdx.x;
  for (int i = 0; i < nv; ++i) {
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
    __syncthreads();
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
  hipLaunchKernelGGL(multi_dot_kernel, dim3(dot_blocks(N)), dim3(kThreads), 0, s,
                     reinterpret_cast<const double2*>(V), ldv, nv,
                     reinterpret_cast<const double2*>(w), N, reinterpret_cast<double2*>(part));
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
