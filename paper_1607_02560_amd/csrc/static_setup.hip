// lsp_stencil_setup_static: the stencil setup of lsp_stencil_setup for a 2D
// problem with no allocation at all, for callers that cannot allocate (code
// under HIP graph capture, serving loops, harnesses that forbid it).
//
// Every intermediate of the setup (the min/max partials, the shift list, the folded cosine table, the Green's partial sums and the
// per-shift tables) lives in one file-scope device array, `scratch`, of
// kStaticScratchBytes per GPU. The array's name is only a host-side stand-in:
// its device address is looked up once per device (hipGetSymbolAddress, with
// that device current) and only that address is handed to kernels. The
// kernels are those of lsp_stencil_setup, launched on the same arguments, so
// the rows and shift indices are bit for bit those of lsp_stencil_setup on a
// problem with the same potential.
//
// Every call on one GPU shares its array, which keeps the last call's
// contents: calls that overlap on one GPU (on different streams, or from
// different threads) race. Every value of the array is written by the
// launch before the one that reads it, so nothing needs clearing.
#include <mutex>

#include "lsp_internal.h"

namespace {

constexpr size_t kStaticScratchBytes = size_t(8) << 20;  // per GPU
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_mu;
unsigned char* g_ptr[kMaxDevices] = {};

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Byte offsets of the setup's buffers in the static array for (n, t, shifts).
struct Carve {
  size_t minmax, S, nS, vrange, cw, part, gtab, gamtab, Mtab, alpha, Ctab, sigma, rho,
      actab, status, total;
};

Carve carve(int n, int t, int shifts) {
  const int W = 2 * t + 1;
  const int m = W * W;
  Carve c{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align256(off + bytes);
    return at;
  };
  c.minmax = take(sizeof(double) * 3 * lsp::kMinMaxBlocks);
  c.S = take(sizeof(double) * lsp::kMaxShifts);
  c.nS = take(sizeof(int));
  c.vrange = take(sizeof(double) * 2);
  c.cw = take(sizeof(double) * (size_t)lsp::cos_table_doubles(n, W));
  c.part = take(sizeof(double) * lsp::green_partial_doubles(2, n, t, shifts));
  c.gtab = take(sizeof(double) * (size_t)shifts * m);
  c.gamtab = take(sizeof(double) * (size_t)shifts * m);
  c.Mtab = take(sizeof(double) * (size_t)shifts * m * m);
  c.alpha = take(sizeof(double) * (size_t)shifts * m);
  c.Ctab = take(sizeof(double) * (size_t)shifts * m);
  c.sigma = take(sizeof(double) * shifts);
  c.rho = take(sizeof(double) * shifts);
  c.actab = take(sizeof(double) * 2 * (size_t)shifts * m);
  c.status = take(sizeof(int) * shifts);
  c.total = off;
  return c;
}

}  // namespace

extern "C" {

size_t lsp_static_scratch_bytes(void) { return kStaticScratchBytes; }

int lsp_stencil_setup_static(int d, int n, const double* v_dev, int t, int num_shifts,
                             int precision, void* P_dev, int32_t* idx_dev, void* stream) {
  if (d != 2) return lsp::set_error(LSP_EINVAL, "the allocation-free setup takes d = 2");
  if (n < 8 || n > 1024 || (n & (n - 1)) != 0)
    return lsp::set_error(LSP_EINVAL, "n must be a power of two in [8, 1024]");
  if (!v_dev || !P_dev) return lsp::set_error(LSP_EINVAL, "NULL argument");
  if (precision != LSP_FP64 && precision != LSP_FP32_REFINE)
    return lsp::set_error(LSP_EINVAL, "unsupported precision");
  if (t < 1 || t > 3) return lsp::set_error(LSP_EINVAL, "d = 2 supports t = 1, 2, 3");
  const int W = 2 * t + 1;
  const int m = W * W;
  const int64_t N = (int64_t)n * n;
  if (W >= n) return lsp::set_error(LSP_EINVAL, "2t+1 must be smaller than n");
  if (N < 2 * (int64_t)m) return lsp::set_error(LSP_EINVAL, "N must be at least 2m");
  if (num_shifts == 0) num_shifts = lsp_default_num_shifts(d, n);
  if (num_shifts < 1 || num_shifts > lsp::kMaxShifts)
    return lsp::set_error(LSP_EINVAL, "num_shifts must be in 0..1024");
  const Carve c = carve(n, t, num_shifts);
  if (c.total > kStaticScratchBytes)
    return lsp::set_error(LSP_EINVAL, "this setup needs " + std::to_string(c.total) +
                                          " bytes of the " + std::to_string(kStaticScratchBytes) +
                                          "-byte static scratch array");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return lsp::hip_check(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return lsp::set_error(LSP_EINVAL, "device index too large");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  unsigned char* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
      void* ptr = nullptr;
      e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !ptr) return lsp::hip_check(e, "hipGetSymbolAddress(scratch)");
      g_ptr[dev] = static_cast<unsigned char*>(ptr);
    }
    base = g_ptr[dev];
  }
  // a problem object on the stack, its workspace carved from the array: the
  // launchers of lsp_stencil_setup take it as they take a created problem
  lsp_problem p;
  p.d = d;
  p.n = n;
  p.N = N;
  p.stream = s;
  p.device = dev;
  p.v = const_cast<double*>(v_dev);  // read only
  p.t = t;
  p.m = m;
  p.num_shifts = num_shifts;
  lsp::Workspace& w = p.ws;
  w.minmax_part = reinterpret_cast<double*>(base + c.minmax);
  w.S = reinterpret_cast<double*>(base + c.S);
  w.nS = reinterpret_cast<int*>(base + c.nS);
  w.vrange = reinterpret_cast<double*>(base + c.vrange);
  w.green_part = reinterpret_cast<double*>(base + c.part);
  w.green_part_cap = lsp::green_partial_doubles(2, n, t, num_shifts);
  w.gtab = reinterpret_cast<double*>(base + c.gtab);
  w.gamtab = reinterpret_cast<double*>(base + c.gamtab);
  w.Mtab = reinterpret_cast<double*>(base + c.Mtab);
  w.alpha = reinterpret_cast<double*>(base + c.alpha);
  w.Ctab = reinterpret_cast<double*>(base + c.Ctab);
  w.sigma = reinterpret_cast<double*>(base + c.sigma);
  w.rho = reinterpret_cast<double*>(base + c.rho);
  w.actab = reinterpret_cast<double*>(base + c.actab);
  w.status = reinterpret_cast<int*>(base + c.status);
  w.cap_shifts = num_shifts;
  w.cap_m = m;
  w.cap_w = m;
  p.cosT = reinterpret_cast<double*>(base + c.cw);
  // min/max partials with the cosine table, then the Green's sums (which form
  // the shift list), the null vectors and the rows, as lsp_stencil_setup
  // launches them
  e = lsp::launch_minmax_parts(p.v, N, w, false, s, n, W, p.cosT);
  if (e == hipSuccess) e = lsp::launch_green_sums(&p, num_shifts);
  if (e == hipSuccess) e = lsp::launch_null_vectors(&p, num_shifts);
  if (e == hipSuccess) e = lsp::launch_assemble(&p, P_dev, precision == LSP_FP32_REFINE, idx_dev);
  if (e != hipSuccess) return lsp::hip_check(e, "allocation-free setup launch");
  return LSP_OK;
}

}  // extern "C"
