// Gram matrix of eq. (A) and the stencil alpha_s (Sec. 3, 4.2), one block
// per shift.
//
// With g = g_s and q = g_s * g_s on the offsets [0, 2t]^d:
//   G_mu,mu[a][b] = g[|a - b|],  A1[a][b] = q[|a - b|],  M = A1 - G_mu,mu G_mu,mu
// and alpha_s is the unit eigenvector of the smallest eigenvalue of M
// (the smallest left singular vector of G_s[mu, mu^c]); sigma_min^2 is that
// eigenvalue and C_s = G_mu,mu alpha_s.
//
// Because g and q are even in every coordinate, all three matrices are block
// diagonal in the parity basis of the neighbourhood (see Parity): 2^d blocks,
// e.g. sizes 9, 6, 6, 4 for d = 2, t = 2. Wave c of the block owns parity
// class c. Lane p holds row p of G_b, A1_b, M_b and X_b = M_b^-1 in
// registers; rows are shared through readlane broadcasts, so no LDS traffic or
// barriers sit on the serial path. Per class:
//   1. rows of G_b and A1_b from the tables, A2_b = G_b G_b, M_b = A1_b - A2_b;
//   2. X_b = M_b^-1 by Gauss-Jordan elimination (M is positive semi-definite;
//      a non-positive pivot restarts on M_b + tau I, which has the same
//      eigenvectors);
//   3. power iteration with X_b (the smallest eigenvector of M_b is the
//      dominant one of X_b) until successive normalised iterates differ by
//      less than 1e-15;
//   4. two inverse-iteration steps whose solve is refined once against the
//      FP64 M_b (y0 = X x, y = y0 + X (x - M y0)), removing the forward error
//      of the explicit inverse;
//   5. lambda_c = x^T M_b x, x^T A1_b x and G_b x.
// The class with the smallest lambda_c gives alpha (ties: lowest class);
// alpha and C are mapped back to the offsets of mu_0^t, normalised to unit
// norm with the largest-magnitude entry positive (lowest offset on ties);
// rho*(s) = sqrt(lambda_c / x^T A1_b x) is the fraction of the row of Q G that
// alpha's truncation drops (eq. A), which the learned setup's check compares
// against.
#include "setup_common.h"

#pragma clang fp contract(off)

namespace {

using lsp::bcast;
using lsp::Nbhd;
using lsp::Parity;
using lsp::Pow;

template <int D, int W>
struct NullShared {
  static constexpr int NC = 1 << D;
  static constexpr int WD = Pow<D, W>::v;
  static constexpr int BMAX = Parity<D, W>::size(0);
  double g[WD];
  double q[WD];
  double lam[NC];
  double ax[NC];  // x^T A1_b x of the class's vector
  double vec[NC][BMAX];
  double gv[NC][BMAX];
  int status[NC];
  double stage[4096];
};

template <int D, int W, int C>
__device__ void solve_class(NullShared<D, W>& sh, int lane, int si, double* Mtab_si) {
  using Pa = Parity<D, W>;
  constexpr int B = Pa::size(C);
  constexpr int NS = 1 << D;  // per-axis term choices of a block entry
  static_assert(3 * Pa::offset(Pa::NC) <= Pow<D, W>::v * Pow<D, W>::v,
                "the M, A1 and G blocks of a shift share its m*m slot");
  const int p = (lane < B) ? lane : 0;
  // 3D with t = 2 (27-row classes): keep fewer values live across the power
  // iteration, so that the kernel stays within the register file: the
  // convergence test tracks only the lane's own entry (then the largest
  // change over the wave, the same maximum), and G_b x and A1_b x at the end
  // read the rows back from the shift's table instead of keeping them
  constexpr bool kLean = (D == 3 && W == 5);

  // per-axis 1D indices of row p
  int jp[D];
#pragma unroll
  for (int i = 0; i < D; ++i) jp[i] = Pa::coord(C, p, i);

  // ---- rows of G_b and A1_b ----
  // In the parity basis a block entry factorises over axes: for 1D indices
  // j (row) and j' (column) of one axis, the reflected pairs collapse to
  //   odd axis:             f(|j - j'|) - f(j + j')
  //   even, j, j' > 0:      f(|j - j'|) + f(j + j')
  //   even, one of them 0:  sqrt2 f(j + j')
  //   even, both 0:         f(0)
  // so an entry of G_b (f = g) or A1_b (f = g*g) is a sum over the 2^D
  // choices of the per-axis terms, each a product of weights times one
  // table value g[dd_1, ..., dd_D].
  double grow[B], arow[B];
#pragma unroll
  for (int qc = 0; qc < B; ++qc) {
    int dd0[D], dd1[D];
    double w0[D], w1[D];
#pragma unroll
    for (int i = 0; i < D; ++i) {
      const int jq = Pa::coord(C, qc, i);
      const int j = jp[i];
      const int dm = (j > jq) ? j - jq : jq - j;
      dd0[i] = dm;
      dd1[i] = j + jq;
      if (Pa::odd(C, i)) {
        w0[i] = 1.0;
        w1[i] = -1.0;
      } else if (j > 0 && jq > 0) {
        w0[i] = 1.0;
        w1[i] = 1.0;
      } else if (j == 0 && jq == 0) {
        w0[i] = 1.0;
        w1[i] = 0.0;
      } else {
        dd0[i] = j + jq;
        w0[i] = 1.4142135623730951;
        w1[i] = 0.0;
      }
    }
    double sg = 0.0, sq = 0.0;
#pragma unroll
    for (int cmb = 0; cmb < NS; ++cmb) {
      double w = 1.0;
      int idx = 0;
#pragma unroll
      for (int i = 0; i < D; ++i) {
        const bool second = (cmb >> (D - 1 - i)) & 1;
        w *= second ? w1[i] : w0[i];
        idx = idx * W + (second ? dd1[i] : dd0[i]);
      }
      sg = fma(w, sh.g[idx], sg);
      sq = fma(w, sh.q[idx], sq);
    }
    grow[qc] = sg;
    arow[qc] = sq;
  }

  // ---- M_b = A1_b - G_b G_b ----
  double mrow[B];
#pragma unroll
  for (int qc = 0; qc < B; ++qc) mrow[qc] = 0.0;
  if constexpr (kLean) {
    // 3D with t = 2: row r of G_b comes from LDS, one broadcast read per
    // entry (all lanes read the same address), in place of a lane-r
    // broadcast through a scalar register per entry: the same operands in
    // the same order. The class's block of the partial-sum staging area
    // (free while the classes run) holds it. Columns go in chunks of KC
    // with a rolled loop over r inside (the lane's own G[p][r] read back
    // from LDS too): fully unrolled, the B*B reads are hoisted and spill.
    static_assert(Pa::offset(Pa::NC) <= (int)(sizeof(sh.stage) / sizeof(double)),
                  "the G blocks fit the staging area");
    double* gb = sh.stage + Pa::offset(C);
    if (lane < B) {
      // the A1 and G blocks go out here (below for the other shapes), so
      // that G's row need not stay live across the product
      double* ao = Mtab_si + Pa::offset(Pa::NC) + Pa::offset(C) + lane * B;
      double* go = Mtab_si + 2 * Pa::offset(Pa::NC) + Pa::offset(C) + lane * B;
#pragma unroll
      for (int qc = 0; qc < B; ++qc) {
        gb[lane * B + qc] = grow[qc];
        ao[qc] = arow[qc];
        go[qc] = grow[qc];
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    constexpr int KC = 9;
#pragma unroll
    for (int c0 = 0; c0 < B; c0 += KC) {
#pragma unroll 1
      for (int r = 0; r < B; ++r) {
        const double gpr = gb[p * B + r];
#pragma unroll
        for (int qc = c0; qc < ((c0 + KC < B) ? c0 + KC : B); ++qc)
          mrow[qc] = fma(gpr, gb[r * B + qc], mrow[qc]);
      }
    }
  } else {
#pragma unroll
    for (int r = 0; r < B; ++r) {
#pragma unroll
      for (int qc = 0; qc < B; ++qc) mrow[qc] = fma(grow[r], bcast(grow[qc], r), mrow[qc]);
    }
  }
#pragma unroll
  for (int qc = 0; qc < B; ++qc) mrow[qc] = arow[qc] - mrow[qc];
  if (lane < B) {
    // the shift's M blocks, then (after all of them) its A1 blocks, then its
    // G blocks (the learned setup forms C = G q from them)
    double* mo = Mtab_si + Pa::offset(C) + lane * B;
    double* ao = Mtab_si + Pa::offset(Pa::NC) + Pa::offset(C) + lane * B;
    double* go = Mtab_si + 2 * Pa::offset(Pa::NC) + Pa::offset(C) + lane * B;
#pragma unroll
    for (int qc = 0; qc < B; ++qc) {
      mo[qc] = mrow[qc];
      if constexpr (!kLean) {
        ao[qc] = arow[qc];
        go[qc] = grow[qc];
      }
    }
  }

  // ---- X_b = (M_b + tau I)^-1 by Gauss-Jordan ----
  double dmax = 0.0;
#pragma unroll
  for (int k = 0; k < B; ++k) {
    double dk = 0.0;
#pragma unroll
    for (int qc = 0; qc < B; ++qc)
      if (qc == k) dk = mrow[qc];
    dmax = fmax(dmax, fabs(bcast(dk, k)));
  }
  double xrow[B];
  double tau = 0.0;
  int tries = 0;
  bool ok = false;
  while (!ok && tries < 4) {
#pragma unroll
    for (int qc = 0; qc < B; ++qc) xrow[qc] = mrow[qc] + ((qc == p) ? tau : 0.0);
    ok = true;
#pragma unroll
    for (int k = 0; k < B; ++k) {
      double rk[B];
#pragma unroll
      for (int qc = 0; qc < B; ++qc) rk[qc] = bcast(xrow[qc], k);
      const double piv = rk[k];
      if (!(piv > 0.0) || !isfinite(piv)) ok = false;  // uniform: piv is broadcast
      const double inv = ok ? lsp::rcp_nr(piv) : 0.0;
      if (lane == k) {
#pragma unroll
        for (int qc = 0; qc < B; ++qc) xrow[qc] = (qc == k) ? inv : rk[qc] * inv;
      } else {
        double xk = 0.0;
#pragma unroll
        for (int qc = 0; qc < B; ++qc)
          if (qc == k) xk = xrow[qc];
        const double f = xk * inv;
#pragma unroll
        for (int qc = 0; qc < B; ++qc) xrow[qc] = (qc == k) ? -f : fma(-f, rk[qc], xrow[qc]);
      }
    }
    if (!ok) {
      ++tries;
      tau = (tau == 0.0) ? 1e-14 * dmax : tau * 100.0;
    }
  }

  // ---- power iteration on X_b (vector replicated in every lane) ----
  double xscale = 0.0;  // 1 / (largest |diagonal| of X_b): keeps iterates O(1)
#pragma unroll
  for (int k = 0; k < B; ++k) {
    double dk = 0.0;
#pragma unroll
    for (int qc = 0; qc < B; ++qc)
      if (qc == k) dk = xrow[qc];
    xscale = fmax(xscale, fabs(bcast(dk, k)));
  }
  xscale = (xscale > 0.0 && isfinite(xscale)) ? 1.0 / xscale : 1.0;
  constexpr int NPREV = kLean ? 1 : B;
  double xa[B], xprev[NPREV];
#pragma unroll
  for (int qc = 0; qc < B; ++qc) xa[qc] = 1.0 + 0.37 * (double)((qc * 7 + 3) % 11) / 11.0;  // generic start
#pragma unroll
  for (int qc = 0; qc < NPREV; ++qc) xprev[qc] = 0.0;
  for (int it = 0; it < 100; ++it) {
#pragma unroll
    for (int rep = 0; rep < 4; ++rep) {
      // three interleaved partial sums: a third of the FMA chain's latency
      double y0 = 0.0, y1 = 0.0, y2 = 0.0;
#pragma unroll
      for (int qc = 0; qc < B; qc += 3) {
        y0 = fma(xrow[qc], xa[qc], y0);
        if (qc + 1 < B) y1 = fma(xrow[qc + 1], xa[qc + 1], y1);
        if (qc + 2 < B) y2 = fma(xrow[qc + 2], xa[qc + 2], y2);
      }
      double y = (y0 + y1) + y2;
      y *= xscale;
#pragma unroll
      for (int qc = 0; qc < B; ++qc) xa[qc] = bcast(y, qc);
    }
    double nrm = 0.0;
#pragma unroll
    for (int qc = 0; qc < B; ++qc) nrm = fma(xa[qc], xa[qc], nrm);
    const double sc = lsp::rsqrt_nr(nrm);
    double dmx = 0.0;
    if constexpr (kLean) {
      double xo = 0.0;
#pragma unroll
      for (int qc = 0; qc < B; ++qc) {
        xa[qc] *= sc;
        if (qc == p) xo = xa[qc];
      }
      dmx = (lane < B) ? fabs(xo - xprev[0]) : 0.0;
      xprev[0] = xo;
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) dmx = fmax(dmx, __shfl_xor(dmx, o));
    } else {
#pragma unroll
      for (int qc = 0; qc < B; ++qc) {
        xa[qc] *= sc;
        dmx = fmax(dmx, fabs(xa[qc] - xprev[qc]));
        xprev[qc] = xa[qc];
      }
    }
    if (dmx < 1e-15) break;
  }

  // ---- two inverse-iteration steps with one refinement of each solve ----
  for (int step = 0; step < 2; ++step) {
    double y0 = 0.0;
#pragma unroll
    for (int qc = 0; qc < B; ++qc) y0 = fma(xrow[qc], xa[qc], y0);
    double y0a[B];
#pragma unroll
    for (int qc = 0; qc < B; ++qc) y0a[qc] = bcast(y0, qc);
    double my = 0.0, xp = 0.0;
#pragma unroll
    for (int qc = 0; qc < B; ++qc) {
      my = fma(mrow[qc], y0a[qc], my);
      if (qc == p) {
        my = fma(tau, y0a[qc], my);
        xp = xa[qc];
      }
    }
    const double rr = xp - my;
    double ra[B];
#pragma unroll
    for (int qc = 0; qc < B; ++qc) ra[qc] = bcast(rr, qc);
    double cy = 0.0;
#pragma unroll
    for (int qc = 0; qc < B; ++qc) cy = fma(xrow[qc], ra[qc], cy);
    const double yp = y0 + cy;
    double nrm = 0.0;
#pragma unroll
    for (int qc = 0; qc < B; ++qc) {
      xa[qc] = bcast(yp, qc);
      nrm = fma(xa[qc], xa[qc], nrm);
    }
    const double sc = lsp::rsqrt_nr(nrm);
#pragma unroll
    for (int qc = 0; qc < B; ++qc) xa[qc] *= sc;
  }

  // ---- lambda_c = x^T M_b x, G_b x ----
  double mx = 0.0, gx = 0.0, ay = 0.0;
  if constexpr (kLean) {
    // row p of G_b and of A1_b as this lane stored them above (lanes past
    // the class read row 0; their values are not used)
    const double* gback = Mtab_si + 2 * Pa::offset(Pa::NC) + Pa::offset(C) + p * B;
    const double* aback = Mtab_si + Pa::offset(Pa::NC) + Pa::offset(C) + p * B;
#pragma unroll
    for (int qc = 0; qc < B; ++qc) {
      mx = fma(mrow[qc], xa[qc], mx);
      gx = fma(gback[qc], xa[qc], gx);
    }
#pragma unroll
    for (int qc = 0; qc < B; ++qc) ay = fma(aback[qc], xa[qc], ay);
  } else {
#pragma unroll
    for (int qc = 0; qc < B; ++qc) {
      mx = fma(mrow[qc], xa[qc], mx);
      gx = fma(grow[qc], xa[qc], gx);
    }
#pragma unroll
    for (int qc = 0; qc < B; ++qc) ay = fma(arow[qc], xa[qc], ay);
  }
  double lam = 0.0, axx = 0.0;
#pragma unroll
  for (int qc = 0; qc < B; ++qc) {
    lam = fma(xa[qc], bcast(mx, qc), lam);
    axx = fma(xa[qc], bcast(ay, qc), axx);
  }
  if (lane < B) {
    double xl = 0.0;
#pragma unroll
    for (int qc = 0; qc < B; ++qc)
      if (qc == lane) xl = xa[qc];
    sh.vec[C][lane] = xl;
    sh.gv[C][lane] = gx;
  }
  if (lane == 0) {
    sh.lam[C] = ok ? lam : INFINITY;
    sh.ax[C] = axx;
    sh.status[C] = ok ? tries : -1;
  }
}

// alpha and C on mu_0^t for m > 64 offsets (3D, t = 2): wave 0, lane l
// holds offsets l + 64 h. Same mapping, sign rule (largest |alpha| positive,
// lowest offset on ties) and outputs as the m <= 64 path.
template <int D, int W>
__device__ void map_back_wide(NullShared<D, W>& sh, int cs, int wid, int lane, int si,
                              double* alpha_out, double* C_out, double* actab) {
  using Pa = Parity<D, W>;
  using Nb = Nbhd<D, W>;
  constexpr int M = Pow<D, W>::v;
  constexpr int H = (M + 63) / 64;
  if (wid != 0) return;
  double av[H], cv[H];
#pragma unroll
  for (int h = 0; h < H; ++h) {
    av[h] = 0.0;
    cv[h] = 0.0;
    const int a = lane + 64 * h;
    if (a < M) {
      double coef = 1.0;
      int pidx = 0;
      for (int i = 0; i < D; ++i) {
        const int xi = Nb::comp(a, i);
        const int ji = xi < 0 ? -xi : xi;
        const int odd = Pa::odd(cs, i);
        if (odd && ji == 0) coef = 0.0;
        if (ji != 0) coef *= (odd && xi < 0) ? -lsp::kInvSqrt2 : lsp::kInvSqrt2;
        pidx = pidx * Pa::count(cs, i) + (ji - odd < 0 ? 0 : ji - odd);
      }
      if (coef != 0.0) {
        av[h] = coef * sh.vec[cs][pidx];
        cv[h] = coef * sh.gv[cs][pidx];
      }
    }
  }
  // largest |alpha| over all offsets, lowest offset on ties
  double am = -1.0;
  int jm = M;
#pragma unroll
  for (int h = 0; h < H; ++h) {
    const int a = lane + 64 * h;
    if (a < M && fabs(av[h]) > am) {  // h increases with a: ties keep the lower
      am = fabs(av[h]);
      jm = a;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double ao = __shfl_xor(am, o);
    const int jo = __shfl_xor(jm, o);
    if (ao > am || (ao == am && jo < jm)) {
      am = ao;
      jm = jo;
    }
  }
  // alpha at offset jm, from the lane that holds it
  double at = 0.0;
#pragma unroll
  for (int h = 0; h < H; ++h)
    if (jm / 64 == h) at = av[h];
  const double sgn = (bcast(at, jm % 64) < 0.0) ? -1.0 : 1.0;
#pragma unroll
  for (int h = 0; h < H; ++h) {
    const int a = lane + 64 * h;
    if (a < M) {
      alpha_out[(int64_t)si * M + a] = av[h] * sgn;
      C_out[(int64_t)si * M + a] = cv[h] * sgn;
      reinterpret_cast<double2*>(actab)[(int64_t)si * M + a] =
          make_double2(av[h] * sgn, cv[h] * sgn);
    }
  }
}

// Partials of shift si: nblk per shift in shift order (3D), or, for the
// balanced 2D launch of NWV waves over SPS steps per shift (sps > 0), the
// pieces (w, si) of the waves w whose ranges meet the shift, at slots w + si.
__device__ __forceinline__ void partial_range(int si, int nS, int nblk, int sps, int nwv,
                                              int* first, int* count) {
  if (sps > 0) {
    const int64_t total = (int64_t)nS * sps;
    const int64_t R = (total + nwv - 1) / nwv;
    const int w0 = (int)(((int64_t)si * sps) / R);
    const int w1 = (int)(((int64_t)(si + 1) * sps - 1) / R);
    *first = w0 + si;
    *count = w1 - w0 + 1;
  } else {
    *first = si * nblk;
    *count = nblk;
  }
}

// WP: the window 2 WP - 1 of the Green's partial sums read (WP >= W); the
// sums of a wider window hold every offset of [0, W - 1]^d, so the radius-1
// tables can be formed from the radius-2 pass. WA: the window of the
// (alpha, C) pair table written (WA > W: the WA^d layout, (0, 0) outside the
// W window, so that rows of both radii read one layout).
template <int D, int W, int WP = W, int WA = W>
__device__ __forceinline__ void null_body(
    NullShared<D, W>& sh, int si, const int* __restrict__ nS, const double* __restrict__ part,
    int nblk, int sps, int nwv, double invN, double* gtab, double* gamtab, double* Mtab,
    double* alpha_out, double* C_out, double* sigma_out, double* rho_out, double* actab,
    int* status, int* clear_counter) {
  using Pa = Parity<D, W>;
  using Nb = Nbhd<D, W>;
  static_assert(WP >= W, "the partial sums must cover the window");
  constexpr int NC = 1 << D;
  constexpr int WD = Pow<D, W>::v;
  constexpr int M = WD;
  // layout of the partial sums (window WP): pairs da <= db, per leading
  // offset in 3D, g then g * g
  constexpr int NP = WP * (WP + 1) / 2;
  constexpr int WO2 = Pow<D - 2, WP>::v;
  constexpr int NV = 2 * WO2 * NP;
  constexpr int T = 64 * NC;
  if (si == 0 && threadIdx.x == 0 && clear_counter) *clear_counter = 0;
  const int nSv = *nS;
  if (si >= nSv) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wid = tid >> 6;

  // ---- sum the partial sums of the Green's kernels (staged through LDS) ----
  // Thread (grp, v) = (tid / NVP, tid % NVP) adds the partials of value v from
  // work units b = grp, grp + G, ... in increasing b; then thread v adds the G
  // group sums in group order (a fixed order, so the result is deterministic).
  constexpr int NVP = (NV <= 32) ? 32 : (NV <= 64) ? 64 : 256;
  constexpr int G = T / NVP;
  static_assert(NV <= NVP && G >= 1 && T % NVP == 0, "partial-sum groups");
  int pfirst = 0, pcount = 0;
  partial_range(si, nSv, nblk, sps, nwv, &pfirst, &pcount);
  const double* ps = part + (int64_t)pfirst * NV;
  const int gv = tid % NVP, grp = tid / NVP;
  double acc = 0.0;
  const int total = pcount * NV;
  constexpr int CHUNK = 4096;
  for (int c0 = 0; c0 < total; c0 += CHUNK) {
    const int cn = min(CHUNK, total - c0);
    // every load of a thread is issued before any is consumed
    constexpr int PER = CHUNK / T;
    double tmp[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + u * T;
      tmp[u] = (e < cn) ? ps[c0 + e] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + u * T;
      if (e < cn) sh.stage[e] = tmp[u];
    }
    __syncthreads();
    if (gv < NV) {
      // units of this chunk holding value gv: global index b*NV + gv
      const int b_first = c0 / NV, b_end = (c0 + cn + NV - 1) / NV;
      int b = b_first + ((grp - b_first % G) + G) % G;
      for (; b < b_end; b += G) {
        const int e = b * NV + gv;
        if (e >= c0 && e < c0 + cn) acc += sh.stage[e - c0];
      }
    }
    __syncthreads();
  }
  sh.stage[grp * NVP + gv] = acc;
  __syncthreads();
  double tot = 0.0;
  if (tid < NV) {
#pragma unroll
    for (int q = 0; q < G; ++q) tot += sh.stage[q * NVP + tid];
  }
  __syncthreads();
  // symmetrised pair sums -> full tables, scaled by 1/N
  if (tid < NV) sh.stage[tid] = tot;
  __syncthreads();
  for (int e = tid; e < WD; e += T) {
    const int db0 = e % W;
    const int da0 = (e / W) % W;
    const int x = (D == 3) ? e / (W * W) : 0;
    const int da = min(da0, db0), db = max(da0, db0);
    const int pi = da * WP - (da * (da - 1)) / 2 + (db - da);
    const double gval = sh.stage[x * NP + pi] * invN;
    const double qval = sh.stage[WO2 * NP + x * NP + pi] * invN;
    sh.g[e] = gval;
    sh.q[e] = qval;
    gtab[(int64_t)si * WD + e] = gval;
    gamtab[(int64_t)si * WD + e] = qval;
  }
  __syncthreads();

  // ---- one parity class per wave ----
  double* Mtab_si = Mtab + (int64_t)si * M * M;
  switch (wid) {
    case 0: solve_class<D, W, 0>(sh, lane, si, Mtab_si); break;
    case 1: solve_class<D, W, 1>(sh, lane, si, Mtab_si); break;
    case 2: solve_class<D, W, 2>(sh, lane, si, Mtab_si); break;
    case 3: solve_class<D, W, 3>(sh, lane, si, Mtab_si); break;
    default:
      // waves w and w + 4 share a SIMD. Class sizes by index are 27, 18,
      // 18, 12, 18, 12, 12, 8 for t = 2 (8, 4, 4, 2, 4, 2, 2, 1 for t = 1):
      // waves 4-7 take classes 7-4, so the largest class shares its SIMD
      // with the smallest instead of an 18-row one
      if constexpr (D == 3) {
        switch (wid) {
          case 4: solve_class<D, W, 7>(sh, lane, si, Mtab_si); break;
          case 5: solve_class<D, W, 6>(sh, lane, si, Mtab_si); break;
          case 6: solve_class<D, W, 5>(sh, lane, si, Mtab_si); break;
          case 7: solve_class<D, W, 4>(sh, lane, si, Mtab_si); break;
        }
      }
      break;
  }
  __syncthreads();

  // ---- pick the class, map back to mu_0^t, normalise the sign ----
  // (every wave reaches the barrier below; only wave 0 writes results)
  int cs = 0;
  for (int c = 1; c < NC; ++c)
    if (sh.lam[c] < sh.lam[cs]) cs = c;
  const double lam = sh.lam[cs];
  if constexpr (M > 64) {
    map_back_wide<D, W>(sh, cs, wid, lane, si, alpha_out, C_out, actab);
  } else {
  double av = 0.0, cv = 0.0;
  if (wid == 0 && lane < M) {
    // offset a = lane: block row and coefficient of a in class cs
    double coef = 1.0;
    int pidx = 0;
    for (int i = 0; i < D; ++i) {
      const int xi = Nb::comp(lane, i);
      const int ji = xi < 0 ? -xi : xi;
      const int odd = Pa::odd(cs, i);
      if (odd && ji == 0) coef = 0.0;
      if (ji != 0) coef *= (odd && xi < 0) ? -lsp::kInvSqrt2 : lsp::kInvSqrt2;
      pidx = pidx * Pa::count(cs, i) + (ji - odd < 0 ? 0 : ji - odd);
    }
    if (coef != 0.0) {
      av = coef * sh.vec[cs][pidx];
      cv = coef * sh.gv[cs][pidx];
    }
  }
  if (wid != 0) return;
  // largest |alpha| over the lanes, lowest offset on ties (wave reduction)
  double am = (lane < M) ? fabs(av) : -1.0;
  int jm = lane;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double ao = __shfl_xor(am, o);
    const int jo = __shfl_xor(jm, o);
    if (ao > am || (ao == am && jo < jm)) {
      am = ao;
      jm = jo;
    }
  }
  const double sgn = (bcast(av, jm) < 0.0) ? -1.0 : 1.0;
  if (lane < M) {
    av *= sgn;
    cv *= sgn;
    alpha_out[(int64_t)si * M + lane] = av;
    C_out[(int64_t)si * M + lane] = cv;
    if constexpr (WA == W)
      reinterpret_cast<double2*>(actab)[(int64_t)si * M + lane] = make_double2(av, cv);
  }
  if constexpr (WA != W) {
    // entry k of the WA^d layout (lane k + 64 h writes it) takes offset src
    // of the W^d layout (same digit order, last axis fastest), or (0, 0)
    static_assert(WA > W && (WA - W) % 2 == 0, "a wider, centred window");
    constexpr int MA = Pow<D, WA>::v;
    constexpr int dt = (WA - W) / 2;
#pragma unroll
    for (int h = 0; h < (MA + 63) / 64; ++h) {
      const int k = lane + 64 * h;
      int rem = k, src = 0, mul = 1;
      bool in = k < MA;
#pragma unroll
      for (int i = 0; i < D; ++i) {
        const int oi = rem % WA - dt;
        rem /= WA;
        in = in && oi >= 0 && oi < W;
        src += oi * mul;
        mul *= W;
      }
      if (!in) src = 0;
      const double a = __shfl(av, src), c = __shfl(cv, src);
      if (k < MA)
        reinterpret_cast<double2*>(actab)[(int64_t)si * MA + k] =
            in ? make_double2(a, c) : make_double2(0.0, 0.0);
    }
  }
  }
  if (wid != 0) return;
  if (lane == 0) {
    sigma_out[si] = sqrt(fmax(lam, 0.0));
    // rho*(s)^2 = alpha^T M alpha / alpha^T A1 alpha, alpha = Q x of the class
    rho_out[si] = sqrt(fmax(lam, 0.0) / sh.ax[cs]);
    status[si] = sh.status[cs];
  }
}

template <int D, int W>
__global__ __launch_bounds__(64 * (1 << D)) void null_vector_kernel(
    const int* __restrict__ nS, const double* __restrict__ part, int nblk, int sps, int nwv,
    double invN, double* gtab, double* gamtab, double* Mtab, double* alpha_out, double* C_out,
    double* sigma_out, double* rho_out, double* actab, int* status, int* clear_counter) {
  __shared__ NullShared<D, W> sh;
  null_body<D, W>(sh, blockIdx.x, nS, part, nblk, sps, nwv, invN, gtab, gamtab, Mtab, alpha_out,
                  C_out, sigma_out, rho_out, actab, status, clear_counter);
}

// one launch for the problems of a batch: block b solves shift map[b].y of
// problem map[b].x
template <int D, int W>
__global__ __launch_bounds__(64 * (1 << D)) void null_batched_kernel(const lsp::BatchRec* recs,
                                                                     const int4* map) {
  const int4 it = map[blockIdx.x];
  const lsp::BatchRec& r = recs[it.x];
  __shared__ NullShared<D, W> sh;
  null_body<D, W>(sh, it.y, r.nS, r.part, r.nunits, r.sps, r.gwaves, r.invN, r.gtab, r.gamtab,
                  r.Mtab, r.alpha, r.Ctab, r.sigma, r.rho, r.actab, r.status, nullptr);
}

// Both radii of the per-point-radius setup from one radius-2 Green's pass:
// blocks 0 .. nreq-1 solve radius 2 into the problem's tables, blocks
// nreq .. 2 nreq - 1 radius 1 into the tables of t1. The two parts share one
// LDS area.
struct NullOut {
  double *gtab, *gamtab, *Mtab, *alpha, *C, *sigma, *rho, *actab;
  int* status;
};

template <int D>
__global__ __launch_bounds__(64 * (1 << D)) void null_nd_kernel(
    const int* __restrict__ nS, const double* __restrict__ part, int nblk, int sps, int nwv,
    double invN, int nreq, NullOut t2, NullOut t1) {
  constexpr size_t B5 = sizeof(NullShared<D, 5>), B3 = sizeof(NullShared<D, 3>);
  __shared__ __align__(16) unsigned char raw[B5 > B3 ? B5 : B3];
  if ((int)blockIdx.x < nreq) {
    null_body<D, 5>(*reinterpret_cast<NullShared<D, 5>*>(raw), blockIdx.x, nS, part, nblk, sps,
                    nwv, invN, t2.gtab, t2.gamtab, t2.Mtab, t2.alpha, t2.C, t2.sigma, t2.rho,
                    t2.actab, t2.status, nullptr);
  } else {
    null_body<D, 3, 5, 5>(*reinterpret_cast<NullShared<D, 3>*>(raw), blockIdx.x - nreq, nS,
                          part, nblk, sps, nwv, invN, t1.gtab, t1.gamtab, t1.Mtab, t1.alpha,
                          t1.C, t1.sigma, t1.rho, t1.actab, t1.status, nullptr);
  }
}

template <int D, int W>
hipError_t run_null(const lsp_problem* p, int num_shifts, int* clear_counter) {
  const double invN = 1.0 / (double)p->N;
  const int sps = (D == 2) ? lsp::green2d_sps(p->n) : 0;
  const int nwv = (D == 2) ? lsp::green2d_waves(p->n, num_shifts, p->tune[LSP_TUNE_GREEN_WAVES]) : 0;
  hipLaunchKernelGGL((null_vector_kernel<D, W>), dim3(num_shifts), dim3(64 * (1 << D)), 0,
                     p->stream, p->ws.nS, p->ws.green_part, p->green_nunits, sps, nwv, invN,
                     p->ws.gtab, p->ws.gamtab, p->ws.Mtab, p->ws.alpha, p->ws.Ctab, p->ws.sigma,
                     p->ws.rho, p->ws.actab, p->ws.status, clear_counter);
  return hipGetLastError();
}

}  // namespace

namespace lsp {

hipError_t launch_null_batched(int d, int t, const BatchRec* recs, const int4* map, int blocks,
                               hipStream_t s) {
  const int W = 2 * t + 1;
#define LSP_NULL_B(D_, W_)                                                                  \
  if (d == D_ && W == W_) {                                                                 \
    hipLaunchKernelGGL((null_batched_kernel<D_, W_>), dim3(blocks), dim3(64 * (1 << D_)), 0, \
                       s, recs, map);                                                       \
    return hipGetLastError();                                                               \
  }
  LSP_NULL_B(2, 3)
  LSP_NULL_B(2, 5)
  LSP_NULL_B(2, 7)
  LSP_NULL_B(3, 3)
#undef LSP_NULL_B
  return hipErrorInvalidValue;
}

hipError_t launch_null_nd(lsp_problem* p, int num_shifts, const NdTables1& t1) {
  if (p->t != 2 || (p->d != 2 && p->d != 3)) return hipErrorInvalidValue;
  const double invN = 1.0 / (double)p->N;
  const int sps = (p->d == 2) ? lsp::green2d_sps(p->n) : 0;
  const int nwv = (p->d == 2) ? lsp::green2d_waves(p->n, num_shifts, p->tune[LSP_TUNE_GREEN_WAVES]) : 0;
  const NullOut o2{p->ws.gtab, p->ws.gamtab, p->ws.Mtab, p->ws.alpha, p->ws.Ctab,
                   p->ws.sigma, p->ws.rho, p->ws.actab, p->ws.status};
  const NullOut o1{t1.gtab, t1.gamtab, t1.Mtab, t1.alpha, t1.C,
                   t1.sigma, t1.rho, reinterpret_cast<double*>(t1.actab), t1.status};
  const dim3 grid(2 * num_shifts), block(64 * (1 << p->d));
  if (p->d == 2)
    hipLaunchKernelGGL(null_nd_kernel<2>, grid, block, 0, p->stream, p->ws.nS, p->ws.green_part,
                       p->green_nunits, sps, nwv, invN, num_shifts, o2, o1);
  else
    hipLaunchKernelGGL(null_nd_kernel<3>, grid, block, 0, p->stream, p->ws.nS, p->ws.green_part,
                       p->green_nunits, sps, nwv, invN, num_shifts, o2, o1);
  return hipGetLastError();
}

hipError_t launch_null_vectors(lsp_problem* p, int num_shifts, int* clear_counter) {
  const int W = 2 * p->t + 1;
  if (p->d == 2 && W == 3) return run_null<2, 3>(p, num_shifts, clear_counter);
  if (p->d == 2 && W == 5) return run_null<2, 5>(p, num_shifts, clear_counter);
  if (p->d == 2 && W == 7) return run_null<2, 7>(p, num_shifts, clear_counter);
  if (p->d == 3 && W == 3) return run_null<3, 3>(p, num_shifts, clear_counter);
  if (p->d == 3 && W == 5) return run_null<3, 5>(p, num_shifts, clear_counter);
  return hipErrorInvalidValue;
}

// Dense orthonormal basis of parity class c as an m x b matrix (column p =
// basis vector p in the offsets of mu_0^t); used on the host to expand the
// packed Gram blocks back to the full m x m matrix.
template <int D, int W>
void parity_basis_host(int c, double* Q) {
  using Pa = Parity<D, W>;
  using Nb = Nbhd<D, W>;
  const int M = Pow<D, W>::v;
  const int B = Pa::size(c);
  for (int i = 0; i < M * B; ++i) Q[i] = 0.0;
  for (int a = 0; a < M; ++a) {
    double coef = 1.0;
    int pidx = 0;
    for (int i = 0; i < D; ++i) {
      const int xi = Nb::comp(a, i);
      const int ji = xi < 0 ? -xi : xi;
      const int odd = Pa::odd(c, i);
      if (odd && ji == 0) coef = 0.0;
      if (ji != 0) coef *= (odd && xi < 0) ? -kInvSqrt2 : kInvSqrt2;
      pidx = pidx * Pa::count(c, i) + (ji - odd < 0 ? 0 : ji - odd);
    }
    if (coef != 0.0) Q[a * B + pidx] = coef;
  }
}

// M_full = sum_c Q_c M_c Q_c^T from the packed blocks.
int expand_gram_host(int d, int t, const double* packed, double* full) {
  const int W = 2 * t + 1;
  int M = 1;
  for (int i = 0; i < d; ++i) M *= W;
  for (int i = 0; i < M * M; ++i) full[i] = 0.0;
  std::vector<double> Q;
  int off = 0;
  for (int c = 0; c < (1 << d); ++c) {
    int B = 1;
    for (int i = 0; i < d; ++i) B *= ((c >> (d - 1 - i)) & 1) ? t : t + 1;
    Q.assign((size_t)M * B, 0.0);
    if (d == 2 && W == 3) parity_basis_host<2, 3>(c, Q.data());
    else if (d == 2 && W == 5) parity_basis_host<2, 5>(c, Q.data());
    else if (d == 2 && W == 7) parity_basis_host<2, 7>(c, Q.data());
    else if (d == 3 && W == 3) parity_basis_host<3, 3>(c, Q.data());
    else if (d == 3 && W == 5) parity_basis_host<3, 5>(c, Q.data());
    else return -1;
    const double* Mc = packed + off;
    for (int a = 0; a < M; ++a)
      for (int b = 0; b < M; ++b) {
        double s = 0.0;
        for (int pp = 0; pp < B; ++pp) {
          const double qa = Q[(size_t)a * B + pp];
          if (qa == 0.0) continue;
          for (int qq = 0; qq < B; ++qq) s += qa * Mc[pp * B + qq] * Q[(size_t)b * B + qq];
        }
        full[(size_t)a * M + b] += s;
      }
    off += B * B;
  }
  return 0;
}

}  // namespace lsp
