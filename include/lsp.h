/*
 * lsp.h -- C ABI of liblsp, the MI355X (gfx950) hot path of the localized
 * sparsifying preconditioner (F. Liu and L. Ying, arXiv 1607.02560) for the
 * periodic pseudospectral system (L + diag v) u = f on [0,1)^d.
 *
 * Notation follows the paper: d dimensions, n points per axis, h = 1/n,
 * N = n^d unknowns on the grid J = {0..n-1}^d (Sec. 2). Grid arrays are in
 * C order: point j = (j_1, ..., j_d) is stored at flat index
 * ((j_1 n + j_2) n + ...) + j_d, the last axis fastest.
 * Complex arrays are complex128, interleaved (re, im) doubles.
 *
 * Memory: every pointer named *_dev is device memory on the current HIP
 * device, owned by the caller; the library never frees it and never keeps it
 * past the call (the potential is copied). Pointers named *_host are host
 * memory. All device work is ordered on the stream given to lsp_create and
 * the calls return without waiting for it unless stated otherwise. One
 * problem object must not be used from two threads at once; separate
 * objects are independent.
 *
 * Errors: every int-returning call returns LSP_OK (0) on success, a negative
 * LSP_E* code when nothing was computed, or a positive warning code.
 * Arguments are validated on the host before any launch. lsp_last_error()
 * returns a message describing the last failure on the calling thread.
 */
#ifndef LSP_H
#define LSP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  LSP_OK = 0,
  LSP_NOT_CONVERGED = 1, /* GMRES stopped at maxit; outputs hold the last iterate */
  LSP_EINVAL = -1,       /* invalid argument (dimension, size, radius, pointer) */
  LSP_ENONFINITE = -2,   /* NaN or Inf in the potential or right-hand side */
  LSP_ERESONANT = -3,    /* a shift makes L + s singular (Sec. 3) */
  LSP_ENOMEM = -4,       /* device or host allocation failed */
  LSP_EHIP = -5,         /* a HIP runtime call failed */
  LSP_ESOLVER = -6,      /* the host P-solve callback reported failure */
  LSP_ESTATE = -7        /* call order violated (e.g. apply before setup) */
};

/* Storage precision of the P rows written by lsp_stencil_setup. Every step of
 * the setup computes in FP64 in both modes (shift list, Green's sums, Gram
 * matrix, null vectors, assignment, P-row formula). LSP_FP32_REFINE stores
 * each P entry rounded once to float32 (half the bytes of the dominant write);
 * the FP64 Krylov iteration around the preconditioner refines the solution. */
enum { LSP_FP64 = 0, LSP_FP32_REFINE = 1 };

typedef struct lsp_problem lsp_problem;

/* Host callback solving P x = rhs for the sparse matrix P of eq. (PC).
 * rhs and x are complex128 interleaved host arrays of N entries.
 * Returns 0 on success; any other value aborts the solve with LSP_ESOLVER. */
typedef int (*lsp_host_solve_fn)(void* user, const double* rhs_host, double* x_host, int64_t N);

/* Human-readable name of a status code. */
const char* lsp_strerror(int code);

/* Message of the last failure on the calling thread ("" if none). */
const char* lsp_last_error(void);

/* Library version string. */
const char* lsp_version(void);

/*
 * Create a problem for (L + diag v) u = f on the grid J (Sec. 2).
 *   d       2 or 3.
 *   n       points per axis: a power of two, 8 <= n <= 1024 for d = 2 and
 *           8 <= n <= 256 for d = 3.
 *   v_dev   N float64 potential samples v_j = v(h j) (Sec. 2), device memory;
 *           copied into the problem. Must be finite (else LSP_ENONFINITE).
 *   stream  hipStream_t on which every later call enqueues its work
 *           (NULL = the default stream).
 *   out     receives the new object; *out is NULL on failure.
 * Allocates the problem's device workspaces and synchronises the stream once
 * (to check the potential).
 */
int lsp_create(int d, int n, const double* v_dev, void* stream, lsp_problem** out);

/* Replace the potential (same d, n) with N float64 values from v_dev; the
 * shift tables built by an earlier setup are invalidated. Synchronises. */
int lsp_set_potential(lsp_problem* p, const double* v_dev);

/* Free the problem and its device memory. NULL is accepted. */
void lsp_destroy(lsp_problem* p);

/*
 * Stencil setup of the localized sparsifying preconditioner (Sec. 4.1-4.2):
 *   1. shift list S: num_shifts bin centres spread evenly over
 *      [v_min, v_max], each snapped to the nearest (4m+2) pi^2, duplicates
 *      removed (Sec. 4.1);
 *   2. for each s in S the Green's kernels g_s = G_s[:,0] and g_s * g_s
 *      (Sec. 3 and 4.2), evaluated at the offsets [-2t, 2t]^d only;
 *   3. the Gram matrix M = A1 - A2 of eq. (A) on the neighbourhood mu_0^t;
 *   4. alpha_s = unit eigenvector of the smallest eigenvalue of M (sign:
 *      largest-magnitude entry positive), sigma_min, and C_s = G_s[mu,mu] alpha_s;
 *   5. per grid point j: idx_j = index in S of the shift closest to v_j
 *      (ties to the lower index) and the P row
 *      P[j, a] = alpha_{s_j}[a] + C_{s_j}[a] (v[j+a] - s_j), a in mu_0^t.
 *   t           neighbourhood radius: t = 1, 2, 3 for d = 2 and t = 1, 2 for d = 3
 *               (m = (2t+1)^d up to 49 and 125), with 2t+1 < n and N >= 2m.
 *               The learned and batched setups take d = 3 only with t = 1.
 *   num_shifts  requested |S| (1..1024); 0 selects n/16 for d = 2, n/4 for d = 3
 *               (at least 1). The effective count |S| may be smaller.
 *   precision   LSP_FP64 (P in float64) or LSP_FP32_REFINE (P in float32,
 *               each entry the FP64 value rounded to nearest).
 *   P_dev       output, N*m entries of the precision's type; row j holds the
 *               m offsets of mu_0^t in lexicographic order over [-t,t]^d
 *               (last axis fastest); the column of entry (j, a) is
 *               (j + a) mod n per axis.
 *   idx_dev     output, N int32 shift indices (may be NULL).
 * Asynchronous: returns once the work is enqueued.
 */
int lsp_stencil_setup(lsp_problem* p, int t, int num_shifts, int precision,
                      void* P_dev, int32_t* idx_dev);

/*
 * Stencil setup of the non-localized sparsifying preconditioner (Sec. 3), the
 * method the localized one refines: one shift s for every grid point, the
 * average of v (so that q = v - s has zero mean). When L + s is singular
 * (x = -s / (4 pi^2) within 2^-30 max(1, |x|) of an integer K >= 0) s moves
 * to (2 - 4K) pi^2, the value of the form (4m+2) pi^2 that lies 2 pi^2 above
 * -4 pi^2 K. Then steps 2-4 of lsp_stencil_setup for that one
 * shift, idx_j = 0 and P[j, a] = alpha[a] + C[a] (v[j+a] - s), i.e.
 * P = Q + C diag(q) with Q's rows alpha. The mean is summed in a fixed order,
 * so repeated calls give identical results.
 *   t, precision, P_dev, idx_dev  as for lsp_stencil_setup (same layouts).
 * lsp_get_tables, lsp_c_apply and lsp_precond_solve then use this setup.
 * Asynchronous: returns once the work is enqueued.
 */
int lsp_stencil_setup_global(lsp_problem* p, int t, int precision, void* P_dev,
                             int32_t* idx_dev);

/*
 * Stencil setup with the per-point radius of Sec. 4.2 (Fig. 3): point j uses
 * radius t_j, the largest that keeps the sparsity nested dissection with
 * leaf box `leaf` needs, capped at 2. Separators are the grid planes
 * j_i = 0 mod leaf; a vertex (every coordinate on a separator) may reach
 * t = leaf, any other point reaches up to the nearest separator plane across
 * its coordinates off the separators. The shift list, s_j and the radius-2
 * tables are those of lsp_stencil_setup with t = 2; the radius-1 tables come
 * from the same Green's sums (their values at offsets [0,2]^d), so they equal
 * those of lsp_stencil_setup with t = 1 up to the order of summation.
 *   leaf        leaf box size b >= 2, dividing n (Sec. 5 uses 8).
 *   num_shifts  as for lsp_stencil_setup.
 *   P_dev       output, N*5^d float64 in the layout of radius 2 (the offsets
 *               of mu_0^2, lexicographic, last axis fastest); a row with
 *               t_j = 1 holds its radius-1 stencil on mu_0^1 and zeros on the
 *               other offsets.
 *   idx_dev     output, N int32 shift indices (may be NULL).
 * Needs 2t+1 = 5 < n. lsp_c_apply and lsp_precond_solve then use the rows
 * C[j, mu_j^{t_j}] of this setup (read from the tables of each point's
 * radius); lsp_get_tables returns the radius-2 tables, lsp_get_tables_nd1
 * the radius-1 tables.
 * Launches directly (no graph). Asynchronous.
 */
int lsp_stencil_setup_nd(lsp_problem* p, int leaf, int num_shifts, double* P_dev,
                         int32_t* idx_dev);

/*
 * Pseudospectral apply y = (L + diag v) u with L = F^-1 diag(4 pi^2 |k|^2) F
 * (Sec. 2, eq. dmodel). u_dev and y_dev: N complex128, device, must not
 * overlap. Asynchronous.
 */
int lsp_ps_apply(lsp_problem* p, const double* u_dev, double* y_dev);

/*
 * First half of the preconditioner P^-1 C of eq. (PC): z = C r with
 * (C r)_j = sum_a C_{s_j}[a] r[(j + a) mod n]. Needs a completed setup.
 * r_dev, z_dev: N complex128, device, must not overlap. Asynchronous.
 */
int lsp_c_apply(lsp_problem* p, const double* r_dev, double* z_dev);

/*
 * Solve (L + diag v) u = f by GMRES(restart) with right preconditioner
 * P^-1 C (eq. PC; Sec. 5 uses restart 40). The P-solve is done on the host
 * by solveP (a sparse factorisation of the P rows from the last setup); every
 * other step runs on the device. x0 = 0; stops when the Arnoldi residual
 * estimate is <= rtol ||f||. f_dev, u_dev: N complex128 device arrays.
 * iters receives the number of Arnoldi steps, relres the true relative
 * residual ||f - A u|| / ||f|| (recomputed at the end). Synchronous.
 * Returns LSP_NOT_CONVERGED (with u the last iterate) if maxit is reached.
 */
int lsp_precond_solve(lsp_problem* p, const double* f_dev, double* u_dev,
                      double rtol, int restart, int maxit,
                      lsp_host_solve_fn solveP, void* user,
                      int* iters, double* relres);

/*
 * Nested-dissection factors of P (Sec. 3, Fig. 1) for the device P-solve of
 * eq. (PC): a multifrontal LU of P computed on the host (the factorisation is
 * a host step; the solve with its factors runs every Krylov iteration, the
 * T_NDapp term of Table 1). Fronts k = 0..nfronts-1 are in elimination order;
 * front k eliminates the grid points F_k (a box interior or a separator
 * piece, f[k] >= 1 of them) and couples to the later points U_k (u[k] >= 0).
 * Every array is host memory (int64 or float64), read only during
 * lsp_psolve_upload and not kept:
 *   f, u            [nfronts] sizes of F_k and U_k
 *   off_F, off_U    [nfronts+1] prefix sums of f and u (off_F[nfronts] = N,
 *                   off_U[nfronts] = nidx_U)
 *   idx_F           [N] the F_k concatenated (flat grid indices)
 *   idx_Fp          [N] the same with each front's row pivoting applied
 *                   (the row of P that pivot row i of front k came from)
 *   idx_U           [nidx_U] the U_k concatenated
 *   off_blk         [4*nfronts] offsets into data of front k's dense
 *                   row-major blocks: L_FF^-1 (f x f, inverse of the unit
 *                   lower factor), L_UF L_FF^-1 (u x f), U_FF^-1 (f x f),
 *                   U_FF^-1 U_FU (f x u)
 *   data            [ndata] the dense blocks
 *   upd_ptr         [N+1], upd_pos [nidx_U]: for grid point i, the entries
 *                   upd_pos[upd_ptr[i] .. upd_ptr[i+1]) are the positions in
 *                   the concatenated U lists that name i, in front order
 *   lev_ptr         [nlevels+1], lev_fronts [nfronts]: fronts grouped into
 *                   levels of mutually independent fronts (one merge step of
 *                   the boxes each); lev_fronts must list 0..nfronts-1 in
 *                   order, so each level is a consecutive range of fronts
 */
typedef struct lsp_nd_factors {
  int64_t nfronts, nlevels, nidx_U, ndata;
  const int64_t *f, *u, *off_F, *off_U, *idx_F, *idx_Fp, *idx_U, *off_blk;
  const double* data;
  const int64_t *upd_ptr, *upd_pos, *lev_ptr, *lev_fronts;
} lsp_nd_factors;

/*
 * Copy the factors to the device (replacing any earlier upload) and
 * precompute the per-level product lists. Every offset, size and index is
 * checked on the host first (LSP_EINVAL: nothing uploaded, an earlier upload
 * stays in place); LSP_ENOMEM or LSP_EHIP if a device allocation or copy
 * fails (then no factors are left). The device copy is owned by the problem and freed
 * by the next upload or lsp_destroy. Synchronous.
 */
int lsp_psolve_upload(lsp_problem* p, const lsp_nd_factors* fac);

/*
 * z = P^-1 r with the uploaded factors: level by level, a forward pass
 * (gather of the right-hand side and of the updates earlier fronts sent,
 * then y_F = L_FF^-1 r_F and the updates (L_UF L_FF^-1) r_F) and a backward
 * pass (x_F = U_FF^-1 y_F - (U_FF^-1 U_FU) x_U), one launch per level and
 * pass. Every sum runs in a fixed order, so the result is deterministic. r_dev, z_dev: N complex128 device arrays,
 * must not overlap. LSP_ESTATE without an upload. Asynchronous.
 */
int lsp_psolve_apply(lsp_problem* p, const double* r_dev, double* z_dev);

/*
 * lsp_precond_solve with every step on the device: GMRES(restart) with the
 * right preconditioner P^-1 C (eq. PC), C from the last setup and P^-1 from
 * lsp_psolve_upload. One Arnoldi step (C-apply, P-solve, pseudospectral
 * apply, classical Gram-Schmidt twice with fixed-order two-stage reductions,
 * Givens rotation of the new Hessenberg column) is a sequence of device
 * launches, replayed from a HIP graph captured once per column k unless
 * LSP_GRAPHS=0; the host reads one residual estimate per step to decide
 * whether to stop. Arguments, x0 = 0, the stopping rule and the outputs are
 * those of lsp_precond_solve. Synchronous.
 */
int lsp_precond_solve_device(lsp_problem* p, const double* f_dev, double* u_dev, double rtol,
                             int restart, int maxit, int* iters, double* relres);

/*
 * Host copies of the per-shift tables of the last setup. Synchronises.
 * Any pointer may be NULL. Sizes: S_host[nS], alpha_host[nS*m], C_host[nS*m],
 * sigma_host[nS], g_host[nS*(2t+1)^d], gam_host[nS*(2t+1)^d] (g_s and
 * g_s * g_s at offsets [0,2t]^d, lexicographic), M_host[nS*m*m].
 * Pass capacity = the number of shifts the arrays can hold; returns
 * LSP_EINVAL if it is smaller than the effective |S| (which is stored in *nS
 * in every case).
 */
int lsp_get_tables(lsp_problem* p, int capacity, int* nS, double* S_host,
                   double* alpha_host, double* C_host, double* sigma_host,
                   double* g_host, double* gam_host, double* M_host);

/*
 * Host copies of the radius-1 tables of the last per-point-radius setup
 * (lsp_stencil_setup_nd; the radius-2 tables are those of lsp_get_tables):
 * alpha_host[nS*3^d], C_host[nS*3^d] (offsets of mu_0^1), sigma_host[nS],
 * g_host[nS*3^d], gam_host[nS*3^d] (g_s and g_s * g_s at offsets [0,2]^d,
 * lexicographic). Any pointer may be NULL. LSP_ESTATE if the last setup was
 * not a per-point-radius setup; LSP_EINVAL if capacity < |S| (stored in
 * *nS in every case). Synchronises.
 */
int lsp_get_tables_nd1(lsp_problem* p, int capacity, int* nS, double* alpha_host,
                       double* C_host, double* sigma_host, double* g_host, double* gam_host);

/* Default shift-list size used when lsp_stencil_setup gets num_shifts = 0:
 * n/16 for d = 2 and n/4 for d = 3, at least 1 (the ratios of Tables 2-9,
 * Sec. 5). Host only; returns LSP_EINVAL for d outside {2, 3} or n < 1. */
int lsp_default_num_shifts(int d, int n);

/*
 * Per-stage timing with HIP events on the problem's stream (for measurement;
 * off by default). Stages: LSP_STAGE_SHIFTS (min/max of v for the shift
 * list), LSP_STAGE_GREEN (shift list and Green's kernel sums), LSP_STAGE_NULL (Gram matrix and null vector),
 * LSP_STAGE_ASSEMBLE (per-point rows; for lsp_stencil_setup_learned the
 * network, check and rows), LSP_STAGE_SETUP (the whole lsp_stencil_setup or
 * lsp_stencil_setup_learned), LSP_STAGE_APPLY (lsp_ps_apply), LSP_STAGE_CAPPLY
 * (lsp_c_apply), LSP_STAGE_PSOLVE (lsp_psolve_apply), LSP_STAGE_ARNOLDI (one
 * Arnoldi step of lsp_precond_solve_device, graph replay included).
 * lsp_profile(p, 1) starts recording and clears the totals; lsp_profile(p, 0)
 * stops. lsp_profile_read synchronises the stream and writes, for each stage
 * s < nstages, the summed milliseconds ms_host[s] and the number of timed
 * calls count_host[s] since recording started.
 */
enum {
  LSP_STAGE_SHIFTS = 0,
  LSP_STAGE_GREEN = 1,
  LSP_STAGE_NULL = 2,
  LSP_STAGE_ASSEMBLE = 3,
  LSP_STAGE_SETUP = 4,
  LSP_STAGE_APPLY = 5,
  LSP_STAGE_CAPPLY = 6,
  LSP_STAGE_PSOLVE = 7,
  LSP_STAGE_ARNOLDI = 8,
  LSP_NUM_STAGES = 9
};
int lsp_profile(lsp_problem* p, int enable);
int lsp_profile_read(lsp_problem* p, int nstages, double* ms_host, int* count_host);

/*
 * Launch-shape tuning (not in the paper). Three shapes of this problem's
 * kernels can be chosen per problem; 0 selects the built-in default:
 *   LSP_TUNE_GREEN_WAVES    2D: the most waves of the Green's-sum launch
 *                           (512, 1024, 1536, 2048 or 3072);
 *   LSP_TUNE_ASSEMBLY_TILE  2D, n >= 128: the assembly's tile, 32, 64 or 128
 *                           points of one row, or 1 for 4 x 128 tiles with
 *                           the shift tables staged in LDS;
 *   LSP_TUNE_APPLY_FORM     n = 256, 512, 1024: the apply's line transform
 *                           with 8 or 16 values per thread.
 * The assembly tile does not change any result; the Green's wave count and
 * the apply form change the order of summation (results agree to rounding).
 * lsp_autotune runs the setup (t, num_shifts, precision, P_dev as for
 * lsp_stencil_setup) and the apply (u_dev to y_dev, N complex128 each) with
 * every candidate of each shape in turn, reps timed calls each (HIP events on
 * the problem's stream), keeps the fastest, and writes the choices to
 * choice_host[LSP_TUNE_COUNT] and the chosen mean times (ms: setup, setup,
 * apply) to ms_host[LSP_TUNE_COUNT] (either may be NULL). The setup's outputs
 * then hold the last candidate's results. Synchronous.
 * lsp_set_tuning sets the choices directly (LSP_EINVAL for a value outside
 * the lists above); lsp_get_tuning reads them.
 */
enum {
  LSP_TUNE_GREEN_WAVES = 0,
  LSP_TUNE_ASSEMBLY_TILE = 1,
  LSP_TUNE_APPLY_FORM = 2,
  LSP_TUNE_COUNT = 3
};
int lsp_autotune(lsp_problem* p, int t, int num_shifts, int precision, void* P_dev,
                 const double* u_dev, double* y_dev, int reps, int* choice_host,
                 double* ms_host);
int lsp_set_tuning(lsp_problem* p, const int* choice_host);
int lsp_get_tuning(const lsp_problem* p, int* choice_host);

/* Number of stencil entries m = (2t+1)^d of the last setup (0 before setup). */
int lsp_stencil_size(const lsp_problem* p);

/*
 * Column pattern of P and C for radius t: col_host[j*m + a] = flat index of
 * (j + a) mod n, a in mu_0^t lexicographic. N*m int64 host entries. The
 * CSR row pointer is j*m.
 */
int lsp_export_pattern(int d, int n, int t, int64_t* col_host);

/*
 * Stencil setup that allocates nothing, for callers that cannot allocate:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc. The same setup as lsp_stencil_setup (same kernels, bit-identical
 * P rows and shift indices) for a 2D problem, without a problem object:
 *   d, n        d must be 2; n a power of two in [8, 1024].
 *   v_dev       N float64 potential samples (device), read in place: not
 *               copied and not checked (it must be finite).
 *   t, num_shifts, precision, P_dev, idx_dev  as for lsp_stencil_setup
 *               (t = 1, 2, 3).
 *   stream      hipStream_t for the launches (NULL = default stream).
 * Every intermediate (shift-list partials, cosine table, Green's partial
 * sums, per-shift tables) lives in one fixed device array of the library,
 * lsp_static_scratch_bytes() bytes per GPU, held until the process ends; a
 * setup needing more (large |S| with t = 3 at n = 1024) returns LSP_EINVAL
 * before any launch. Calls no hipMalloc, hipFree or allocating routine on
 * success. All calls on one GPU share its array, which keeps the last call's
 * contents: calls that overlap on one GPU (different streams or threads)
 * race. The per-shift tables are not exported; lsp_c_apply and
 * lsp_precond_solve need a problem object. Asynchronous.
 */
int lsp_stencil_setup_static(int d, int n, const double* v_dev, int t, int num_shifts,
                             int precision, void* P_dev, int32_t* idx_dev, void* stream);

/* Bytes of the fixed device array of lsp_stencil_setup_static (per GPU). */
size_t lsp_static_scratch_bytes(void);

/* ------------------------------------------------------------------------
 * Learned stencils (a surrogate beside the method; not part of the paper).
 * A network with two hidden SiLU layers maps the m + 2 features of a grid
 * point (h^2 v_j, h^2 v[j + a] for a in mu_0^t, h = 1/n, and h^2 s_j for the
 * shift s_j of Sec. 4.1 nearest to v_j) to its 2m rows
 * (the P row of Sec. 4.1 and the C row of its shift, eq. (PC), times |s_j|).
 * Training and inference run in hand-written BF16 MFMA kernels with FP32
 * accumulation and FP32 master weights (Adam). Inputs and targets are
 * standardised per feature; the loss is the mean squared error of the
 * standardised outputs.
 * ------------------------------------------------------------------------ */
typedef struct lsp_mlp lsp_mlp;

/* Create a network with n_in inputs, n_hidden units per hidden layer (a
 * multiple of 16) and n_out outputs, taking batches of up to batch_rows
 * rows, on a HIP stream (NULL = default). Weights start at zero and the
 * standardisation at (0, 1): set both before use. */
int lsp_mlp_create(int n_in, int n_hidden, int n_out, int batch_rows, void* stream,
                   lsp_mlp** out);
void lsp_mlp_destroy(lsp_mlp* q);

/* Number of parameters: n_hidden (n_in + n_hidden + n_out + 2) + n_out. */
int lsp_mlp_num_params(const lsp_mlp* q);

/* Host FP32 parameters in the order W1 [n_hidden][n_in], b1, W2
 * [n_hidden][n_hidden], b2, W3 [n_out][n_hidden], b3 (row-major). Setting
 * them also resets the Adam state. */
int lsp_mlp_set_params(lsp_mlp* q, const float* params_host);
int lsp_mlp_get_params(lsp_mlp* q, float* params_host);

/* Standardisation, host FP32: mu_x [n_in], sd_x [n_in], mu_y [n_out],
 * sd_y [n_out] (deviations > 0). */
int lsp_mlp_set_normalisation(lsp_mlp* q, const float* norm_host);
int lsp_mlp_get_normalisation(lsp_mlp* q, float* norm_host);

/* Set the standardisation to the column means and deviations of X_dev
 * [rows][n_in] and T_dev [rows][n_out] (device FP32). */
int lsp_mlp_fit_normalisation(lsp_mlp* q, const float* X_dev, const float* T_dev, int rows);

/* Y_dev [rows][n_out] = de-standardised outputs for X_dev [rows][n_in]
 * (device FP32), rows <= batch_rows. Asynchronous. */
int lsp_mlp_forward(lsp_mlp* q, const float* X_dev, int rows, float* Y_dev);

/* Loss and gradients of one batch without updating: grad_host (may be NULL)
 * receives the gradients in the parameter order above, loss_host the loss.
 * Synchronous. */
int lsp_mlp_loss_grad(lsp_mlp* q, const float* X_dev, const float* T_dev, int rows,
                      float* grad_host, double* loss_host);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) on a batch
 * of rows <= batch_rows; loss_host (may be NULL) receives the batch loss
 * before the step (synchronises when given). */
int lsp_mlp_train_step(lsp_mlp* q, const float* X_dev, const float* T_dev, int rows, float lr,
                       double* loss_host);

/* Save the network (parameters, standardisation, Adam moments and step
 * count) to one file: a 64-byte header (magic "LSPMLP01", version 1, n_in,
 * n_hidden, n_out, Adam steps, parameter count, FNV-1a 64 checksum) and the
 * FP32 payload. Synchronous. LSP_EINVAL if the file cannot be written. */
int lsp_mlp_save(lsp_mlp* q, const char* path);

/* Create a network from a file written by lsp_mlp_save, taking batches of
 * up to batch_rows rows on a HIP stream (NULL = default); training resumes
 * where it stopped. LSP_EINVAL for a missing, truncated or corrupted file
 * (header or checksum mismatch). */
int lsp_mlp_load(const char* path, int batch_rows, void* stream, lsp_mlp** out);

/* Training rows of the points points_dev [count] (device int64 flat indices)
 * from a completed exact FP64 setup of p whose P rows are P_dev [N*m]:
 * X_dev [count][m+2] features, T_dev [count][2m] targets (device FP32).
 * Indices outside [0, N) give rows of NaN. Returns LSP_ESTATE without a
 * completed exact setup. */
int lsp_training_rows(lsp_problem* p, const double* P_dev, const int64_t* points_dev,
                      int count, float* X_dev, float* T_dev);

/* Learned setup: the shift tables of Sec. 4.1-4.2 as in lsp_stencil_setup,
 * then, for every point, the network's outputs p (P row) and c (C row),
 * which propose the stencil q = p - c (v[mu_j] - s_j) (the row of Q). The
 * stencil is checked with the exact Gram matrices of the point's shift:
 * rho = sqrt(q^T M q / q^T A1 q) (M = A1 - A2, eq. (A)) is the fraction of
 * the row of Q G that the truncation to mu drops (Sec. 3). The exact stencil
 * itself drops rho*(s) > 0 (about 0.05 for d = 3, t = 1), so the test is on
 * the excess. A kept point takes the rows its stencil defines,
 * C[j, mu_j] = (Q G)[j, mu_j] = G_mu,mu q and P = q + C (v[mu_j] - s_j)
 * (Sec. 4.1, eq. (PC)); a point with rho > rho*(s_j) + threshold (or a
 * non-finite output) takes the exact P and C rows (fallback_dev[j] = 1).
 *   P_dev         output, N*m float64 (layout of lsp_stencil_setup).
 *   fallback_dev  output, N int32 (1 = exact row used).
 *   n_fallback_host  receives the number of fallback rows; with NULL the call
 *                 returns without waiting for the GPU.
 * The per-point C rows stay with the problem; lsp_c_apply and
 * lsp_precond_solve use them until the next setup. The network's kernels
 * run on the problem's stream (work pending on the network's own stream is
 * waited for first); calls that use one network or one problem at the same
 * time from several threads race. Errors: LSP_EINVAL (NULL pointer,
 * threshold < 0 or NaN, a network without m + 2 inputs and 2m outputs, the
 * sizes of lsp_stencil_setup), LSP_ENOMEM, LSP_EHIP. Synchronous when
 * n_fallback_host is given, asynchronous on the problem's stream otherwise. */
int lsp_stencil_setup_learned(lsp_problem* p, lsp_mlp* mlp, int t, int num_shifts,
                              double threshold, double* P_dev, int32_t* fallback_dev,
                              int* n_fallback_host);

/* ------------------------------------------------------------------------
 * Batches (a form beside the plain method): many independent problems of
 * uneven n set up together with one launch per setup stage over the work
 * items of all of them, replayed as one HIP graph when the problems' stream
 * is not the legacy default stream (LSP_GRAPHS=0 launches directly).
 * ------------------------------------------------------------------------ */
typedef struct lsp_batch lsp_batch;

/* A batch over count problems created with lsp_create. They must share d,
 * the HIP stream and the device, and have n >= 16; the batch refers to them
 * (it does not own them) and must be destroyed before any of them. */
int lsp_batch_create(int count, lsp_problem* const* problems, lsp_batch** out);
void lsp_batch_destroy(lsp_batch* b);

/* lsp_stencil_setup (Sec. 4.1-4.2) of every problem of the batch with a
 * common t and precision: num_shifts[i] (NULL: the defaults), P_dev[i] (rows
 * of problem i, layout of lsp_stencil_setup), idx_dev (NULL, or NULL
 * entries, to skip s_j). Each problem receives exactly the tables and rows of
 * its own lsp_stencil_setup, and its per-problem entry points (C-apply,
 * GMRES, tables) use them afterwards. The first call for a set of sizes (and
 * t, precision) also times the assembly tile widths that divide every n and
 * keeps the fastest. Errors: those of lsp_stencil_setup for each problem,
 * LSP_EINVAL for NULL rows. Asynchronous on the batch's stream after the
 * first call for a set of arguments. */
int lsp_batch_stencil_setup(lsp_batch* b, int t, const int* num_shifts, int precision,
                            void* const* P_dev, int32_t* const* idx_dev);

/* y_i = (L + diag v_i) u_i (Sec. 2) for every problem i: u_dev[i], y_dev[i]
 * device complex128 of N_i entries. The problems may run concurrently, so no
 * y_dev[i] may overlap any u_dev[j] or another y_dev[j] (identical pointers
 * are refused with LSP_EINVAL; partial overlaps are not detected).
 * Asynchronous. */
int lsp_batch_ps_apply(lsp_batch* b, const double* const* u_dev, double* const* y_dev);

/* The assembly tile width the tuner chose (0 before the first setup), and
 * optionally the four candidate widths (0 = not a candidate) and their mean
 * times in ms (arrays of 4). Width 1 is the 2D form with tiles of 8 rows x 64
 * points and the shift tables copied into LDS (a candidate when every n is a
 * multiple of 64 and |S| m <= 1024 for every problem; the smallest width
 * gives way to it when four widths divide every n). */
int lsp_batch_tile(const lsp_batch* b, int* tile_width, int* candidates, float* ms);

/* Fix the assembly tile width of the following setups of the batch instead of
 * tuning it: 16, 32, 64 or 128 (must divide every n), or 1 (the LDS-table
 * form: 2D, every n a multiple of 64, |S| m <= 1024 for every problem); 0
 * returns to the tuner. Every width gives the same rows. LSP_EINVAL for
 * another value here, or at the next lsp_batch_stencil_setup if the width
 * does not fit that batch (nothing is launched then). */
int lsp_batch_set_tile(lsp_batch* b, int tile_width);

#ifdef __cplusplus
}
#endif

#endif /* LSP_H */
