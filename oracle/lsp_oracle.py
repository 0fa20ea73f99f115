"""FP64 CPU oracle for the localized sparsifying preconditioner.

TEST INFRASTRUCTURE ONLY. Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import this module. The HIP library never
calls it, and it shares no code with the HIP path: it is written from
F. Liu and L. Ying, "Localized Sparsifying Preconditioner for Periodic
Indefinite Systems" (arXiv 1607.02560), section by section, with plain
numpy/scipy routines as the only building blocks.

Every function follows one passage of the paper:

  wavenumbers, symbol      Sec. 2 (grid K, symbol 4 pi^2 |k|^2)
  ps_apply                 Sec. 2, eq. (dmodel): (L + diag v) u
  dense_laplacian          Sec. 2, L = F^-1 diag(4 pi^2 |k|^2) F, as a dense matrix
  shift_list               Sec. 4.1 (shifts evenly in [v_min, v_max], form (4m+2) pi^2)
  green_kernels            Sec. 3 (G = (L+s)^-1 by FFT) and Sec. 4.2 (g_s * g_s by FFT)
  offsets                  Sec. 4.2, neighbourhood mu_0^t
  gram                     Sec. 4.2, eq. (A): A1 - A2
  null_vector              Sec. 4.2: eigenvector of the smallest eigenvalue of A1 - A2
  null_vector_svd          Sec. 3: last left singular vector of G[mu, mu^c] (the definition)
  assign_shifts            Sec. 4.1: s_j = the shift of S closest to v_j
  assemble                 Sec. 4.1/4.2: Q, C and P rows
  stencil_setup            all of the above in the paper's order
  global_shift, global_setup
                           Sec. 3: the non-localized preconditioner, one
                           shift s = mean(v) for every point
  nd_tmap, nd_setup        Sec. 4.2 and Fig. 3: the per-point radius t_j that
                           nested dissection with leaf box b allows
  sparse_P, sparse_C       eq. (PC) as sparse matrices
  gmres_right              Sec. 5: GMRES with restart, preconditioner P^-1 C

Readings of passages that are silent or garbled (each also listed in the
design notes of the repository):
  * s_j is printed as a min of distances; read as the argmin shift, ties to
    the lower (smaller) shift.
  * shifts: bin centres v_min + (i + 1/2)(v_max - v_min)/|S|, each snapped to
    the nearest value of the form (4m+2) pi^2 with m = floor(s / (4 pi^2)),
    then duplicates removed.
  * neighbourhood offsets are ordered lexicographically over [-t, t]^d, last
    axis fastest.
  * alpha is defined up to sign: unit 2-norm, sign chosen so that the entry of
    largest magnitude is positive (ties: lowest offset index). Scaling a row of
    both P and C leaves P^-1 C unchanged, so the choice is immaterial to the solve.
  * GMRES: right preconditioning, x0 = 0, the iteration count is the total
    number of Arnoldi steps.
  * per-point radius (Sec. 4.2, Fig. 3): separators are the grid planes
    j_i = 0 mod b; a vertex (all coordinates on separators) takes t = b, any
    other point the smallest distance from its off-separator coordinates to a
    separator plane; then t_j = min(that, t_max). This reproduces every value
    of Fig. 3.
  * non-localized shift (Sec. 3): the mean of v, moved only when L + s is
    singular: x = -s / (4 pi^2) within RESONANCE_TOL * max(1, |x|) of an
    integer K >= 0 counts as singular, and s then goes to (4m+2) pi^2 with
    m = -K (the resonance-free form of Sec. 4.1, 2 pi^2 above -4 pi^2 K; the
    two values of that form nearest to -4 pi^2 K are equally near, and
    choosing by K rather than by s keeps the choice stable under rounding).
"""
from __future__ import annotations

import itertools
import math

import numpy as np
import scipy.linalg
import scipy.sparse
import scipy.sparse.linalg

FOUR_PI2 = 4.0 * math.pi ** 2


# --------------------------------------------------------------------------
# Section 2: grids, Fourier transform, pseudospectral Laplacian
# --------------------------------------------------------------------------
def wavenumbers(n: int) -> np.ndarray:
    """Integer frequencies of the grid K = [-n/2, n/2) in FFT storage order:
    position i holds i for i < n/2 and i - n otherwise (Sec. 2, grid K)."""
    i = np.arange(n)
    return np.where(i < n // 2, i, i - n)


def symbol(d: int, n: int) -> np.ndarray:
    """lambda_k = 4 pi^2 |k|^2 on K, FFT storage order, shape (n,)*d (Sec. 2, L)."""
    k = wavenumbers(n).astype(np.float64)
    lam = np.zeros((n,) * d)
    for ax in range(d):
        shape = [1] * d
        shape[ax] = n
        lam = lam + (k * k).reshape(shape)
    return FOUR_PI2 * lam


def ps_apply(v: np.ndarray, u: np.ndarray) -> np.ndarray:
    """(L + diag v) u with L = F^-1 diag(4 pi^2 |k|^2) F (Sec. 2, eq. dmodel).

    numpy's fftn is the unnormalised forward sum and ifftn carries 1/N, so
    ifftn(lambda * fftn(u)) equals F^-1 diag(lambda) F u for the unitary pair
    of the paper (the two factors n^{-d/2} combine into 1/N)."""
    d, n = u.ndim, u.shape[0]
    lam = symbol(d, n)
    return np.fft.ifftn(lam * np.fft.fftn(u)) + v * u


def laplacian_1d_dense(n: int) -> np.ndarray:
    """Dense 1D matrix of L on n points, written out in closed form.

    Entry (p, q) is (1/n) sum_{k in K} 4 pi^2 k^2 exp(2 pi i k (p-q)/n). Summing
    the series gives pi^2 (n^2 + 2)/3 on the diagonal and
    2 pi^2 (-1)^r / sin^2(pi r / n) for r = p - q != 0 (the periodic spectral
    second-derivative matrix, rescaled from [0, 2 pi) to [0, 1) and negated)."""
    p = np.arange(n)
    r = (p[:, None] - p[None, :]) % n
    out = np.empty((n, n))
    off = r != 0
    rr = r[off]
    out[off] = 2.0 * math.pi ** 2 * np.where(rr % 2 == 0, 1.0, -1.0) / np.sin(math.pi * rr / n) ** 2
    out[~off] = math.pi ** 2 * (n * n + 2) / 3.0
    return out


def dense_laplacian(d: int, n: int) -> np.ndarray:
    """Dense L on (n,)*d, C order, as the Kronecker sum of 1D matrices."""
    L1 = laplacian_1d_dense(n)
    eye = np.eye(n)
    N = n ** d
    L = np.zeros((N, N))
    for ax in range(d):
        term = np.ones((1, 1))
        for b in range(d):
            term = np.kron(term, L1 if b == ax else eye)
        L += term
    return L


def dense_operator(v: np.ndarray) -> np.ndarray:
    """A = L + diag(v) as a dense matrix (tiny grids only)."""
    d, n = v.ndim, v.shape[0]
    return dense_laplacian(d, n) + np.diag(v.reshape(-1))


# --------------------------------------------------------------------------
# Section 4.1: shift list and assignment
# --------------------------------------------------------------------------
def snap_shift(s: float) -> float:
    """Nearest value of the form (4m + 2) pi^2, m integer (Sec. 4.1, resonance).
    With x = s/(4 pi^2), the candidates are 4 pi^2 (m + 1/2); m = floor(x)."""
    m = math.floor(s / FOUR_PI2)
    return (4 * m + 2) * math.pi ** 2


def shift_list(v: np.ndarray, num_shifts: int) -> np.ndarray:
    """Shift list S (Sec. 4.1): num_shifts bin centres spread evenly over
    [v_min, v_max], snapped to the form (4m+2) pi^2 and de-duplicated.
    Returned sorted increasing."""
    if num_shifts < 1:
        raise ValueError("num_shifts must be >= 1")
    vmin, vmax = float(np.min(v)), float(np.max(v))
    width = (vmax - vmin) / num_shifts
    out = []
    for i in range(num_shifts):
        centre = vmin + (i + 0.5) * width
        s = snap_shift(centre)
        if not out or s != out[-1]:
            out.append(s)
    return np.asarray(out, dtype=np.float64)


def assign_shifts(v: np.ndarray, S: np.ndarray) -> np.ndarray:
    """idx_j = argmin_i |S_i - v_j| (Sec. 4.1, the shift closest to v_j);
    np.argmin keeps the first minimiser, i.e. ties go to the lower index."""
    flat = v.reshape(-1)
    idx = np.empty(flat.size, dtype=np.int32)
    chunk = 1 << 16
    for a in range(0, flat.size, chunk):
        blk = flat[a:a + chunk]
        idx[a:a + chunk] = np.argmin(np.abs(S[None, :] - blk[:, None]), axis=1)
    return idx.reshape(v.shape)


# --------------------------------------------------------------------------
# Sections 3 and 4.2: Green's kernels, neighbourhoods, Gram identity
# --------------------------------------------------------------------------
def green_kernels(d: int, n: int, s: float):
    """g_s = G_s[:, 0] and gamma_s = (g_s * g_s), both on the full grid.

    G_s = (L + s)^-1 = F^-1 diag(1/(lambda_k + s)) F (Sec. 3), so its first
    column is ifftn(1/(lambda + s)) (ifftn's 1/N again matches the unitary
    pair). The periodic self-convolution g_s * g_s has symbol 1/(lambda+s)^2
    and is obtained by one more inverse FFT (Sec. 4.2)."""
    lam = symbol(d, n)
    den = lam + s
    if np.min(np.abs(den)) == 0.0:
        raise ZeroDivisionError("L + s is singular for this shift")
    g = np.fft.ifftn(1.0 / den)
    gam = np.fft.ifftn(1.0 / den ** 2)
    # lambda is even in every coordinate, so both kernels are real.
    assert np.max(np.abs(g.imag)) <= 1e-9 * np.max(np.abs(g.real)) + 1e-300
    assert np.max(np.abs(gam.imag)) <= 1e-9 * np.max(np.abs(gam.real)) + 1e-300
    return np.ascontiguousarray(g.real), np.ascontiguousarray(gam.real)


def offsets(d: int, t: int) -> np.ndarray:
    """Offsets of mu_0^t = {i : ||i||_inf <= t} (Sec. 4.2), lexicographic,
    last axis fastest. Shape (m, d), m = (2t+1)^d."""
    rng = range(-t, t + 1)
    return np.asarray(list(itertools.product(*([rng] * d))), dtype=np.int64)


def _take(arr: np.ndarray, delta: np.ndarray) -> np.ndarray:
    """arr[delta mod n] for an array of integer offsets (last dim = d)."""
    n = arr.shape[0]
    idx = tuple((delta[..., ax] % n) for ax in range(arr.ndim))
    return arr[idx]


def gram(g: np.ndarray, gam: np.ndarray, offs: np.ndarray):
    """Eq. (A): G_mu,mu, A1 = G[mu,:] G[mu,:]^T and A2 = G[mu,mu] G[mu,mu]^T.

    G_s[j1, j2] = g_s[j1 - j2] and the entries of A1 are values of the
    self-convolution: A1[a, b] = (g_s * g_s)[a - b] (Sec. 4.2)."""
    diff = offs[:, None, :] - offs[None, :, :]
    Gmm = _take(g, diff)
    A1 = _take(gam, diff)
    A2 = Gmm @ Gmm.T
    return Gmm, A1, A2, A1 - A2


def normalise_sign(alpha: np.ndarray) -> np.ndarray:
    """Unit 2-norm, entry of largest magnitude positive (lowest index on ties)."""
    alpha = alpha / np.linalg.norm(alpha)
    i = int(np.argmax(np.abs(alpha)))
    return alpha if alpha[i] > 0 else -alpha


def null_vector(M: np.ndarray):
    """alpha = eigenvector of the smallest eigenvalue of M = A1 - A2 (Sec. 4.2).

    Returns alpha, the eigenvalues in increasing order, sigma_min =
    sqrt(max(lambda_1, 0)), and kappa = lambda_max / (lambda_2 - lambda_1),
    the first-order sensitivity of the eigenvector to perturbations of M."""
    w, V = np.linalg.eigh(M)
    alpha = normalise_sign(V[:, 0])
    gap = w[1] - w[0]
    kappa = w[-1] / gap if gap > 0 else math.inf
    return alpha, w, math.sqrt(max(w[0], 0.0)), kappa


def offneighbourhood_block(g: np.ndarray, offs: np.ndarray) -> np.ndarray:
    """B = G_s[mu_0, mu_0^c] explicitly: rows a in mu_0, columns j not in mu_0,
    B[a, j] = g_s[a - j] (Sec. 3, translation invariance of G_s)."""
    d, n = g.ndim, g.shape[0]
    N = n ** d
    all_j = np.stack(np.unravel_index(np.arange(N), (n,) * d), axis=-1)
    mu_flat = np.ravel_multi_index(tuple((offs % n).T), (n,) * d)
    mask = np.ones(N, dtype=bool)
    mask[mu_flat] = False
    cols = all_j[mask]
    diff = offs[:, None, :] - cols[None, :, :]
    return _take(g, diff)


def null_vector_svd(g: np.ndarray, offs: np.ndarray):
    """The definition route (Sec. 3): SVD of B = G_s[mu_0, mu_0^c]; alpha is the
    left singular vector of the smallest singular value, which is the optimum
    of min ||alpha^T B||_2 over unit alpha."""
    B = offneighbourhood_block(g, offs)
    U, sv, _ = np.linalg.svd(B, full_matrices=False)
    return normalise_sign(U[:, -1]), sv


# --------------------------------------------------------------------------
# Section 4: stencils and the sparse system
# --------------------------------------------------------------------------
def shift_tables(d: int, n: int, S: np.ndarray, t: int):
    """For each shift of S: g, gamma on [-2t, 2t]^d, M, alpha, C = G_mu,mu alpha,
    sigma_min and kappa (Sec. 4.2)."""
    offs = offsets(d, t)
    m = offs.shape[0]
    tab = {
        "alpha": np.zeros((len(S), m)), "C": np.zeros((len(S), m)),
        "sigma_min": np.zeros(len(S)), "kappa": np.zeros(len(S)),
        "M": np.zeros((len(S), m, m)), "eig": np.zeros((len(S), m)),
        "g": [], "gamma": [],
    }
    for i, s in enumerate(S):
        g, gam = green_kernels(d, n, s)
        Gmm, A1, A2, M = gram(g, gam, offs)
        alpha, w, smin, kappa = null_vector(M)
        tab["alpha"][i] = alpha
        tab["C"][i] = Gmm @ alpha        # C[j, mu] = Q[j, mu] G[mu, mu]; G_mu,mu symmetric
        tab["sigma_min"][i] = smin
        tab["kappa"][i] = kappa
        tab["M"][i] = M
        tab["eig"][i] = w
        tab["g"].append(g)
        tab["gamma"].append(gam)
    tab["offsets"] = offs
    return tab


def green_window(g: np.ndarray, t: int) -> np.ndarray:
    """g restricted to offsets [-2t, 2t]^d, returned as an array indexed by
    delta + 2t (shape (4t+1,)*d)."""
    d = g.ndim
    rng = np.arange(-2 * t, 2 * t + 1)
    grids = np.meshgrid(*([rng] * d), indexing="ij")
    delta = np.stack(grids, axis=-1)
    return _take(g, delta)


def assemble(v: np.ndarray, S: np.ndarray, alpha: np.ndarray, C: np.ndarray,
             idx: np.ndarray, offs: np.ndarray) -> np.ndarray:
    """P rows (Sec. 4.1/4.2): P[j, a] = alpha_{s_j}[a] + C_{s_j}[a] (v[j+a] - s_j),
    for a in mu_0^t. Returns shape (N, m)."""
    d, n = v.ndim, v.shape[0]
    flat_idx = idx.reshape(-1)
    m = offs.shape[0]
    P = np.empty((v.size, m))
    s_j = S[flat_idx]
    for a in range(m):
        va = np.roll(v, shift=tuple(-offs[a]), axis=tuple(range(d))).reshape(-1)
        P[:, a] = alpha[flat_idx, a] + C[flat_idx, a] * (va - s_j)
    return P


def stencil_setup(v: np.ndarray, t: int, num_shifts: int) -> dict:
    """The whole setup in the paper's order: S, per-shift tables, s_j, P."""
    d, n = v.ndim, v.shape[0]
    S = shift_list(v, num_shifts)
    tab = shift_tables(d, n, S, t)
    idx = assign_shifts(v, S)
    P = assemble(v, S, tab["alpha"], tab["C"], idx, tab["offsets"])
    tab.update(S=S, idx=idx, P=P)
    return tab


# --------------------------------------------------------------------------
# Section 3: the non-localized sparsifying preconditioner
# --------------------------------------------------------------------------
RESONANCE_TOL = 2.0 ** -30


def global_shift(v: np.ndarray) -> float:
    """The one shift of the non-localized preconditioner (Sec. 3): the
    average of v, so that q = v - s has zero mean. L + s is singular when
    s = -4 pi^2 K for an integer K = |k|^2 >= 0; the paper then perturbs s
    slightly. Here such an s (to RESONANCE_TOL) is replaced by (4m+2) pi^2
    with m = -K, the value of that form 2 pi^2 above the singular point."""
    s = float(np.mean(v, dtype=np.float64))
    x = -s / FOUR_PI2
    K = math.floor(x + 0.5)
    if K >= 0 and abs(x - K) <= RESONANCE_TOL * max(1.0, abs(x)):
        s = (4 * (-K) + 2) * math.pi ** 2
    return s


def global_setup(v: np.ndarray, t: int) -> dict:
    """The non-localized setup of Sec. 3 with neighbourhood radius t: the
    tables of the single shift s = global_shift(v), every point assigned to
    it, and P = Q + C diag(v - s) in the row layout of `assemble`."""
    d, n = v.ndim, v.shape[0]
    S = np.asarray([global_shift(v)], dtype=np.float64)
    tab = shift_tables(d, n, S, t)
    idx = np.zeros(v.shape, dtype=np.int32)
    P = assemble(v, S, tab["alpha"], tab["C"], idx, tab["offsets"])
    tab.update(S=S, idx=idx, P=P)
    return tab


# --------------------------------------------------------------------------
# Section 4.2, Fig. 3: the radius each point may use under nested dissection
# --------------------------------------------------------------------------
def nd_tmap(d: int, n: int, b: int, tmax: int) -> np.ndarray:
    """t_j of Sec. 4.2: the largest radius that keeps the sparsity nested
    dissection with leaf box b needs (Fig. 3), capped at tmax. Separators are
    the planes j_i = 0 mod b. A vertex (every coordinate on a separator) may
    reach t = b; any other point reaches up to the nearest separator plane
    across its coordinates off the separators."""
    if n % b != 0 or b < 2:
        raise ValueError("the leaf box b must divide n")
    coords = np.stack(np.unravel_index(np.arange(n ** d), (n,) * d), axis=-1)
    r = coords % b
    dist = np.minimum(r, b - r)
    off = r != 0
    reach = np.where(off, dist, n).min(axis=1)
    t = np.where(off.any(axis=1), reach, b)
    return np.minimum(t, tmax).reshape((n,) * d)


def nd_setup(v: np.ndarray, b: int, tmax: int, num_shifts: int) -> dict:
    """Stencils with the per-point radius t_j = nd_tmap (Sec. 4.2): the tables
    of every radius t <= tmax for each shift, and rows j of P and C from the
    tables of (s_j, t_j). Rows use the layout of radius tmax (offsets
    mu_0^tmax); entries outside mu_0^{t_j} are zero."""
    d, n = v.ndim, v.shape[0]
    S = shift_list(v, num_shifts)
    idx = assign_shifts(v, S)
    flat_idx = idx.reshape(-1)
    tm = nd_tmap(d, n, b, tmax).reshape(-1)
    offs = offsets(d, tmax)
    where = {tuple(o): k for k, o in enumerate(offs)}
    P = np.zeros((v.size, offs.shape[0]))
    Crows = np.zeros_like(P)
    tables = {}
    for t in range(1, tmax + 1):
        tab = shift_tables(d, n, S, t)
        tables[t] = tab
        pos = np.array([where[tuple(o)] for o in tab["offsets"]])
        sel = np.nonzero(tm == t)[0]
        Pt = assemble(v, S, tab["alpha"], tab["C"], idx, tab["offsets"])
        P[np.ix_(sel, pos)] = Pt[sel]
        Crows[np.ix_(sel, pos)] = tab["C"][flat_idx[sel]]
    return {"S": S, "idx": idx, "tmap": tm.reshape(v.shape), "P": P, "Crows": Crows,
            "offsets": offs, "tables": tables}


def neighbour_columns(d: int, n: int, offs: np.ndarray) -> np.ndarray:
    """Column index (j + a) mod n, flattened, for each row j and offset a."""
    N = n ** d
    j = np.stack(np.unravel_index(np.arange(N), (n,) * d), axis=-1)
    cols = (j[:, None, :] + offs[None, :, :]) % n
    return np.ravel_multi_index(tuple(np.moveaxis(cols, -1, 0)), (n,) * d)


def sparse_rows(values: np.ndarray, d: int, n: int, offs: np.ndarray):
    """CSR matrix with row j holding values[j, a] at column (j + a) mod n."""
    N = n ** d
    m = offs.shape[0]
    cols = neighbour_columns(d, n, offs)
    indptr = np.arange(0, N * m + 1, m)
    return scipy.sparse.csr_matrix((values.reshape(-1), cols.reshape(-1), indptr), shape=(N, N))


def sparse_P(setup: dict, d: int, n: int):
    return sparse_rows(setup["P"], d, n, setup["offsets"])


def sparse_C(setup: dict, d: int, n: int):
    """C rows C[j, mu_j] = C_{s_j} (Sec. 4.1), zero elsewhere."""
    Crows = setup["C"][setup["idx"].reshape(-1)]
    return sparse_rows(Crows, d, n, setup["offsets"])


# --------------------------------------------------------------------------
# Section 5: GMRES with the preconditioner P^-1 C
# --------------------------------------------------------------------------
def gmres_right(apply_A, apply_M, f: np.ndarray, rtol: float, restart: int, maxit: int):
    """Restarted GMRES with right preconditioning: solve A M y = f, u = M y.

    Arnoldi with modified Gram-Schmidt and Givens rotations, x0 = 0. Stops
    when the Arnoldi residual estimate falls to rtol ||f||. Returns
    (u, iterations, estimated relative residual, true relative residual)."""
    b = f.reshape(-1).astype(np.complex128)
    N = b.size
    bnorm = np.linalg.norm(b)
    x = np.zeros(N, dtype=np.complex128)
    if bnorm == 0.0:
        return x, 0, 0.0, 0.0
    iters = 0
    est = 1.0
    while iters < maxit:
        r = b - apply_A(x)
        beta = np.linalg.norm(r)
        est = beta / bnorm
        if est <= rtol:
            break
        V = np.zeros((restart + 1, N), dtype=np.complex128)
        H = np.zeros((restart + 1, restart), dtype=np.complex128)
        cs = np.zeros(restart, dtype=np.complex128)
        sn = np.zeros(restart, dtype=np.complex128)
        e = np.zeros(restart + 1, dtype=np.complex128)
        e[0] = beta
        V[0] = r / beta
        k_used = 0
        for k in range(restart):
            w = apply_A(apply_M(V[k]))
            for i in range(k + 1):
                H[i, k] = np.vdot(V[i], w)
                w = w - H[i, k] * V[i]
            H[k + 1, k] = np.linalg.norm(w)
            if H[k + 1, k] != 0:
                V[k + 1] = w / H[k + 1, k]
            for i in range(k):
                tmp = np.conj(cs[i]) * H[i, k] + np.conj(sn[i]) * H[i + 1, k]
                H[i + 1, k] = -sn[i] * H[i, k] + cs[i] * H[i + 1, k]
                H[i, k] = tmp
            a, bb = H[k, k], H[k + 1, k]
            rho = math.hypot(abs(a), abs(bb))
            cs[k] = a / rho if rho else 1.0
            sn[k] = bb / rho if rho else 0.0
            H[k, k] = rho
            H[k + 1, k] = 0.0
            e[k + 1] = -sn[k] * e[k]
            e[k] = np.conj(cs[k]) * e[k]
            iters += 1
            k_used = k + 1
            est = abs(e[k + 1]) / bnorm
            if est <= rtol or iters >= maxit:
                break
        y = scipy.linalg.solve_triangular(H[:k_used, :k_used], e[:k_used])
        x = x + apply_M(V[:k_used].T @ y)
        if est <= rtol:
            break
    true_rel = np.linalg.norm(b - apply_A(x)) / bnorm
    return x, iters, est, true_rel


def precond_solve(v: np.ndarray, f: np.ndarray, t: int, num_shifts: int,
                  rtol: float = 1e-8, restart: int = 40, maxit: int = 400,
                  non_localized: bool = False, nd_leaf: int = 0):
    """Solve (L + diag v) u = f by GMRES(restart) with the preconditioner
    P^-1 C of eq. (PC); P is factorised by a sparse LU. non_localized=True
    builds P and C by the one-shift method of Sec. 3 (num_shifts unused);
    nd_leaf = b > 0 uses the per-point radius of Sec. 4.2 with leaf box b and
    t as its cap."""
    d, n = v.ndim, v.shape[0]
    if nd_leaf:
        setup = nd_setup(v, nd_leaf, t, num_shifts)
        P = sparse_rows(setup["P"], d, n, setup["offsets"]).tocsc().astype(np.complex128)
        Cm = sparse_rows(setup["Crows"], d, n, setup["offsets"]).astype(np.complex128)
    else:
        setup = global_setup(v, t) if non_localized else stencil_setup(v, t, num_shifts)
        P = sparse_P(setup, d, n).tocsc().astype(np.complex128)
        Cm = sparse_C(setup, d, n).astype(np.complex128)
    lu = scipy.sparse.linalg.splu(P)

    def apply_A(x):
        return ps_apply(v, x.reshape(v.shape)).reshape(-1)

    def apply_M(x):
        return lu.solve(Cm @ x)

    u, iters, est, true_rel = gmres_right(apply_A, apply_M, f, rtol, restart, maxit)
    return u.reshape(v.shape), iters, est, true_rel, setup
