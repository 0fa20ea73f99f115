"""Nested-dissection factorisation of the sparsified matrix P (Sec. 3, Fig. 1).

This is the plain host-side step beside the hot path: the paper factorises P
by nested dissection and applies the factors in every GMRES iteration. Here
the factorisation is a multifrontal LU over the box hierarchy of the periodic
grid, written with numpy/scipy dense kernels; its factors are exported as
plain arrays so that the library can apply them on the device
(lsp_psolve_upload / lsp_psolve_apply), or applied on the host (solve()).

Ordering (Fig. 1). Leaf boxes have side b (b divides n). The boxes are merged
one axis at a time, axes in turn (sizes (b, b) -> (2b, b) -> (2b, 2b) -> ...
in 2D), until every side is n. A point is interior to its box at box sizes s
when no coordinate is a multiple of the box side along its axis; its front is
the first merge step at which it is interior, and the box it is interior to.
Points that are never interior (a coordinate equal to 0, the planes where the
periodic grid closes) form the last front. Fronts are eliminated step by step,
boxes in lexicographic order, points of a front in grid order.

Fronts (multifrontal LU). The frontal matrix of a front F is indexed by F
followed by U(F), the points of the boundary of F's closed box (all later in
the order). It collects the entries of P whose first-eliminated index is in F
and the update (Schur complement) matrices of F's children, the fronts of the
boxes merged into F's box at the previous step. The F block is factorised
with partial pivoting inside F; the Schur complement of F is passed to the
parent. This needs every row of P to stay inside the closed box of its point's
front, which the radii of Sec. 4.2 guarantee (uniform t = 1 with b >= 2, or the
per-point radius t_j of Fig. 3); other patterns raise ValueError.

Solve. With the frontal matrix [[A_FF, A_FU], [A_UF, A_UU]] and Pi A_FF = L U:
  forward  (fronts in order):   y_F = L^-1 Pi r_F,  r_U -= L_UF y_F
  backward (reverse order):     x_F = U^-1 (y_F - U_FU x_U)
with U_FU = L^-1 Pi A_FU and L_UF = A_UF U^-1.
"""
from __future__ import annotations

import dataclasses
import itertools

import numpy as np
import scipy.linalg
import scipy.sparse


@dataclasses.dataclass
class Front:
    step: int
    F: np.ndarray          # int64 grid indices eliminated here, grid order
    U: np.ndarray          # int64 update indices (later in the order)
    parent: int = -1       # index of the parent front (-1: the last one)


def merge_schedule(d: int, n: int, b: int):
    """Box sizes after each merge step: (b,..,b), then one axis doubled per
    step, axes in turn, until every side is n."""
    if b < 2 or n % b != 0 or (n // b) & (n // b - 1):
        raise ValueError("the leaf box b must be >= 2 and divide n by a power of two")
    sizes = [b] * d
    out = [tuple(sizes)]
    ax = 0
    while any(s < n for s in sizes):
        while sizes[ax] >= n:
            ax = (ax + 1) % d
        sizes[ax] *= 2
        out.append(tuple(sizes))
        ax = (ax + 1) % d
    return out


def nd_fronts(d: int, n: int, b: int):
    """Fronts of the nested-dissection order of the periodic (n,)*d grid with
    leaf box b, in elimination order, and the elimination position of every
    grid point."""
    N = n ** d
    coords = np.stack(np.unravel_index(np.arange(N), (n,) * d), axis=1)
    sched = merge_schedule(d, n, b)
    M = len(sched)
    step = np.full(N, M, dtype=np.int64)
    for m in range(M - 1, -1, -1):
        inside = np.all(coords % np.asarray(sched[m]) != 0, axis=1)
        step[inside] = m
    fronts = []
    key_of = {}
    for m in range(M):
        sel = np.nonzero(step == m)[0]
        if sel.size == 0:
            continue
        boxes = coords[sel] // np.asarray(sched[m])
        order = np.lexsort(tuple(boxes[:, i] for i in range(d - 1, -1, -1)))
        sel, boxes = sel[order], boxes[order]
        cut = np.nonzero(np.any(np.diff(boxes, axis=0) != 0, axis=1))[0] + 1
        for part, bx in zip(np.split(sel, cut), np.split(boxes, cut)):
            key_of[(m, tuple(bx[0]))] = len(fronts)
            fronts.append(Front(m, np.sort(part), np.empty(0, dtype=np.int64)))
    last = np.nonzero(step == M)[0]
    if last.size:
        key_of[(M, ())] = len(fronts)
        fronts.append(Front(M, last, np.empty(0, dtype=np.int64)))
    pos = np.empty(N, dtype=np.int64)
    pos[np.concatenate([f.F for f in fronts])] = np.arange(N)
    # update sets: the boundary of the closed box; parents: the front of the
    # merged box at the next step that holds this box
    for k, f in enumerate(fronts):
        if f.step == M:
            continue
        s = np.asarray(sched[f.step])
        lo = (coords[f.F[0]] // s) * s
        axes = [((lo[i] + np.arange(s[i] + 1)) % n) if s[i] < n else np.arange(n)
                for i in range(d)]
        closed = np.stack([g.reshape(-1) for g in np.meshgrid(*axes, indexing="ij")], axis=1)
        on_edge = np.any(closed % s == 0, axis=1)
        U = np.unique(np.ravel_multi_index(tuple(closed[on_edge].T), (n,) * d))
        f.U = U[np.argsort(pos[U], kind="stable")]
        if f.step + 1 < M:
            s1 = np.asarray(sched[f.step + 1])
            f.parent = key_of.get((f.step + 1, tuple(coords[f.F[0]] // s1)), -1)
        if f.parent < 0 or f.step + 1 >= M:
            f.parent = key_of[(M, ())]
    return fronts, pos


@dataclasses.dataclass
class NDFactor:
    """Factors of P in the nested-dissection order (see the module notes)."""
    N: int
    fronts: list
    piv: list              # row permutation of each front's F block (positions in F)
    L: list                # unit lower triangle of each F block (f x f)
    Ublk: list             # upper triangle (f x f)
    LUF: list              # L_UF (u x f)
    UFU: list              # U_FU (f x u)

    def solve(self, r: np.ndarray) -> np.ndarray:
        """x = P^-1 r (host, any dtype of r)."""
        r = np.array(r, dtype=np.result_type(r, np.float64), copy=True).reshape(-1)
        y = np.empty_like(r)
        for k, f in enumerate(self.fronts):
            rf = r[f.F][self.piv[k]]
            yf = scipy.linalg.solve_triangular(self.L[k], rf, lower=True, unit_diagonal=True)
            y[f.F] = yf
            if f.U.size:
                r[f.U] -= self.LUF[k] @ yf
        x = np.empty_like(r)
        for k in range(len(self.fronts) - 1, -1, -1):
            f = self.fronts[k]
            rhs = y[f.F] - (self.UFU[k] @ x[f.U] if f.U.size else 0.0)
            x[f.F] = scipy.linalg.solve_triangular(self.Ublk[k], rhs, lower=False)
        return x

    def levels(self):
        """Groups of fronts that depend on none of each other (one merge step)."""
        steps = sorted({f.step for f in self.fronts})
        return [[k for k, f in enumerate(self.fronts) if f.step == s] for s in steps]

    def export(self):
        """Plain arrays of the factors for the device solve: per front its
        sizes and offsets, the index lists, four dense blocks, the front
        levels, and, per grid point, the positions of the updates other fronts
        send to it. The blocks are L_FF^-1, L_UF L_FF^-1, U_FF^-1 and
        U_FF^-1 U_FU, so that with r_F the front's gathered right-hand side
        both forward products (y_F = L_FF^-1 r_F and the updates
        L_UF y_F = (L_UF L_FF^-1) r_F) read r_F only, and the backward step
        x_F = U_FF^-1 y_F - (U_FF^-1 U_FU) x_U is one product per row."""
        nf = len(self.fronts)
        f_sz = np.array([f.F.size for f in self.fronts], dtype=np.int64)
        u_sz = np.array([f.U.size for f in self.fronts], dtype=np.int64)
        off_F = np.concatenate([[0], np.cumsum(f_sz)]).astype(np.int64)
        off_U = np.concatenate([[0], np.cumsum(u_sz)]).astype(np.int64)
        idx_F = np.concatenate([f.F for f in self.fronts]).astype(np.int64)
        idx_Fp = np.concatenate([f.F[self.piv[k]] for k, f in enumerate(self.fronts)]).astype(np.int64)
        idx_U = (np.concatenate([f.U for f in self.fronts]) if u_sz.sum() else
                 np.zeros(0)).astype(np.int64)
        blocks = []
        off_blk = np.zeros((nf, 4), dtype=np.int64)   # Linv, LUF Linv, Uinv, Uinv UFU
        cur = 0
        for k in range(nf):
            f = int(f_sz[k])
            Linv = scipy.linalg.solve_triangular(self.L[k], np.eye(f), lower=True,
                                                 unit_diagonal=True)
            Uinv = scipy.linalg.solve_triangular(self.Ublk[k], np.eye(f), lower=False)
            for j, blk in enumerate((Linv, self.LUF[k] @ Linv, Uinv, Uinv @ self.UFU[k])):
                off_blk[k, j] = cur
                blocks.append(np.ascontiguousarray(blk, dtype=np.float64).reshape(-1))
                cur += blk.size
        data = np.concatenate(blocks) if blocks else np.zeros(0)
        # updates sent to each point: position in the concatenated U lists
        # (the forward pass stores L_UF y_F there), in front order
        src = np.argsort(idx_U, kind="stable")
        counts = np.bincount(idx_U, minlength=self.N)
        upd_ptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
        upd_pos = src.astype(np.int64)
        lev = self.levels()
        lev_ptr = np.concatenate([[0], np.cumsum([len(x) for x in lev])]).astype(np.int64)
        lev_fronts = np.concatenate([np.asarray(x) for x in lev]).astype(np.int64)
        return {"f": f_sz, "u": u_sz, "off_F": off_F, "off_U": off_U, "idx_F": idx_F,
                "idx_Fp": idx_Fp, "idx_U": idx_U, "off_blk": off_blk.reshape(-1),
                "data": data, "upd_ptr": upd_ptr, "upd_pos": upd_pos,
                "lev_ptr": lev_ptr, "lev_fronts": lev_fronts}


def factor(P, d: int, n: int, b: int) -> NDFactor:
    """Multifrontal LU of the N x N sparse matrix P (any scipy format, real)
    in the nested-dissection order of the periodic grid with leaf box b."""
    N = n ** d
    A = scipy.sparse.csr_matrix(P, dtype=np.float64)
    A.eliminate_zeros()   # rows of radius t_j < t_max are stored zero-padded
    At = scipy.sparse.csr_matrix(A.T)
    fronts, pos = nd_fronts(d, n, b)
    children = [[] for _ in fronts]
    for k, f in enumerate(fronts):
        if k != len(fronts) - 1:
            children[f.parent].append(k)
    upd = [None] * len(fronts)
    piv, Ls, Us, LUFs, UFUs = [], [], [], [], []
    local = np.full(N, -1, dtype=np.int64)
    for k, f in enumerate(fronts):
        idx = np.concatenate([f.F, f.U])
        nF = f.F.size
        local[idx] = np.arange(idx.size)
        Fm = np.zeros((idx.size, idx.size))
        first = pos[f.F[0]]
        # rows of F: entries whose column is not eliminated before F
        for li, i in enumerate(f.F):
            cols = A.indices[A.indptr[i]:A.indptr[i + 1]]
            vals = A.data[A.indptr[i]:A.indptr[i + 1]]
            keep = pos[cols] >= first
            lj = local[cols[keep]]
            if np.any(lj < 0):
                raise ValueError("P couples a point outside its nested-dissection box; "
                                 "use t = 1 or the per-point radius of Sec. 4.2")
            np.add.at(Fm[li], lj, vals[keep])
        # columns of F: entries in rows of U (later than F)
        for li, i in enumerate(f.F):
            rows = At.indices[At.indptr[i]:At.indptr[i + 1]]
            vals = At.data[At.indptr[i]:At.indptr[i + 1]]
            later = pos[rows] >= first + nF
            lr = local[rows[later]]
            if np.any(lr < 0):
                raise ValueError("P couples a point outside its nested-dissection box; "
                                 "use t = 1 or the per-point radius of Sec. 4.2")
            np.add.at(Fm[:, li], lr, vals[later])
        for c in children[k]:
            lu_c = local[fronts[c].U]
            if np.any(lu_c < 0):
                raise ValueError("a child's update set leaves its parent front")
            Fm[np.ix_(lu_c, lu_c)] += upd[c]
            upd[c] = None
        lu, pv = scipy.linalg.lu_factor(Fm[:nF, :nF], check_finite=True)
        perm = np.arange(nF)
        for a, bb in enumerate(pv):           # LAPACK swaps -> a permutation of F
            perm[a], perm[bb] = perm[bb], perm[a]
        L = np.tril(lu, -1) + np.eye(nF)
        Ub = np.triu(lu)
        A_FU = Fm[:nF, nF:][perm]
        U_FU = scipy.linalg.solve_triangular(L, A_FU, lower=True, unit_diagonal=True)
        L_UF = scipy.linalg.solve_triangular(Ub, Fm[nF:, :nF].T, trans="T", lower=False).T
        if f.U.size:
            upd[k] = Fm[nF:, nF:] - L_UF @ U_FU
        piv.append(perm)
        Ls.append(L)
        Us.append(Ub)
        LUFs.append(L_UF)
        UFUs.append(U_FU)
        local[idx] = -1
    return NDFactor(N, fronts, piv, Ls, Us, LUFs, UFUs)
