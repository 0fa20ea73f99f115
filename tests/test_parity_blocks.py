"""The Gram matrix M = A1 - A2 of eq. (A) is invariant under the reflection of
any axis (g_s is even in every coordinate, Sec. 4.2), so it is block diagonal
in the orthonormal parity basis of the neighbourhood; the HIP null-vector
kernel solves one block per parity class. This checks the property on the
oracle's M, with the basis built here from its definition."""
import math

import numpy as np
import pytest

from oracle import lsp_oracle as O


def parity_basis(d, t):
    """Columns grouped by class c (bit d-1-i = parity along axis i); inside a
    class, lexicographic over the per-axis 1D indices (0..t even, 1..t odd)."""
    offs = O.offsets(d, t)
    m = offs.shape[0]
    cols, classes = [], []
    for c in range(1 << d):
        odd = [(c >> (d - 1 - i)) & 1 for i in range(d)]
        ranges = [range(1, t + 1) if odd[i] else range(0, t + 1) for i in range(d)]
        for js in np.ndindex(*[len(r) for r in ranges]):
            j = [ranges[i][js[i]] for i in range(d)]
            col = np.zeros(m)
            for a in range(m):
                x = offs[a]
                coef = 1.0
                for i in range(d):
                    if abs(x[i]) != j[i]:
                        coef = 0.0
                        break
                    if j[i] != 0:
                        coef *= (-1.0 if (odd[i] and x[i] < 0) else 1.0) / math.sqrt(2.0)
                col[a] = coef
            cols.append(col)
            classes.append(c)
    return np.stack(cols, axis=1), np.asarray(classes)


@pytest.mark.parametrize("d,t,n,mshift", [(2, 1, 16, -20), (2, 2, 32, -60), (2, 3, 32, -40),
                                          (3, 1, 8, -9)])
def test_gram_is_block_diagonal_in_parity_basis(d, t, n, mshift):
    s = (4 * mshift + 2) * math.pi ** 2
    g, gam = O.green_kernels(d, n, s)
    offs = O.offsets(d, t)
    _, _, _, M = O.gram(g, gam, offs)
    Q, cls = parity_basis(d, t)
    assert np.allclose(Q.T @ Q, np.eye(Q.shape[1]), atol=1e-14)
    Mb = Q.T @ M @ Q
    off = cls[:, None] != cls[None, :]
    assert np.max(np.abs(Mb[off])) <= 1e-12 * np.max(np.abs(M))
    # the smallest eigenvalue of M is the smallest over the class blocks, and
    # its eigenvector is supported on one class
    w = np.linalg.eigvalsh(M)
    block_min = min(np.linalg.eigvalsh(Mb[np.ix_(cls == c, cls == c)])[0] for c in set(cls))
    assert block_min == pytest.approx(w[0], rel=1e-6, abs=1e-10 * w[-1])
    alpha, *_ = O.null_vector(M)
    comp = Q.T @ alpha
    by_class = [np.linalg.norm(comp[cls == c]) for c in sorted(set(cls))]
    assert max(by_class) == pytest.approx(1.0, abs=1e-6)


def test_block_sizes():
    for d, t, sizes in [(2, 2, [9, 6, 6, 4]), (2, 1, [4, 2, 2, 1]),
                        (3, 1, [8, 4, 4, 2, 4, 2, 2, 1])]:
        _, cls = parity_basis(d, t)
        assert [int(np.sum(cls == c)) for c in range(1 << d)] == sizes
