"""The per-point radius of Sec. 4.2 (lsp_stencil_setup_nd) through the C ABI:
radius-2 rows equal, bit for bit, the rows of the uniform radius-2 setup;
radius-1 rows (padded with zeros) equal, bit for bit, the row formula on the
setup's own radius-1 tables, which are formed from the radius-2 Green's pass
(the same sums at offsets [0, 2]^d, added in another order) and agree with
the uniform radius-1 setup's tables to rounding; the radius map matches the
oracle's (pinned to Fig. 3), the rows match the oracle's nd_setup to 1e-8,
the C-apply uses the per-point C rows, and GMRES counts are within one of the
oracle's."""
import numpy as np
import pytest

from oracle import lsp_oracle as O
from paper_1607_02560_amd import workloads as W
from tests.test_gpu_parity import lsp_mod, torch_dev  # noqa: F401

pytestmark = pytest.mark.gpu


def run_nd(torch_dev, v, leaf, nS):
    torch, dev = torch_dev
    lsp = lsp_mod()
    d, n = v.ndim, v.shape[0]
    N, M = n ** d, 5 ** d
    prob = lsp.Problem(d, n, torch.from_numpy(np.ascontiguousarray(v).reshape(-1)).to(dev))
    P = torch.full((N * M,), float("nan"), dtype=torch.float64, device=dev)
    idx = torch.full((N,), -1, dtype=torch.int32, device=dev)
    prob.stencil_setup_nd(leaf, nS, P, idx)
    torch.cuda.synchronize()
    return prob, P.cpu().numpy().reshape(N, M), idx.cpu().numpy()


def uniform(torch_dev, v, t, nS, tables=False):
    torch, dev = torch_dev
    lsp = lsp_mod()
    d, n = v.ndim, v.shape[0]
    N, m = n ** d, (2 * t + 1) ** d
    prob = lsp.Problem(d, n, torch.from_numpy(np.ascontiguousarray(v).reshape(-1)).to(dev))
    P = torch.empty(N * m, dtype=torch.float64, device=dev)
    prob.stencil_setup(t, nS, P)
    torch.cuda.synchronize()
    out = P.cpu().numpy().reshape(N, m)
    tab = prob.get_tables() if tables else None
    prob.close()
    return (out, tab) if tables else out


def rows_from_tables(v, S, idx, alpha, C, t):
    """P[j, a] = alpha[a] + C[a] (v[j + a] - s_j) on the host, one rounding per
    operation in the kernels' order (Sec. 4.1)."""
    d = v.ndim
    offs = O.offsets(d, t)
    N = v.size
    vj = np.stack([np.roll(v, tuple(-o), axis=tuple(range(d))).reshape(-1) for o in offs], axis=1)
    s = S[idx][:, None]
    return alpha[idx] + C[idx] * (vj - s)


@pytest.mark.parametrize("d,n,leaf,nS,seed", [(2, 64, 8, 4, 0), (2, 32, 4, 3, 1),
                                             (3, 16, 8, 4, 2)])
def test_nd_rows_are_the_uniform_rows_of_their_radius(torch_dev, d, n, leaf, nS, seed):
    print(f"[nd setup] d={d} n={n} leaf={leaf} nS={nS}", flush=True)
    r = np.random.default_rng(seed)
    v = r.uniform(-8.0 * n * n, -1.5 * n * n, (n,) * d)
    prob, P, idx = run_nd(torch_dev, v, leaf, nS)
    tm = O.nd_tmap(d, n, leaf, 2).reshape(-1)
    offs = O.offsets(d, 2)
    inner = np.all(np.abs(offs) <= 1, axis=1)
    P1, tab1 = uniform(torch_dev, v, 1, nS, tables=True)
    P2 = uniform(torch_dev, v, 2, nS)
    two, one = tm == 2, tm == 1
    assert two.any() and one.any()
    assert np.array_equal(P[two], P2[two])
    # radius 1: the row formula on this setup's radius-1 tables, bit for bit
    t1 = prob.get_tables_nd1()
    S = prob.get_tables()["S"]
    R1 = rows_from_tables(v, S, idx, t1["alpha"], t1["C"], 1)
    assert np.array_equal(P[np.ix_(one, inner)], R1[one])
    assert np.all(P[np.ix_(one, ~inner)] == 0.0)
    # ... and those tables are the uniform radius-1 tables up to the order of
    # the Green's sums (well-separated 2D/3D null vectors: a plain bound)
    for key, tol in (("g", 1e-13), ("gamma", 1e-13), ("alpha", 1e-10), ("C", 1e-10)):
        a, b = t1[key].reshape(len(S), -1), tab1[key].reshape(len(S), -1)
        assert np.linalg.norm(a - b) <= tol * np.linalg.norm(b), key
    assert np.linalg.norm(P[np.ix_(one, inner)] - P1[one]) <= 1e-10 * np.linalg.norm(P1[one])
    assert np.array_equal(idx, O.assign_shifts(v, O.shift_list(v, nS)).reshape(-1))
    if d == 2:
        # (the uniform setups carry the conditioning-aware comparison with the
        # oracle; 2D alpha is well separated, so a plain bound holds here)
        ref = O.nd_setup(v, leaf, 2, nS)
        assert np.linalg.norm(P - ref["P"]) <= 1e-8 * np.linalg.norm(ref["P"])
    prob.close()


def test_nd_c_apply_uses_per_point_rows(torch_dev):
    """z = C r with C[j, mu_j^{t_j}] = C^{t_j}_{s_j}: against the sparse rows
    built from the setup's own tables of both radii, to 1e-13."""
    torch, dev = torch_dev
    lsp = lsp_mod()
    p = W.helm2d_cross(64)
    prob, P, idx = run_nd(torch_dev, p.v, 8, p.num_shifts)
    C1 = prob.get_tables_nd1()["C"]
    C2 = prob.get_tables()["C"]
    tm = O.nd_tmap(2, p.n, 8, 2).reshape(-1)
    offs = O.offsets(2, 2)
    inner = np.all(np.abs(offs) <= 1, axis=1)
    Crows = np.zeros((p.N, 25))
    Crows[tm == 2] = C2[idx[tm == 2]]
    Crows[np.ix_(tm == 1, inner)] = C1[idx[tm == 1]]
    Cm = O.sparse_rows(Crows, 2, p.n, offs)
    r = np.random.default_rng(5)
    x = r.standard_normal(p.N) + 1j * r.standard_normal(p.N)
    xt = torch.from_numpy(x).to(dev)
    zt = torch.empty_like(xt)
    prob.c_apply(xt, zt)
    z = zt.cpu().numpy()
    z_ref = Cm @ x
    assert np.linalg.norm(z - z_ref) <= 1e-13 * np.linalg.norm(z_ref)
    prob.close()


def test_nd_precond_solve(torch_dev):
    """GMRES(40) with the per-point radius (leaf box 8, t <= 2) on the cross
    profile at n = 128: iterations within +-1 of the oracle's."""
    torch, dev = torch_dev
    lsp = lsp_mod()
    p = W.helm2d_cross(128)
    prob, P, idx = run_nd(torch_dev, p.v, 8, p.num_shifts)
    solve = lsp.host_lu_solver(P, 2, p.n, 2)
    ft = torch.from_numpy(p.f.reshape(-1)).to(dev)
    ut = torch.zeros_like(ft)
    code, iters, relres = prob.precond_solve(ft, ut, solve, rtol=1e-8, restart=40, maxit=200)
    assert code == lsp.LSP_OK and relres <= 1e-8
    _, it_or, _, rel_or, _ = O.precond_solve(p.v, p.f, 2, p.num_shifts, rtol=1e-8, nd_leaf=8)
    print(f"[gmres nd] gpu iters {iters} relres {relres:.2e}; oracle {it_or} {rel_or:.2e}",
          flush=True)
    assert abs(iters - it_or) <= 1
    prob.close()


def test_nd_rejects_bad_leaf(torch_dev):
    torch, dev = torch_dev
    lsp = lsp_mod()
    prob = lsp.Problem(2, 32, torch.full((1024,), -500.0, dtype=torch.float64, device=dev))
    P = torch.empty(1024 * 25, dtype=torch.float64, device=dev)
    for leaf in (1, 3, 64):
        with pytest.raises(lsp.LSPError):
            prob.stencil_setup_nd(leaf, 2, P)
    prob.close()
