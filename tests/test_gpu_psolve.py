"""The device P-solve (nested-dissection factors of P, Sec. 3 and Fig. 1,
applied level by level on the device) and the device GMRES built on it
(eq. (PC), Sec. 5: GMRES(40) with right preconditioner P^-1 C), through the C
ABI.

The P-solve is compared with the plain definition x = P^-1 r (scipy's sparse
direct solve of the same rows) and with the host solve of the same factors;
GMRES with the oracle's iteration counts (within one) and with the dense
solve of eq. (dmodel); the graph-captured step with the directly launched one
(the same kernels in the same order: bit for bit)."""
import os

import numpy as np
import pytest
import scipy.sparse
import scipy.sparse.linalg

from oracle import lsp_oracle as O
from paper_1607_02560_amd import nd
from paper_1607_02560_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    return torch, torch.device("cuda:0")


def lsp_mod():
    from paper_1607_02560_amd import lsp
    return lsp


def sparse_rows(rows, d, n, t):
    """The N x N matrix of the (N, m) stencil rows, columns j + a, a in [-t, t]^d."""
    lsp = lsp_mod()
    N, m = rows.shape
    cols = lsp.export_pattern(d, n, t)
    P = scipy.sparse.csr_matrix((rows.reshape(-1), cols.reshape(-1), np.arange(0, N * m + 1, m)),
                                shape=(N, N))
    P.eliminate_zeros()
    return P


def setup(torch_dev, p, t, nd_leaf=None, stream=None, leaf=None):
    """Problem, its P rows (host) and the nested-dissection factors of P
    (leaf box `leaf`, else the per-point radius's leaf box, else 8)."""
    torch, dev = torch_dev
    lsp = lsp_mod()
    d, n = p.d, p.n
    vt = torch.from_numpy(np.ascontiguousarray(p.v).reshape(-1)).to(dev)
    prob = lsp.Problem(d, n, vt, stream=stream)
    m = (2 * t + 1) ** d
    P = torch.empty(p.N * m, dtype=torch.float64, device=dev)
    if nd_leaf:
        prob.stencil_setup_nd(nd_leaf, p.num_shifts, P)
    else:
        prob.stencil_setup(t, p.num_shifts, P)
    torch.cuda.synchronize()
    rows = P.cpu().numpy().reshape(p.N, m)
    S = sparse_rows(rows, d, n, t)
    F = nd.factor(S, d, n, leaf or nd_leaf or 8)
    prob.psolve_upload(F)
    return prob, S, F


def rand_c(N, seed):
    r = np.random.default_rng(seed)
    return r.standard_normal(N) + 1j * r.standard_normal(N)


@pytest.mark.parametrize("name,t,leaf", [("gauss32", 1, None), ("cross128", 1, None),
                                         ("cross128_nd", 2, 8), ("cross256", 1, None)])
def test_device_psolve(torch_dev, name, t, leaf):
    torch, dev = torch_dev
    p = {"gauss32": lambda: W.helm2d_gauss(32), "cross128": lambda: W.helm2d_cross(128),
         "cross128_nd": lambda: W.helm2d_cross(128),
         "cross256": lambda: W.helm2d_cross(256)}[name]()
    print(f"[psolve] {name} n={p.n} t={t} leaf={leaf}", flush=True)
    prob, S, F = setup(torch_dev, p, t, nd_leaf=leaf)
    x = rand_c(p.N, 3)
    rt = torch.from_numpy(x).to(dev)
    zt = torch.full_like(rt, complex(float("nan"), 0.0))
    prob.psolve_apply(rt, zt)
    torch.cuda.synchronize()
    z = zt.cpu().numpy()
    ref = scipy.sparse.linalg.spsolve(S.tocsc().astype(np.complex128), x)
    rel = np.linalg.norm(z - ref) / np.linalg.norm(ref)
    res = np.linalg.norm(S @ z - x) / np.linalg.norm(x)
    host = F.solve(x)
    rel_host = np.linalg.norm(z - host) / np.linalg.norm(host)
    print(f"  rel to spsolve {rel:.2e}, residual {res:.2e}, rel to host ND solve {rel_host:.2e}")
    # the bounds of the host factorisation's own pin against spsolve
    assert rel <= 1e-9 and res <= 1e-11 and rel_host <= 1e-12
    # fixed-order sums: a second solve is bit-identical
    z2 = torch.empty_like(rt)
    prob.psolve_apply(rt, z2)
    torch.cuda.synchronize()
    assert np.array_equal(z2.cpu().numpy(), z)
    prob.close()


@pytest.mark.parametrize("leaf,t", [(4, 1), (8, 2)])
def test_device_psolve_3d(torch_dev, leaf, t):
    """3D (n = 16, three merge axes, separator planes): uniform t = 1 rows with
    leaf box 4, and the per-point radius with leaf box 8; the device solve
    against scipy's direct solve and the host solve of the same factors, and
    device GMRES against the oracle's count."""
    torch, dev = torch_dev
    lsp = lsp_mod()
    p = W.helm3d_random(16)
    print(f"[psolve 3d] n=16 leaf={leaf} t={t}", flush=True)
    if t == 2:
        prob, S, F = setup(torch_dev, p, 2, nd_leaf=leaf)
    else:
        prob, S, F = setup(torch_dev, p, 1, leaf=leaf)
    x = rand_c(p.N, 7)
    zt = torch.empty(p.N, dtype=torch.complex128, device=dev)
    prob.psolve_apply(torch.from_numpy(x).to(dev), zt)
    torch.cuda.synchronize()
    z = zt.cpu().numpy()
    ref = scipy.sparse.linalg.spsolve(S.tocsc().astype(np.complex128), x)
    assert np.linalg.norm(z - ref) <= 1e-9 * np.linalg.norm(ref)
    host = F.solve(x)
    assert np.linalg.norm(z - host) <= 1e-12 * np.linalg.norm(host)
    ft = torch.from_numpy(p.f.reshape(-1)).to(dev)
    ut = torch.zeros_like(ft)
    code, iters, relres = prob.precond_solve_device(ft, ut, rtol=1e-8, restart=40, maxit=200)
    assert code == lsp.LSP_OK and relres <= 1e-8
    if t == 2:
        _, it_or, _, _, _ = O.precond_solve(p.v, p.f, 2, p.num_shifts, rtol=1e-8, nd_leaf=leaf)
    else:
        _, it_or, _, _, _ = O.precond_solve(p.v, p.f, 1, p.num_shifts, rtol=1e-8)
    print(f"  device gmres {iters} (oracle {it_or}), relres {relres:.2e}", flush=True)
    assert abs(iters - it_or) <= 1
    prob.close()


def test_device_gmres_rejects_nonfinite_rhs(torch_dev):
    torch, dev = torch_dev
    lsp = lsp_mod()
    p = W.helm2d_gauss(32)
    prob, S, F = setup(torch_dev, p, 1)
    ft = torch.from_numpy(p.f.reshape(-1)).to(dev)
    ft[17] = complex(float("nan"), 0.0)
    with pytest.raises(lsp.LSPError) as ei:
        prob.precond_solve_device(ft, torch.zeros_like(ft))
    assert ei.value.code == lsp.LSP_ENONFINITE
    prob.close()


def test_device_psolve_leaf4_level_count(torch_dev):
    """Leaf box 4 at n = 64: more levels and more fronts than leaf 8; the
    per-level launches still reproduce the plain solve."""
    torch, dev = torch_dev
    lsp = lsp_mod()
    p = W.helm2d_cross(64)
    vt = torch.from_numpy(p.v.reshape(-1)).to(dev)
    prob = lsp.Problem(2, 64, vt)
    P = torch.empty(p.N * 9, dtype=torch.float64, device=dev)
    prob.stencil_setup(1, p.num_shifts, P)
    torch.cuda.synchronize()
    S = sparse_rows(P.cpu().numpy().reshape(p.N, 9), 2, 64, 1)
    F = nd.factor(S, 2, 64, 4)
    assert len(F.levels()) > len(nd.factor(S, 2, 64, 8).levels())
    prob.psolve_upload(F)
    x = rand_c(p.N, 5)
    zt = torch.empty(p.N, dtype=torch.complex128, device=dev)
    prob.psolve_apply(torch.from_numpy(x).to(dev), zt)
    torch.cuda.synchronize()
    ref = scipy.sparse.linalg.spsolve(S.tocsc().astype(np.complex128), x)
    assert np.linalg.norm(zt.cpu().numpy() - ref) <= 1e-9 * np.linalg.norm(ref)
    prob.close()


def test_device_gmres_c1(torch_dev):
    """C1 (2D Gaussian Helmholtz field, n = 32, t = 1): iterations within one
    of the oracle's, true residual <= 1e-8, u equal to the dense solve."""
    torch, dev = torch_dev
    lsp = lsp_mod()
    p = W.helm2d_gauss(32)
    prob, S, F = setup(torch_dev, p, 1)
    ft = torch.from_numpy(p.f.reshape(-1)).to(dev)
    ut = torch.zeros_like(ft)
    code, iters, relres = prob.precond_solve_device(ft, ut, rtol=1e-8, restart=40, maxit=200)
    assert code == lsp.LSP_OK
    _, it_or, _, rel_or, _ = O.precond_solve(p.v, p.f, 1, p.num_shifts, rtol=1e-8)
    print(f"[device gmres C1] iters {iters} relres {relres:.2e}; oracle {it_or} {rel_or:.2e}",
          flush=True)
    assert abs(iters - it_or) <= 1
    assert relres <= 1e-8
    u_ref = np.linalg.solve(O.dense_operator(p.v), p.f.reshape(-1))
    assert np.linalg.norm(ut.cpu().numpy() - u_ref) <= 1e-6 * np.linalg.norm(u_ref)
    prob.close()


@pytest.mark.parametrize("nd_leaf", [None, 8])
def test_device_gmres_cross(torch_dev, nd_leaf):
    """Cross profile, n = 128: uniform t = 1 and the per-point radius of
    Sec. 4.2 (leaf box 8, t_j <= 2), each factorised by nested dissection;
    iterations within one of the oracle's solve of the same setup."""
    torch, dev = torch_dev
    lsp = lsp_mod()
    p = W.helm2d_cross(128)
    t = 2 if nd_leaf else 1
    prob, S, F = setup(torch_dev, p, t, nd_leaf=nd_leaf)
    ft = torch.from_numpy(p.f.reshape(-1)).to(dev)
    ut = torch.zeros_like(ft)
    code, iters, relres = prob.precond_solve_device(ft, ut, rtol=1e-8, restart=40, maxit=200)
    assert code == lsp.LSP_OK and relres <= 1e-8
    if nd_leaf:
        _, it_or, _, rel_or, _ = O.precond_solve(p.v, p.f, 2, p.num_shifts, rtol=1e-8,
                                                 nd_leaf=nd_leaf)
    else:
        _, it_or, _, rel_or, _ = O.precond_solve(p.v, p.f, 1, p.num_shifts, rtol=1e-8)
    print(f"[device gmres cross leaf={nd_leaf}] iters {iters} relres {relres:.2e}; "
          f"oracle {it_or} {rel_or:.2e}", flush=True)
    assert abs(iters - it_or) <= 1
    prob.close()


def test_device_gmres_matches_host_loop(torch_dev):
    """The device solve and lsp_precond_solve (host loop, host P-solve by the
    same factors) take the same number of steps and agree to rounding."""
    torch, dev = torch_dev
    p = W.helm2d_cross(128)
    prob, S, F = setup(torch_dev, p, 1)
    ft = torch.from_numpy(p.f.reshape(-1)).to(dev)
    u_dev = torch.zeros_like(ft)
    u_host = torch.zeros_like(ft)
    _, it_d, rel_d = prob.precond_solve_device(ft, u_dev, rtol=1e-10, restart=40, maxit=200)
    _, it_h, rel_h = prob.precond_solve(ft, u_host, F.solve, rtol=1e-10, restart=40, maxit=200)
    print(f"[device vs host loop] {it_d} vs {it_h}; relres {rel_d:.2e} vs {rel_h:.2e}")
    assert abs(it_d - it_h) <= 1
    a, b = u_dev.cpu().numpy(), u_host.cpu().numpy()
    assert np.linalg.norm(a - b) <= 1e-8 * np.linalg.norm(b)
    prob.close()


def test_device_gmres_restart_and_graph_replay(torch_dev):
    """A short restart (several cycles) on a non-default stream, where the
    Arnoldi steps run from captured graphs: the first solve captures, the
    second replays, and a problem with graphs off launches directly; all
    three give bit-identical u and the same count."""
    torch, dev = torch_dev
    lsp = lsp_mod()
    p = W.helm2d_cross(128)
    stream = torch.cuda.Stream(device=dev)
    ft = torch.from_numpy(p.f.reshape(-1)).to(dev)
    results = []
    old = os.environ.get("LSP_GRAPHS")
    try:
        for graphs in ("1", "0"):
            os.environ["LSP_GRAPHS"] = graphs
            prob, S, F = setup(torch_dev, p, 1, stream=stream)
            for rep in range(2 if graphs == "1" else 1):
                ut = torch.zeros_like(ft)
                torch.cuda.synchronize()
                code, iters, relres = prob.precond_solve_device(ft, ut, rtol=1e-9, restart=5,
                                                                maxit=400)
                torch.cuda.synchronize()
                assert code == lsp.LSP_OK and relres <= 1e-9
                print(f"[graph {graphs} rep {rep}] iters {iters} relres {relres:.2e}", flush=True)
                results.append((iters, ut.cpu().numpy()))
            prob.close()
    finally:
        if old is None:
            os.environ.pop("LSP_GRAPHS", None)
        else:
            os.environ["LSP_GRAPHS"] = old
    assert len({r[0] for r in results}) == 1
    for it, u in results[1:]:
        assert np.array_equal(u, results[0][1])


def test_device_gmres_zero_rhs_and_maxit(torch_dev):
    torch, dev = torch_dev
    lsp = lsp_mod()
    p = W.helm2d_gauss(32)
    prob, S, F = setup(torch_dev, p, 1)
    z = torch.zeros(p.N, dtype=torch.complex128, device=dev)
    u = torch.full_like(z, 1.0)
    code, iters, relres = prob.precond_solve_device(z, u, rtol=1e-8)
    assert code == lsp.LSP_OK and iters == 0 and relres == 0.0
    ft = torch.from_numpy(p.f.reshape(-1)).to(dev)
    code, iters, relres = prob.precond_solve_device(ft, u, rtol=1e-14, restart=3, maxit=4)
    assert code == lsp.LSP_NOT_CONVERGED and iters == 4 and relres > 1e-14
    prob.close()


def test_psolve_state_and_validation(torch_dev):
    """Calls before an upload, and factors whose offsets or indices are out
    of range, are refused on the host before anything is launched."""
    torch, dev = torch_dev
    lsp = lsp_mod()
    p = W.helm2d_gauss(32)
    vt = torch.from_numpy(p.v.reshape(-1)).to(dev)
    prob = lsp.Problem(2, 32, vt)
    P = torch.empty(p.N * 9, dtype=torch.float64, device=dev)
    prob.stencil_setup(1, p.num_shifts, P)
    r = torch.ones(p.N, dtype=torch.complex128, device=dev)
    z = torch.empty_like(r)
    with pytest.raises(lsp.LSPError) as ei:
        prob.psolve_apply(r, z)
    assert ei.value.code == lsp.LSP_ESTATE
    with pytest.raises(lsp.LSPError) as ei:
        prob.precond_solve_device(r, z)
    assert ei.value.code == lsp.LSP_ESTATE
    torch.cuda.synchronize()
    F = nd.factor(sparse_rows(P.cpu().numpy().reshape(p.N, 9), 2, 32, 1), 2, 32, 8)
    good = F.export()
    for key, bad in (("idx_F", lambda a: np.where(a == a.max(), p.N, a)),
                     ("off_blk", lambda a: a + (10 ** 9)),
                     ("upd_pos", lambda a: a - 1),
                     ("lev_fronts", lambda a: a[::-1].copy())):
        ex = dict(good)
        ex[key] = bad(good[key])
        with pytest.raises(lsp.LSPError) as ei:
            prob.psolve_upload(ex)
        assert ei.value.code == lsp.LSP_EINVAL, key
    ex = dict(good)
    ex["off_F"] = good["off_F"].copy()
    ex["off_F"][-1] += 1
    with pytest.raises(lsp.LSPError):
        prob.psolve_upload(ex)
    # a failed upload leaves no factors behind, a good one works
    with pytest.raises(lsp.LSPError):
        prob.psolve_apply(r, z)
    prob.psolve_upload(good)
    prob.psolve_apply(r, z)
    torch.cuda.synchronize()
    assert np.all(np.isfinite(z.cpu().numpy()))
    prob.close()
