"""3D with t = 2 (125-point stencils, Gram blocks of 27, 18, 12 and 8 in the
parity basis): parity of the setup, its non-localized form and GMRES with the
oracle through the C ABI, tolerances as in test_gpu_parity; the learned and
batched forms reject the shape."""
import numpy as np
import pytest

from oracle import lsp_oracle as O
from paper_1607_02560_amd import workloads as W
from tests.test_gpu_parity import check_setup, gpu_setup, lsp_mod, torch_dev  # noqa: F401

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,nS,seed", [(8, 2, 0), (16, 4, 1), (32, 8, 2)])
def test_setup_3d_t2_random_potential(torch_dev, n, nS, seed):
    r = np.random.default_rng(seed)
    v = r.uniform(-8.0 * n * n, -1.5 * n * n, (n,) * 3)
    check_setup(torch_dev, v, 2, nS)


def test_setup_3d_t2_helmholtz(torch_dev):
    """The 3D Helmholtz field at n = 64 with t = 2 and |S| = 16."""
    p = W.helm3d_random(64, t=2)
    check_setup(torch_dev, p.v, p.t, p.num_shifts)


def test_setup_3d_t2_non_localized(torch_dev):
    p = W.helm3d_gauss(32, t=2)
    check_setup(torch_dev, p.v, p.t, 0, global_=True)


def test_precond_solve_3d_t2(torch_dev):
    """GMRES(40) with 5x5x5 stencils on the 3D Helmholtz field at n = 16:
    iterations within +-1 of the oracle's, true residual <= 1e-8."""
    torch, dev = torch_dev
    lsp = lsp_mod()
    p = W.helm3d_random(16, t=2)
    prob, P, idx, tab = gpu_setup(torch_dev, p.v, p.t, p.num_shifts)
    solve = lsp.host_lu_solver(P, 3, p.n, p.t)
    ft = torch.from_numpy(p.f.reshape(-1)).to(dev)
    ut = torch.zeros_like(ft)
    code, iters, relres = prob.precond_solve(ft, ut, solve, rtol=1e-8, restart=40, maxit=200)
    assert code == lsp.LSP_OK
    _, it_or, _, rel_or, _ = O.precond_solve(p.v, p.f, p.t, p.num_shifts, rtol=1e-8)
    print(f"[gmres 3d t=2] gpu iters {iters} relres {relres:.2e}; oracle {it_or} {rel_or:.2e}",
          flush=True)
    assert abs(iters - it_or) <= 1 and relres <= 1e-8


def test_3d_t2_learned_and_batched_are_rejected(torch_dev):
    torch, dev = torch_dev
    lsp = lsp_mod()
    n, m = 16, 125
    prob = lsp.Problem(3, n, torch.full((n ** 3,), -900.0, dtype=torch.float64, device=dev))
    P = torch.empty(n ** 3 * m, dtype=torch.float64, device=dev)
    fb = torch.empty(n ** 3, dtype=torch.int32, device=dev)
    net = lsp.MLP(m + 2, 32, 2 * m, batch_rows=256)
    with pytest.raises(lsp.LSPError) as ei:
        prob.stencil_setup_learned(net, 2, 4, 1e-3, P, fb)
    assert ei.value.code == lsp.LSP_EINVAL
    net.close()
    b = lsp.Batch([prob])
    with pytest.raises(lsp.LSPError) as ei:
        b.stencil_setup(2, [4], [P])
    assert ei.value.code == lsp.LSP_EINVAL
    b.close()
    prob.close()
