"""Launch-shape tuning (lsp_autotune, lsp_set_tuning) through the C ABI.

Every candidate shape must compute what the default computes: the assembly
tiles the same rows bit for bit; the Green's-sum wave count and the apply's
line transform only reorder sums, so tables, rows and outputs agree to
rounding (the bounds are those of the FP64 sums: 1e-13 relative on the
Green's values and the apply; the rows move with the null vectors, which FP64
data fix to about eps kappa_s, the conditioning bound of the parity tests)."""
import numpy as np
import pytest

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


def run(torch_dev, prob, p, t, P, idx, precision=0):
    torch, dev = torch_dev
    prob.stencil_setup(t, p.num_shifts, P, idx, precision=precision)
    tab = prob.get_tables()
    torch.cuda.synchronize()
    return P.cpu().numpy().copy(), idx.cpu().numpy().copy(), tab


def rel(a, b):
    a = np.asarray(a)
    return np.linalg.norm(a.astype(np.result_type(a, b, np.float64)) - b) / np.linalg.norm(b)


def row_bound(tab):
    """Rows move with alpha, which FP64 data fix only to about eps kappa_s,
    kappa_s = lambda_max / (lambda_2 - lambda_1) of the shift's Gram matrix
    (Davis-Kahan, as in the parity tests)."""
    kap = 0.0
    for M in tab["M"]:
        lam = np.linalg.eigvalsh(0.5 * (M + M.T))
        kap = max(kap, lam[-1] / max(lam[1] - lam[0], 1e-300))
    return max(1e-9, 20 * np.finfo(np.float64).eps * kap)


@pytest.mark.parametrize("n", [256, 1024])
def test_every_shape_computes_the_same(torch_dev, n):
    torch, dev = torch_dev
    lsp = lsp_mod()
    p = W.helm2d_random(n)
    t, m = p.t, (2 * p.t + 1) ** 2
    print(f"[tuning] n={n} t={t} |S|={p.num_shifts}", flush=True)
    prob = lsp.Problem(2, n, torch.from_numpy(p.v.reshape(-1)).to(dev))
    P = torch.empty(p.N * m, dtype=torch.float64, device=dev)
    P32 = torch.empty(p.N * m, dtype=torch.float32, device=dev)
    idx = torch.empty(p.N, dtype=torch.int32, device=dev)
    u = torch.from_numpy(p.f.reshape(-1)).to(dev)
    y = torch.empty_like(u)
    P0, i0, tab0 = run(torch_dev, prob, p, t, P, idx)
    P032, _, _ = run(torch_dev, prob, p, t, P32, idx, precision=lsp.LSP_FP32_REFINE)
    prob.ps_apply(u, y)
    torch.cuda.synchronize()
    y0 = y.cpu().numpy().copy()
    for tile in (32, 64, 128, 1):
        prob.set_tuning(assembly_tile=tile)
        P1, i1, _ = run(torch_dev, prob, p, t, P, idx)
        assert np.array_equal(P1, P0) and np.array_equal(i1, i0), tile
        P132, _, _ = run(torch_dev, prob, p, t, P32, idx, precision=lsp.LSP_FP32_REFINE)
        assert np.array_equal(P132, P032), tile
    bound = row_bound(tab0)
    print(f"  row bound {bound:.2e}", flush=True)
    for waves in (512, 1024, 1536, 2048, 3072):
        prob.set_tuning(green_waves=waves)
        P1, i1, tab1 = run(torch_dev, prob, p, t, P, idx)
        assert np.array_equal(i1, i0)
        assert rel(tab1["g"], tab0["g"]) <= 1e-13 and rel(tab1["gamma"], tab0["gamma"]) <= 1e-13
        assert rel(P1, P0) <= bound, (waves, rel(P1, P0))
    for form in (8, 16):
        prob.set_tuning(apply_form=form)
        prob.ps_apply(u, y)
        torch.cuda.synchronize()
        assert rel(y.cpu().numpy(), y0) <= 1e-13, form
    prob.set_tuning()
    ch = prob.autotune(t, p.num_shifts, P, u, y, reps=3)
    print(f"  autotune: {ch}", flush=True)
    assert ch["green_waves"][0] in (512, 1024, 1536, 2048, 3072)
    assert ch["assembly_tile"][0] in (32, 64, 128, 1)
    assert ch["apply_form"][0] in (8, 16)
    assert prob.get_tuning() == {k: v[0] for k, v in ch.items()}
    # the tuned problem still sets up and applies within the bounds above
    P1, i1, _ = run(torch_dev, prob, p, t, P, idx)
    assert np.array_equal(i1, i0) and rel(P1, P0) <= bound
    prob.ps_apply(u, y)
    torch.cuda.synchronize()
    assert rel(y.cpu().numpy(), y0) <= 1e-13
    prob.close()


def test_invalid_tuning_refused(torch_dev):
    torch, dev = torch_dev
    lsp = lsp_mod()
    prob = lsp.Problem(2, 64, torch.full((64 * 64,), -500.0, dtype=torch.float64, device=dev))
    for kw in ({"green_waves": 100}, {"assembly_tile": 48}, {"apply_form": 4}):
        with pytest.raises(lsp.LSPError) as ei:
            prob.set_tuning(**kw)
        assert ei.value.code == lsp.LSP_EINVAL
    assert prob.get_tuning() == {"green_waves": 0, "assembly_tile": 0, "apply_form": 0}
    prob.close()
