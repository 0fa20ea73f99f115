"""GPU tests of the batched form (lsp_batch_*): one launch per setup stage over
many problems of uneven n.

Every problem of a batch must receive exactly (bit for bit) the tables, rows
and s_j of its own single-problem setup, which the parity suite checks against
the FP64 oracle; the batched apply must equal the single apply bit for bit.
"""
import numpy as np
import pytest

from oracle import lsp_oracle as O
from paper_1607_02560_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    return torch, torch.device("cuda:0")


def make_problems(torch_dev, fields, stream):
    torch, dev = torch_dev
    from paper_1607_02560_amd import lsp
    probs = []
    for v in fields:
        vt = torch.from_numpy(np.ascontiguousarray(v).reshape(-1)).to(dev)
        probs.append(lsp.Problem(v.ndim, v.shape[0], vt, stream=stream))
    return probs


def single_setup(torch_dev, v, t, nS, precision, stream):
    torch, dev = torch_dev
    from paper_1607_02560_amd import lsp
    d, n = v.ndim, v.shape[0]
    N, m = n ** d, (2 * t + 1) ** d
    prob = make_problems(torch_dev, [v], stream)[0]
    P = torch.full((N * m,), float("nan"), dtype=torch.float32 if precision else torch.float64,
                   device=dev)
    idx = torch.full((N,), -1, dtype=torch.int32, device=dev)
    torch.cuda.synchronize()  # the fills run on torch's stream, the setup on `stream`
    prob.stencil_setup(t, 0 if nS is None else nS, P, idx, precision=precision)
    tabs = prob.get_tables()
    torch.cuda.synchronize()
    out = (P.cpu().numpy(), idx.cpu().numpy(), tabs)
    prob.close()
    return out


def run_batch(torch_dev, fields, t, nS, precision, stream, probs=None):
    torch, dev = torch_dev
    from paper_1607_02560_amd import lsp
    if probs is None:
        probs = make_problems(torch_dev, fields, stream)
    batch = lsp.Batch(probs)
    Ps, idxs = [], []
    for p in probs:
        m = (2 * t + 1) ** p.d
        Ps.append(torch.full((p.N * m,), float("nan"),
                             dtype=torch.float32 if precision else torch.float64, device=dev))
        idxs.append(torch.full((p.N,), -1, dtype=torch.int32, device=dev))
    torch.cuda.synchronize()  # the fills run on torch's stream, the setup on `stream`
    batch.stencil_setup(t, nS, Ps, idxs, precision=precision)
    torch.cuda.synchronize()
    return batch, probs, Ps, idxs


def check_equal_to_singles(torch_dev, fields, t, nS, precision, stream, batch, probs, Ps, idxs):
    for i, v in enumerate(fields):
        P1, i1, tab1 = single_setup(torch_dev, v, t, None if nS is None else nS[i], precision,
                                    stream)
        assert np.array_equal(Ps[i].cpu().numpy(), P1, equal_nan=False), i
        assert np.array_equal(idxs[i].cpu().numpy(), i1), i
        tab = probs[i].get_tables()
        for key in ("S", "alpha", "C", "sigma_min", "g", "gamma", "M"):
            assert np.array_equal(tab[key], tab1[key]), (i, key)


SIZES_2D = [16, 32, 64, 128, 256, 64, 32, 128]


@pytest.mark.parametrize("graphs", [True, False])
@pytest.mark.parametrize("precision", [0, 1])
def test_batch_setup_equals_single_setups(torch_dev, graphs, precision, monkeypatch):
    torch, dev = torch_dev
    stream = torch.cuda.Stream()
    monkeypatch.setenv("LSP_GRAPHS", "1" if graphs else "0")  # read at creation
    fields = [W.helm2d_random(n, seed=10 + i, t=2).v for i, n in enumerate(SIZES_2D)]
    nS = [max(1, n // 16) for n in SIZES_2D]
    batch, probs, Ps, idxs = run_batch(torch_dev, fields, 2, nS, precision, stream)
    monkeypatch.delenv("LSP_GRAPHS", raising=False)
    tw, cand, ms = batch.tile()
    print(f"[batch] graphs={graphs} precision={precision} tile {tw} of {cand} ({ms} ms)",
          flush=True)
    assert tw in cand and all(n % c == 0 for n in SIZES_2D for c in cand)
    check_equal_to_singles(torch_dev, fields, 2, nS, precision, stream, batch, probs, Ps, idxs)
    batch.close()
    for p in probs:
        p.close()


def test_batch_replay_with_new_potentials(torch_dev, monkeypatch):
    """Second and third setups of the same batch (graph replays) follow new
    potentials set on the problems."""
    torch, dev = torch_dev
    stream = torch.cuda.Stream()
    sizes = [32, 64, 16]
    fields = [W.helm2d_random(n, seed=i, t=1).v for i, n in enumerate(sizes)]
    monkeypatch.setenv("LSP_GRAPHS", "1")
    batch, probs, Ps, idxs = run_batch(torch_dev, fields, 1, None, 0, stream)
    monkeypatch.delenv("LSP_GRAPHS")
    for rep in range(2):
        new = [W.helm2d_random(n, seed=100 + 10 * rep + i, t=1).v for i, n in enumerate(sizes)]
        for p, v in zip(probs, new):
            p.set_potential(torch.from_numpy(v.reshape(-1)).to(dev))
        torch.cuda.synchronize()
        batch.stencil_setup(1, None, Ps, idxs)
        torch.cuda.synchronize()
        check_equal_to_singles(torch_dev, new, 1, None, 0, stream, batch, probs, Ps, idxs)
    batch.close()
    for p in probs:
        p.close()


def test_batch_3d(torch_dev):
    torch, dev = torch_dev
    stream = torch.cuda.Stream()
    fields = [W.helm3d_random(n, seed=i).v for i, n in enumerate([16, 32, 16])]
    batch, probs, Ps, idxs = run_batch(torch_dev, fields, 1, [4, 8, 2], 0, stream)
    check_equal_to_singles(torch_dev, fields, 1, [4, 8, 2], 0, stream, batch, probs, Ps, idxs)
    batch.close()
    for p in probs:
        p.close()


@pytest.mark.parametrize("graphs", [True, False])
def test_batch_ps_apply(torch_dev, graphs, monkeypatch):
    torch, dev = torch_dev
    stream = torch.cuda.Stream()
    sizes = [16, 64, 256, 1024, 32]
    fields = [W.helm2d_random(n, seed=i, t=2).v for i, n in enumerate(sizes)]
    probs = make_problems(torch_dev, fields, stream)
    from paper_1607_02560_amd import lsp
    monkeypatch.setenv("LSP_GRAPHS", "1" if graphs else "0")
    batch = lsp.Batch(probs)
    monkeypatch.delenv("LSP_GRAPHS", raising=False)
    r = np.random.default_rng(4)
    us = [torch.from_numpy(r.standard_normal(n * n) + 1j * r.standard_normal(n * n)).to(dev)
          for n in sizes]
    ys = [torch.empty_like(u) for u in us]
    for rep in range(3):  # graph capture, then replays
        for y in ys:
            y.fill_(float("nan"))
        torch.cuda.synchronize()  # torch's fills before the library's stream
        batch.ps_apply(us, ys)
        torch.cuda.synchronize()
        for i, p in enumerate(probs):
            y1 = torch.empty_like(us[i])
            p.ps_apply(us[i], y1)
            torch.cuda.synchronize()
            assert torch.equal(ys[i], y1), (rep, i)
    # one against the oracle
    u0 = us[0].cpu().numpy().reshape(16, 16)
    ref = O.ps_apply(fields[0], u0).reshape(-1)
    got = ys[0].cpu().numpy()
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)
    batch.close()
    for p in probs:
        p.close()


def test_batch_problems_solve_after_batched_setup(torch_dev):
    """The per-problem entry points use the tables of a batched setup:
    GMRES(40) with the host LU of the batched P rows reaches 1e-8."""
    torch, dev = torch_dev
    from paper_1607_02560_amd import lsp
    stream = torch.cuda.Stream()
    ps = [W.helm2d_gauss(32), W.helm2d_random(64, seed=3, t=2)]
    batch, probs, Ps, idxs = run_batch(torch_dev, [p.v for p in ps], 1, None, 0, stream)
    for i, p in enumerate(ps):
        prob = probs[i]
        N, m = p.N, 9
        solve = lsp.host_lu_solver(Ps[i].cpu().numpy().reshape(N, m), 2, p.n, 1)
        ft = torch.from_numpy(p.f.reshape(-1)).to(dev)
        ut = torch.zeros_like(ft)
        torch.cuda.synchronize()
        code, iters, relres = prob.precond_solve(ft, ut, solve, rtol=1e-8, restart=40, maxit=400)
        print(f"[batch gmres] problem {i} n={p.n}: {iters} iterations, relres {relres:.1e}",
              flush=True)
        assert code == lsp.LSP_OK and relres <= 1e-8
    batch.close()
    for q in probs:
        q.close()


def test_batch_rejects_bad_arguments(torch_dev):
    torch, dev = torch_dev
    from paper_1607_02560_amd import lsp
    stream = torch.cuda.Stream()
    small = make_problems(torch_dev, [W.helm2d_random(8, seed=0, t=1).v], stream)
    with pytest.raises(lsp.LSPError):
        lsp.Batch(small)
    mixed = make_problems(torch_dev, [W.helm2d_random(16, seed=0, t=1).v,
                                      W.helm3d_random(16, seed=0).v], stream)
    with pytest.raises(lsp.LSPError):
        lsp.Batch(mixed)
    other = make_problems(torch_dev, [W.helm2d_random(16, seed=0, t=1).v], None)
    with pytest.raises(lsp.LSPError):
        lsp.Batch([mixed[0], other[0]])
    # the problems of a batched apply may run concurrently: an output may not
    # be another problem's input or output
    pair = make_problems(torch_dev, [W.helm2d_random(16, seed=i, t=1).v for i in (1, 2)], stream)
    batch = lsp.Batch(pair)
    u = [torch.zeros(256, dtype=torch.complex128, device=dev) for _ in range(2)]
    y = [torch.zeros(256, dtype=torch.complex128, device=dev) for _ in range(2)]
    torch.cuda.synchronize()
    with pytest.raises(lsp.LSPError):
        batch.ps_apply(u, [y[0], y[0]])
    with pytest.raises(lsp.LSPError):
        batch.ps_apply(u, [y[0], u[0]])
    batch.ps_apply(u, y)
    torch.cuda.synchronize()
    batch.close()
    for p in small + mixed + other + pair:
        p.close()


def test_batch_c5_workload(torch_dev):
    """The 64-problem workload with n drawn from {64, 128, 256, 512}, t = 2,
    |S_p| = n_p / 16, FP32 rows: every problem equals its single setup."""
    torch, dev = torch_dev
    stream = torch.cuda.Stream()
    ps = W.batch2d(64, seed=0)
    fields = [p.v for p in ps]
    nS = [p.num_shifts for p in ps]
    batch, probs, Ps, idxs = run_batch(torch_dev, fields, 2, nS, 1, stream)
    print(f"[batch c5] sizes {sorted(set(p.n for p in ps))}, total points "
          f"{sum(p.N for p in ps)}, tile {batch.tile()}", flush=True)
    check_equal_to_singles(torch_dev, fields, 2, nS, 1, stream, batch, probs, Ps, idxs)
    batch.close()
    for p in probs:
        p.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_every_tile_width(torch_dev, precision):
    """Every assembly tile width the tuner may pick (set with
    lsp_batch_set_tile, including the LDS-table form 1) gives each problem
    its single setup's rows bit for bit; widths that do not fit the batch are
    refused before anything is launched."""
    torch, dev = torch_dev
    from paper_1607_02560_amd import lsp
    stream = torch.cuda.Stream()
    sizes = [64, 128, 64, 256]
    fields = [W.helm2d_random(n, seed=30 + i, t=2).v for i, n in enumerate(sizes)]
    nS = [max(1, n // 16) for n in sizes]
    probs = make_problems(torch_dev, fields, stream)
    batch = lsp.Batch(probs)
    Ps, idxs = [], []
    for p in probs:
        Ps.append(torch.empty(p.N * 25, dtype=torch.float32 if precision else torch.float64,
                              device=dev))
        idxs.append(torch.empty(p.N, dtype=torch.int32, device=dev))
    singles = [single_setup(torch_dev, v, 2, nS[i], precision, stream)
               for i, v in enumerate(fields)]
    for tw in (1, 16, 32, 64, 0):
        batch.set_tile(tw)
        for P in Ps:
            P.fill_(float("nan"))
        for ix in idxs:
            ix.fill_(-1)
        torch.cuda.synchronize()
        batch.stencil_setup(2, nS, Ps, idxs, precision=precision)
        torch.cuda.synchronize()
        got_tw = batch.tile()[0]
        print(f"[batch tile] requested {tw}, used {got_tw}", flush=True)
        if tw:
            assert got_tw == tw
        for i in range(len(sizes)):
            assert np.array_equal(Ps[i].cpu().numpy(), singles[i][0]), (tw, i)
            assert np.array_equal(idxs[i].cpu().numpy(), singles[i][1]), (tw, i)
    with pytest.raises(lsp.LSPError) as ei:
        batch.set_tile(48)
    assert ei.value.code == lsp.LSP_EINVAL
    batch.set_tile(128)  # does not divide n = 64: refused at the setup
    with pytest.raises(lsp.LSPError) as ei:
        batch.stencil_setup(2, nS, Ps, idxs, precision=precision)
    assert ei.value.code == lsp.LSP_EINVAL
    batch.close()
    for p in probs:
        p.close()
