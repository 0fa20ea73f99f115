"""GPU tests of the learned-stencil surrogate against the FP64 reference.

Tolerances: the kernels round inputs, weights and activations to BF16
(8 significant bits, unit roundoff 2^-9 ~ 2e-3) and accumulate in FP32.
  * forward: against a reference that rounds at the same points (FP64
    products of the same BF16 values), relative l2 <= 2e-3 (only FP32
    accumulation order and the FP32 exponential differ, which occasionally
    moves an activation by one BF16 step); against the plain FP64 network
    with BF16-rounded weights, relative l2 <= 3e-2.
  * gradients: against the FP64 gradients (oracle, pinned by central
    differences) of the same BF16 weights and inputs, relative l2 <= 5e-2 per
    tensor: the backward pass rounds dY and dZ to BF16 as well.
  * Adam: bit-level agreement up to FP32 rounding of the update.
  * learned setup: fallback rows equal the exact rows bit for bit, kept rows
    equal the network's output bit for bit, and the fallback decision agrees
    with the FP64 residual of the reference wherever it is not within 1e-6
    of the limit.
"""
import numpy as np
import pytest

from oracle import lsp_oracle as O
from oracle import mlp_oracle as MO
from paper_1607_02560_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    return torch, torch.device("cuda:0")


def bf16(x):
    """Round float32 values to the nearest BF16 (ties to even), as float64."""
    a = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    a = (a + 0x7FFF + ((a >> 16) & 1)) & 0xFFFF0000
    return a.astype(np.uint32).view(np.float32).astype(np.float64)


def unflatten(flat, n_in, H, n_out):
    sizes = [("W1", (H, n_in)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)),
             ("W3", (n_out, H)), ("b3", (n_out,))]
    p, k = {}, 0
    for name, shp in sizes:
        cnt = int(np.prod(shp))
        p[name] = np.asarray(flat[k:k + cnt], dtype=np.float64).reshape(shp)
        k += cnt
    return p


def flatten(p):
    return np.concatenate([p[k].reshape(-1) for k in ("W1", "b1", "W2", "b2", "W3", "b3")])


def setup_net(torch_dev, n_in=28, H=128, n_out=54, seed=0, batch=512):
    from paper_1607_02560_amd import lsp
    p = MO.init_params(n_in, H, n_out, seed)
    r = np.random.default_rng(seed + 1)
    for k in ("b1", "b2", "b3"):
        p[k] = r.standard_normal(p[k].shape) * 0.2
    flat = flatten(p).astype(np.float32)
    mlp = lsp.MLP(n_in, H, n_out, batch)
    mlp.set_params(flat)
    mu_x = r.standard_normal(n_in).astype(np.float32)
    sd_x = (0.5 + r.random(n_in)).astype(np.float32)
    mu_y = r.standard_normal(n_out).astype(np.float32)
    sd_y = (0.5 + r.random(n_out)).astype(np.float32)
    mlp.set_normalisation(mu_x, sd_x, mu_y, sd_y)
    pf = unflatten(flat, n_in, H, n_out)
    return mlp, pf, (mu_x, sd_x, mu_y, sd_y)


def standardised_inputs(X, mu, sd):
    return bf16((np.asarray(X, np.float32) - mu) / sd)


def test_forward_matches_reference(torch_dev):
    torch, dev = torch_dev
    mlp, p, (mu_x, sd_x, mu_y, sd_y) = setup_net(torch_dev)
    r = np.random.default_rng(3)
    rows = 300
    X = (mu_x + sd_x * r.standard_normal((rows, 28))).astype(np.float32)
    Xt = torch.from_numpy(X).to(dev)
    Yt = torch.empty((rows, 54), dtype=torch.float32, device=dev)
    mlp.forward(Xt, Yt)
    Y = Yt.cpu().numpy().astype(np.float64)
    Xn = standardised_inputs(X, mu_x, sd_x)
    pb = {k: (bf16(v) if k.startswith("W") else v) for k, v in p.items()}
    # the reference rounded at the kernels' points
    A1 = bf16(MO.silu(Xn @ pb["W1"].T + pb["b1"]))
    A2 = bf16(MO.silu(A1 @ pb["W2"].T + pb["b2"]))
    Ye = mu_y + sd_y * (A2 @ pb["W3"].T + pb["b3"])
    rel = np.linalg.norm(Y - Ye) / np.linalg.norm(Ye)
    # the plain FP64 network with BF16 weights
    Yr, _ = MO.forward(pb, Xn)
    rel64 = np.linalg.norm(Y - (mu_y + sd_y * Yr)) / np.linalg.norm(mu_y + sd_y * Yr)
    print(f"[mlp forward] rel vs rounded reference {rel:.2e}, vs FP64 {rel64:.2e}", flush=True)
    assert rel <= 2e-3
    assert rel64 <= 3e-2
    mlp.close()


def test_gradients_match_reference(torch_dev):
    torch, dev = torch_dev
    mlp, p, (mu_x, sd_x, mu_y, sd_y) = setup_net(torch_dev, seed=5)
    r = np.random.default_rng(6)
    rows = 200  # not a multiple of 16: padded rows must not contribute
    X = (mu_x + sd_x * r.standard_normal((rows, 28))).astype(np.float32)
    T = (mu_y + sd_y * r.standard_normal((rows, 54))).astype(np.float32)
    loss, g = mlp.loss_grad(torch.from_numpy(X).to(dev), torch.from_numpy(T).to(dev))
    gd = unflatten(g, 28, 128, 54)
    Xn = standardised_inputs(X, mu_x, sd_x)
    Tn = (T.astype(np.float64) - mu_y) / sd_y
    pb = {k: (bf16(v) if k.startswith("W") else v) for k, v in p.items()}
    loss_ref, g_ref = MO.loss_and_grads(pb, Xn, Tn)
    print(f"[mlp grad] loss gpu {loss:.6f} ref {loss_ref:.6f}", flush=True)
    assert loss == pytest.approx(loss_ref, rel=1e-2)
    for k in g_ref:
        rel = np.linalg.norm(gd[k] - g_ref[k]) / np.linalg.norm(g_ref[k])
        print(f"   {k}: rel {rel:.2e}", flush=True)
        assert rel <= 5e-2, k
    mlp.close()


def test_adam_step_matches_reference(torch_dev):
    torch, dev = torch_dev
    mlp, p, (mu_x, sd_x, mu_y, sd_y) = setup_net(torch_dev, seed=9)
    r = np.random.default_rng(10)
    rows = 128
    Xt = torch.from_numpy((mu_x + sd_x * r.standard_normal((rows, 28))).astype(np.float32)).to(dev)
    Tt = torch.from_numpy((mu_y + sd_y * r.standard_normal((rows, 54))).astype(np.float32)).to(dev)
    p0 = mlp.get_params().astype(np.float64)
    _, g = mlp.loss_grad(Xt, Tt)
    lr = 2e-3
    mlp.train_step(Xt, Tt, lr)
    p1 = mlp.get_params().astype(np.float64)
    ref = unflatten(p0, 28, 128, 54)
    MO.adam_step(ref, unflatten(g.astype(np.float64), 28, 128, 54), {}, lr)
    ref1 = flatten(ref)
    assert np.all(np.abs(p1 - ref1) <= 1e-6 * np.abs(p0) + 1e-6 * lr)
    mlp.close()


def test_rejects_bad_arguments(torch_dev):
    torch, dev = torch_dev
    from paper_1607_02560_amd import lsp
    with pytest.raises(lsp.LSPError):
        lsp.MLP(28, 100, 54, 64)   # hidden width not a multiple of 16
    mlp = lsp.MLP(4, 16, 3, 32)
    X = torch.zeros((40, 4), dtype=torch.float32, device=dev)
    Y = torch.zeros((40, 3), dtype=torch.float32, device=dev)
    with pytest.raises(lsp.LSPError):
        mlp.forward(X, Y)          # more rows than the batch size
    with pytest.raises(lsp.LSPError):
        mlp.set_normalisation(np.zeros(4), np.zeros(4), np.zeros(3), np.ones(3))  # sd 0
    mlp.close()


# --------------------------------------------------------------- problems ----
def small_problem(torch_dev, n=16, seed=0):
    torch, dev = torch_dev
    from paper_1607_02560_amd import lsp
    p = W.helm3d_random(n, seed=seed)
    prob = lsp.Problem(3, n, torch.from_numpy(p.v.reshape(-1)).to(dev))
    return p, prob


def test_training_rows_match_reference(torch_dev):
    torch, dev = torch_dev
    p, prob = small_problem(torch_dev)
    N, m = p.N, 27
    P = torch.empty(N * m, dtype=torch.float64, device=dev)
    prob.stencil_setup(1, p.num_shifts, P)
    tab = prob.get_tables()
    pts = np.array([0, 5, 777, 4095, 2048], dtype=np.int64)
    X = torch.empty((5, m + 2), dtype=torch.float32, device=dev)
    T = torch.empty((5, 2 * m), dtype=torch.float32, device=dev)
    prob.training_rows(P, torch.from_numpy(pts).to(dev), X, T)
    Xr = MO.features(p.v, 1, tab["S"])[pts].astype(np.float32)
    idx = O.assign_shifts(p.v, tab["S"]).reshape(-1)
    Tr = MO.targets(P.cpu().numpy().reshape(N, m), tab["S"], tab["C"], idx)[pts].astype(np.float32)
    assert np.array_equal(X.cpu().numpy(), Xr)
    assert np.array_equal(T.cpu().numpy(), Tr)
    # an index outside the grid yields NaN rows, not a read
    bad = torch.tensor([N + 3], dtype=torch.int64, device=dev)
    Xb = torch.zeros((1, m + 2), dtype=torch.float32, device=dev)
    Tb = torch.zeros((1, 2 * m), dtype=torch.float32, device=dev)
    prob.training_rows(P, bad, Xb, Tb)
    assert torch.isnan(Xb).all() and torch.isnan(Tb).all()
    prob.close()


def field(d, n, t, seed):
    return W.helm3d_random(n, seed=seed, t=t) if d == 3 else W.helm2d_random(n, seed=seed, t=t)


def trained_net(torch_dev, steps=400, seeds=(1, 2, 3), n=16, d=3, t=1, hidden=128):
    torch, dev = torch_dev
    from paper_1607_02560_amd import lsp
    from paper_1607_02560_amd import surrogate as SG
    fields = [field(d, n, t, s).v for s in seeds]
    X, T = SG.gather_rows(fields, t, 0, 4096, seed=11, device=dev)
    m = (2 * t + 1) ** d
    mlp = lsp.MLP(m + 2, hidden, 2 * m, 1024)
    mlp.set_params(SG.glorot_params(m + 2, hidden, 2 * m, 12))
    mlp.fit_normalisation(X, T)
    hist = SG.train(mlp, X, T, steps, 1024, 3e-3, seed=13, report_every=max(steps // 4, 1),
                    lr_final=3e-4)
    return mlp, hist


def test_training_reduces_loss(torch_dev):
    mlp, hist = trained_net(torch_dev)
    print("[mlp training] loss by step:", [(s, round(l, 5)) for s, l in hist], flush=True)
    assert hist[-1][1] < 0.2 * hist[0][1]
    mlp.close()


# (d, n, t, hidden, shifts): the fused pass serves hidden width 128 with t = 1
# (2D and 3D) and t = 2 (2D) while its per-shift tables fit in LDS; the other
# cases take the chunked path (network batches, then a row kernel): width 64,
# t = 3, and 3D with 96 shifts (too many for the fused pass's LDS). n = 8 in
# 2D leaves most lanes of the fused pass idle. shifts None: the workload's own.
LEARNED_CASES = [(3, 16, 1, 128, None), (3, 16, 1, 64, None), (2, 32, 2, 128, None),
                 (2, 32, 1, 128, None), (2, 8, 1, 128, None), (2, 32, 3, 128, None),
                 (3, 16, 1, 128, 96)]


@pytest.mark.parametrize("d,n,t,hidden,shifts", LEARNED_CASES)
def test_learned_setup_rows_and_fallback(torch_dev, d, n, t, hidden, shifts):
    """Kept rows are the network's output, fallback rows are the exact rows,
    and the decision matches the reference residual rho > rho* + threshold."""
    torch, dev = torch_dev
    from paper_1607_02560_amd import lsp
    mlp, _ = trained_net(torch_dev, steps=200, n=n, d=d, t=t, hidden=hidden)
    p = field(d, n, t, 0)
    nS = p.num_shifts if shifts is None else shifts
    N, m = p.N, (2 * t + 1) ** d
    prob = lsp.Problem(d, n, torch.from_numpy(p.v.reshape(-1)).to(dev))
    Pex = torch.empty(N * m, dtype=torch.float64, device=dev)
    prob.stencil_setup(t, nS, Pex)
    Pl = torch.full((N * m,), float("nan"), dtype=torch.float64, device=dev)
    fb = torch.full((N,), -1, dtype=torch.int32, device=dev)
    thr = 0.01
    nf = prob.stencil_setup_learned(mlp, t, nS, thr, Pl, fb)
    fbh = fb.cpu().numpy()
    assert set(np.unique(fbh)) <= {0, 1} and int(fbh.sum()) == nf
    print(f"[learned setup] d={d} n={n} t={t} hidden={hidden} shifts={nS} threshold {thr}: "
          f"{nf} of {N} rows fall back", flush=True)
    Pl_h = Pl.cpu().numpy().reshape(N, m)
    Pex_h = Pex.cpu().numpy().reshape(N, m)
    sel = fbh == 1
    assert np.array_equal(Pl_h[sel], Pex_h[sel])
    # kept rows are the network's P outputs for the point's features
    tab = prob.get_tables()
    S = tab["S"]
    feats = MO.features(p.v, t, S)
    X = torch.from_numpy(feats.astype(np.float32)).to(dev)
    Y = torch.empty((N, 2 * m), dtype=torch.float32, device=dev)
    for j0 in range(0, N, 1024):
        mlp.forward(X[j0:j0 + 1024], Y[j0:j0 + 1024])
    Yh = Y.cpu().numpy().astype(np.float64)
    assert np.array_equal(Pl_h[~sel], Yh[~sel, :m])
    # decisions against the FP64 reference residual
    idx = O.assign_shifts(p.v, S).reshape(-1)
    offs = O.offsets(d, t)
    tabs = O.shift_tables(d, n, S, t)
    rho_star = [MO.residual(tabs["alpha"][i], tabs["g"][i], tabs["gamma"][i], offs)
                for i in range(len(S))]
    r = np.random.default_rng(17)
    checked = 0
    picks = r.choice(N, min(N, 200), replace=False)
    for j in picks:
        s = S[idx[j]]
        vm = feats[j, 1:m + 1] * n * n - s
        c = Yh[j, m:] / abs(s)
        q = Yh[j, :m] - c * vm
        rho = MO.residual(q, tabs["g"][idx[j]], tabs["gamma"][idx[j]], offs)
        lim = rho_star[idx[j]] + thr
        if abs(rho - lim) > 1e-6:
            assert fbh[j] == (1 if rho > lim else 0), (j, rho, lim)
            checked += 1
    assert checked > 0.75 * len(picks)
    prob.close()
    mlp.close()


def test_learned_setup_c_apply_uses_point_rows(torch_dev):
    """After a learned setup the C-apply uses the per-point C rows: the
    network's C rows where they were kept (threshold 1 keeps every finite
    row), the shift's exact row elsewhere."""
    torch, dev = torch_dev
    from paper_1607_02560_amd import lsp
    mlp, _ = trained_net(torch_dev, steps=100)
    p, prob = small_problem(torch_dev, seed=0)
    N, m = p.N, 27
    Pl = torch.empty(N * m, dtype=torch.float64, device=dev)
    fb = torch.empty(N, dtype=torch.int32, device=dev)
    prob.stencil_setup_learned(mlp, 1, p.num_shifts, 1.0, Pl, fb)  # keeps every finite row
    fbh = fb.cpu().numpy()
    tab = prob.get_tables()
    S = tab["S"]
    idx = O.assign_shifts(p.v, S).reshape(-1)
    X = torch.from_numpy(MO.features(p.v, 1, S).astype(np.float32)).to(dev)
    Y = torch.empty((N, 2 * m), dtype=torch.float32, device=dev)
    for j0 in range(0, N, 1024):
        mlp.forward(X[j0:j0 + 1024], Y[j0:j0 + 1024])
    Yh = Y.cpu().numpy().astype(np.float64)
    Crows = Yh[:, m:] / np.abs(S[idx])[:, None]
    Crows[fbh == 1] = tab["C"][idx[fbh == 1]]
    r = np.random.default_rng(3)
    x = r.standard_normal(N) + 1j * r.standard_normal(N)
    xt = torch.from_numpy(x).to(dev)
    zt = torch.empty_like(xt)
    prob.c_apply(xt, zt)
    z_ref = O.sparse_rows(Crows, 3, 16, O.offsets(3, 1)) @ x
    assert np.linalg.norm(zt.cpu().numpy() - z_ref) <= 1e-12 * np.linalg.norm(z_ref)
    prob.close()
    mlp.close()


def test_learned_gmres_and_gain(torch_dev):
    """GMRES(40) to 1e-8 with the learned rows (exact fallback) on an
    evaluation field whose seed the training did not use; the trained network
    keeps more rows than the untrained one at the same threshold."""
    torch, dev = torch_dev
    from paper_1607_02560_amd import lsp
    from paper_1607_02560_amd import surrogate as SG
    mlp, _ = trained_net(torch_dev, steps=400)
    raw = SG.make_mlp(3, 1, seed=12, batch_rows=1024)
    raw.set_normalisation(*mlp.get_normalisation())
    p, prob = small_problem(torch_dev, seed=0)
    N, m = p.N, 27
    thr = 0.02
    counts = {}
    for name, net in (("trained", mlp), ("untrained", raw)):
        P = torch.empty(N * m, dtype=torch.float64, device=dev)
        fb = torch.empty(N, dtype=torch.int32, device=dev)
        nf = prob.stencil_setup_learned(net, 1, p.num_shifts, thr, P, fb)
        solve = lsp.host_lu_solver(P.cpu().numpy().reshape(N, m), 3, 16, 1)
        ft = torch.from_numpy(p.f.reshape(-1)).to(dev)
        ut = torch.zeros_like(ft)
        code, iters, relres = prob.precond_solve(ft, ut, solve, rtol=1e-8, restart=40, maxit=400)
        counts[name] = (nf, iters, relres, code)
    P = torch.empty(N * m, dtype=torch.float64, device=dev)
    prob.stencil_setup(1, p.num_shifts, P)
    solve = lsp.host_lu_solver(P.cpu().numpy().reshape(N, m), 3, 16, 1)
    ft = torch.from_numpy(p.f.reshape(-1)).to(dev)
    ut = torch.zeros_like(ft)
    code, iters_ex, rel_ex = prob.precond_solve(ft, ut, solve, rtol=1e-8, restart=40, maxit=400)
    print(f"[learned gmres] exact: {iters_ex} iterations; " +
          "; ".join(f"{k}: {v[0]} of {N} rows fall back, {v[1]} iterations, relres {v[2]:.1e}"
                    for k, v in counts.items()), flush=True)
    assert code == lsp.LSP_OK and rel_ex <= 1e-8
    assert counts["trained"][3] == lsp.LSP_OK and counts["trained"][2] <= 1e-8
    assert counts["trained"][0] < counts["untrained"][0]
    prob.close()
    mlp.close()
    raw.close()


def test_save_load_round_trip(torch_dev, tmp_path):
    """A saved network loads with the same parameters, standardisation and
    Adam state: forward outputs are identical and the next training step of
    the loaded copy equals that of the original."""
    torch, dev = torch_dev
    from paper_1607_02560_amd import lsp
    mlp, _ = trained_net(torch_dev, steps=50)
    path = str(tmp_path / "net.lspmlp")
    mlp.save(path)
    other = lsp.MLP.load(path, batch_rows=1024)
    assert (other.n_in, other.n_hidden, other.n_out) == (29, 128, 54)
    assert np.array_equal(other.get_params(), mlp.get_params())
    for a, b in zip(other.get_normalisation(), mlp.get_normalisation()):
        assert np.array_equal(a, b)
    r = np.random.default_rng(21)
    X = torch.from_numpy(r.standard_normal((300, 29)).astype(np.float32) * 0.01).to(dev)
    T = torch.from_numpy(r.standard_normal((300, 54)).astype(np.float32)).to(dev)
    Y1 = torch.empty((300, 54), dtype=torch.float32, device=dev)
    Y2 = torch.empty_like(Y1)
    mlp.forward(X, Y1)
    other.forward(X, Y2)
    torch.cuda.synchronize()
    assert torch.equal(Y1, Y2)
    mlp.train_step(X, T, 1e-3)
    other.train_step(X, T, 1e-3)
    assert np.array_equal(other.get_params(), mlp.get_params())
    # a corrupted payload is refused
    raw = bytearray(open(path, "rb").read())
    raw[100] ^= 0xFF
    bad = str(tmp_path / "bad.lspmlp")
    open(bad, "wb").write(bytes(raw))
    with pytest.raises(lsp.LSPError):
        lsp.MLP.load(bad)
    with pytest.raises(lsp.LSPError):
        lsp.MLP.load(str(tmp_path / "missing.lspmlp"))
    mlp.close()
    other.close()


def test_learned_setup_edge_cases(torch_dev):
    """A network with non-finite outputs sends every row to the exact fallback;
    the asynchronous call (no count) writes the same rows; bad arguments are
    refused."""
    torch, dev = torch_dev
    from paper_1607_02560_amd import lsp
    from paper_1607_02560_amd import surrogate as SG
    p, prob = small_problem(torch_dev, seed=2)
    N, m = p.N, 27
    Pex = torch.empty(N * m, dtype=torch.float64, device=dev)
    prob.stencil_setup(1, p.num_shifts, Pex)
    nan_net = SG.make_mlp(3, 1, seed=1, batch_rows=256)
    flat = nan_net.get_params()
    flat[-54:] = np.nan  # output biases
    nan_net.set_params(flat)
    Pl = torch.empty(N * m, dtype=torch.float64, device=dev)
    fb = torch.empty(N, dtype=torch.int32, device=dev)
    nf = prob.stencil_setup_learned(nan_net, 1, p.num_shifts, 0.01, Pl, fb)
    assert nf == N and int(fb.sum()) == N
    assert torch.equal(Pl, Pex)
    # asynchronous call with a trained network equals the counted one
    mlp, _ = trained_net(torch_dev, steps=100)
    P1 = torch.empty_like(Pl)
    P2 = torch.full_like(Pl, float("nan"))
    f1 = torch.empty_like(fb)
    f2 = torch.full_like(fb, -1)
    prob.stencil_setup_learned(mlp, 1, p.num_shifts, 0.01, P1, f1)
    assert prob.stencil_setup_learned(mlp, 1, p.num_shifts, 0.01, P2, f2, count=False) is None
    torch.cuda.synchronize()
    assert torch.equal(P1, P2) and torch.equal(f1, f2)
    with pytest.raises(lsp.LSPError):
        prob.stencil_setup_learned(mlp, 1, p.num_shifts, -0.5, P1, f1)  # threshold < 0
    wrong = lsp.MLP(28, 128, 54, 64)  # m + 1 inputs: not this problem's network
    with pytest.raises(lsp.LSPError):
        prob.stencil_setup_learned(wrong, 1, p.num_shifts, 0.01, P1, f1)
    for q in (nan_net, mlp, wrong):
        q.close()
    prob.close()
