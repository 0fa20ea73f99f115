"""Training and use of the learned-stencil surrogate (lsp_mlp_* of the C ABI).

The surrogate is not part of the paper. A network with two hidden SiLU
layers of width 128 maps the m + 2 features of a grid point (h^2 v_j, the
potential patch h^2 v[j + a], a in mu_0^t, and h^2 s_j for the shift assigned
to the point) to its exact P row (Sec. 4.1) and
the C row of its shift times |s_j| (eq. PC). Training rows come from exact
setups on fields that are not the evaluation field; the learned setup
checks every predicted row against the exact Gram matrices of eq. (A) and
falls back to the exact row where the check fails (lsp_stencil_setup_learned).

Every numerical step runs in the library's kernels; this module draws the
initial weights and the sample indices on the host (they are inputs), moves
arguments and loops over batches.
"""
from __future__ import annotations

import numpy as np

from . import lsp

HIDDEN = 128


def glorot_params(n_in: int, n_hidden: int, n_out: int, seed: int) -> np.ndarray:
    """Glorot-uniform weights and zero biases, flattened in the ABI's order
    W1, b1, W2, b2, W3, b3."""
    r = np.random.default_rng(seed)

    def glorot(fo, fi):
        lim = np.sqrt(6.0 / (fi + fo))
        return r.uniform(-lim, lim, (fo, fi))

    parts = [glorot(n_hidden, n_in), np.zeros(n_hidden), glorot(n_hidden, n_hidden),
             np.zeros(n_hidden), glorot(n_out, n_hidden), np.zeros(n_out)]
    return np.concatenate([p.reshape(-1) for p in parts]).astype(np.float32)


def gather_rows(fields, t: int, num_shifts: int, rows_per_field: int, seed: int, device):
    """Exact setups of each potential in `fields` (numpy arrays of shape
    (n,)*d) and the features / targets of `rows_per_field` random points of
    each. Returns device tensors X [rows][m+2], T [rows][2m] (float32)."""
    import torch
    r = np.random.default_rng(seed)
    xs, ts = [], []
    for v in fields:
        d, n = v.ndim, v.shape[0]
        N = n ** d
        m = (2 * t + 1) ** d
        prob = lsp.Problem(d, n, torch.from_numpy(np.ascontiguousarray(v).reshape(-1)).to(device))
        P = torch.empty(N * m, dtype=torch.float64, device=device)
        prob.stencil_setup(t, num_shifts, P)
        cnt = min(rows_per_field, N)
        pts = torch.from_numpy(np.sort(r.choice(N, cnt, replace=False)).astype(np.int64)).to(device)
        X = torch.empty((cnt, m + 2), dtype=torch.float32, device=device)
        T = torch.empty((cnt, 2 * m), dtype=torch.float32, device=device)
        prob.training_rows(P, pts, X, T)
        torch.cuda.synchronize(device)
        xs.append(X)
        ts.append(T)
        prob.close()
        del P
    return torch.cat(xs), torch.cat(ts)


def train(mlp: "lsp.MLP", X, T, steps: int, batch: int, lr: float, seed: int,
          report_every: int = 0, lr_final: float | None = None):
    """Adam on random batches of the rows (indices drawn on the device from a
    seeded generator, the batch gathered on the device, so a step makes no
    host-to-device copy). The learning rate decays geometrically to lr_final
    when given. Returns the list of (step, loss) reported."""
    import torch
    rows = X.shape[0]
    dev = X.device
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    Xb = torch.empty((batch, X.shape[1]), dtype=torch.float32, device=dev)
    Tb = torch.empty((batch, T.shape[1]), dtype=torch.float32, device=dev)
    idx = torch.empty(batch, dtype=torch.int64, device=dev)
    hist = []
    decay = 1.0 if lr_final is None else (lr_final / lr) ** (1.0 / max(steps - 1, 1))
    for it in range(steps):
        torch.randint(0, rows, (batch,), generator=gen, device=dev, out=idx)
        torch.index_select(X, 0, idx, out=Xb)
        torch.index_select(T, 0, idx, out=Tb)
        want = report_every > 0 and (it % report_every == 0 or it == steps - 1)
        loss = mlp.train_step(Xb, Tb, lr * decay ** it, want_loss=want)
        if want:
            hist.append((it, loss))
    return hist


def make_mlp(d: int, t: int, seed: int, batch_rows: int = 8192) -> "lsp.MLP":
    m = (2 * t + 1) ** d
    mlp = lsp.MLP(m + 2, HIDDEN, 2 * m, batch_rows)
    mlp.set_params(glorot_params(m + 2, HIDDEN, 2 * m, seed))
    return mlp
