"""FP64 CPU reference of the learned-stencil surrogate.

TEST INFRASTRUCTURE ONLY. Only the test-suite and the smoke check may import
this module; the HIP library never calls it and shares no code with it.

The surrogate is not part of the paper: it is the project's own addition
beside the method. Its definition (inputs, network, targets, loss, fallback
test) is written out here in plain numpy so that the GPU training and
inference kernels can be checked against it:

  features         the m + 2 inputs of grid point j: h^2 v_j, h^2 v[j + a]
                   for the offsets a of mu_0^t (Sec. 4.2), h = 1/n, and h^2 s_j
                   for the shift s_j assigned to the point (Sec. 4.1); the
                   exact row depends on v_j only through the patch and on the
                   bin of v_j through s_j, which jumps between bins
  targets          the exact rows of point j: P[j, a] (Sec. 4.1) and the C row
                   of its shift (eq. PC) scaled by |s_j| (an O(1) quantity,
                   since C = G alpha and G ~ 1/|s|)
  forward          two hidden layers with SiLU, linear output, on inputs and
                   outputs standardised by per-feature mean and deviation
  loss_and_grads   mean squared error over all outputs and its gradients by
                   the chain rule (backpropagation)
  adam_step        the Adam update (Kingma and Ba, 2015) with bias correction
  residual         the fallback test: for the stencil q = p - c (v[mu] - s)
                   predicted for a point, rho = sqrt(q^T M q / q^T A1 q) with
                   M = A1 - A2 of eq. (A): the fraction of the row of Q G that
                   the truncation to mu drops (Sec. 3); 0 <= rho <= 1.
"""
from __future__ import annotations

import numpy as np

from . import lsp_oracle as O


# ----------------------------------------------------------------- data ----
def features(v: np.ndarray, t: int, S: np.ndarray) -> np.ndarray:
    """(N, m + 2) inputs, rows in the grid's C order: h^2 v_j, then
    h^2 v[(j + a) mod n] for the offsets a of mu_0^t in lexicographic order,
    then h^2 s_j with s_j the entry of the shift list S nearest to v_j."""
    d, n = v.ndim, v.shape[0]
    h2 = 1.0 / (n * n)
    offs = O.offsets(d, t)
    cols = [h2 * v.reshape(-1)]
    for a in offs:
        cols.append(h2 * np.roll(v, tuple(-a), axis=tuple(range(d))).reshape(-1))
    cols.append(h2 * S[O.assign_shifts(v, S).reshape(-1)])
    return np.stack(cols, axis=1)


def targets(P: np.ndarray, S: np.ndarray, C: np.ndarray, idx: np.ndarray) -> np.ndarray:
    """(N, 2m) targets: the P row of each point, then the C row of its shift
    times |s_j|."""
    idx = idx.reshape(-1)
    s = S[idx]
    return np.concatenate([P, C[idx] * np.abs(s)[:, None]], axis=1)


def split_outputs(Y: np.ndarray, S: np.ndarray, idx: np.ndarray, m: int):
    """Inverse of `targets`: (P rows, C rows) from (N, 2m) outputs."""
    s = S[idx.reshape(-1)]
    return Y[:, :m], Y[:, m:] / np.abs(s)[:, None]


# -------------------------------------------------------------- network ----
def init_params(n_in: int, n_hidden: int, n_out: int, seed: int) -> dict:
    """Glorot-uniform weights, zero biases."""
    r = np.random.default_rng(seed)

    def glorot(fo, fi):
        lim = np.sqrt(6.0 / (fi + fo))
        return r.uniform(-lim, lim, (fo, fi))

    return {"W1": glorot(n_hidden, n_in), "b1": np.zeros(n_hidden),
            "W2": glorot(n_hidden, n_hidden), "b2": np.zeros(n_hidden),
            "W3": glorot(n_out, n_hidden), "b3": np.zeros(n_out)}


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def silu(z):
    return z * sigmoid(z)


def silu_grad(z):
    sg = sigmoid(z)
    return sg * (1.0 + z * (1.0 - sg))


def forward(p: dict, X: np.ndarray):
    """Outputs of the standardised network and the intermediate values."""
    Z1 = X @ p["W1"].T + p["b1"]
    A1 = silu(Z1)
    Z2 = A1 @ p["W2"].T + p["b2"]
    A2 = silu(Z2)
    Y = A2 @ p["W3"].T + p["b3"]
    return Y, (X, Z1, A1, Z2, A2)


def loss_and_grads(p: dict, X: np.ndarray, T: np.ndarray):
    """Mean squared error over the B x n_out outputs and its gradients."""
    Y, (X, Z1, A1, Z2, A2) = forward(p, X)
    B, n_out = Y.shape
    R = Y - T
    loss = float(np.sum(R * R) / (B * n_out))
    dY = 2.0 * R / (B * n_out)
    g = {}
    g["W3"] = dY.T @ A2
    g["b3"] = dY.sum(axis=0)
    dZ2 = (dY @ p["W3"]) * silu_grad(Z2)
    g["W2"] = dZ2.T @ A1
    g["b2"] = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ p["W2"]) * silu_grad(Z1)
    g["W1"] = dZ1.T @ X
    g["b1"] = dZ1.sum(axis=0)
    return loss, g


def adam_step(p: dict, g: dict, state: dict, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step in place; state holds m, v (per parameter) and the step count."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in p:
        m = state.setdefault("m_" + k, np.zeros_like(p[k]))
        v = state.setdefault("v_" + k, np.zeros_like(p[k]))
        m *= beta1
        m += (1.0 - beta1) * g[k]
        v *= beta2
        v += (1.0 - beta2) * g[k] * g[k]
        mh = m / (1.0 - beta1 ** t)
        vh = v / (1.0 - beta2 ** t)
        p[k] -= lr * mh / (np.sqrt(vh) + eps)


def standardise(A: np.ndarray):
    """Per-column mean and deviation (deviation 1 where a column is constant)."""
    mu = A.mean(axis=0)
    sd = A.std(axis=0)
    sd = np.where(sd > 0, sd, 1.0)
    return mu, sd


# ------------------------------------------------------------- fallback ----
def residual(q: np.ndarray, g: np.ndarray, gam: np.ndarray, offs: np.ndarray) -> float:
    """rho = sqrt(q^T M q / q^T A1 q) for a stencil q on mu_0^t, with
    A1 = (G_s^2)[mu, mu] and M = A1 - G_mu,mu G_mu,mu of eq. (A)."""
    Gmm, A1, _, M = O.gram(g, gam, offs)
    num = float(q @ M @ q)
    den = float(q @ A1 @ q)
    return float(np.sqrt(max(num, 0.0) / den))
