"""Pins of the FP64 surrogate reference (oracle/mlp_oracle.py) to things other
than itself: central finite differences for every gradient, the closed form
of Adam's first step, SiLU's values and derivative at known points, brute-force
feature extraction, and the fallback residual against the dropped fraction of
the row of Q G built with the dense inverse of L + s I."""
import math

import numpy as np
import pytest

from oracle import lsp_oracle as O
from oracle import mlp_oracle as MO


def small_net(seed=0, n_in=5, n_hidden=7, n_out=3):
    p = MO.init_params(n_in, n_hidden, n_out, seed)
    r = np.random.default_rng(seed + 100)
    for k in ("b1", "b2", "b3"):
        p[k] = r.standard_normal(p[k].shape) * 0.3
    return p


@pytest.mark.parametrize("shape", [(5, 7, 3, 4), (28, 128, 54, 6)])
def test_gradients_match_central_differences(shape):
    n_in, n_hidden, n_out, B = shape
    p = small_net(1, n_in, n_hidden, n_out)
    r = np.random.default_rng(2)
    X = r.standard_normal((B, n_in))
    T = r.standard_normal((B, n_out))
    loss, g = MO.loss_and_grads(p, X, T)
    h = 1e-6
    for k in p:
        flat = p[k].reshape(-1)
        picks = range(flat.size) if flat.size <= 40 else r.choice(flat.size, 25, replace=False)
        for i in picks:
            old = flat[i]
            flat[i] = old + h
            lp, _ = MO.loss_and_grads(p, X, T)
            flat[i] = old - h
            lm, _ = MO.loss_and_grads(p, X, T)
            flat[i] = old
            fd = (lp - lm) / (2 * h)
            an = g[k].reshape(-1)[i]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (k, i, fd, an)


def test_adam_first_step_closed_form():
    """With zero moments, bias correction makes the first step -lr g / (|g| + eps)."""
    p = small_net(3)
    r = np.random.default_rng(4)
    g = {k: r.standard_normal(v.shape) for k, v in p.items()}
    p0 = {k: v.copy() for k, v in p.items()}
    st = {}
    MO.adam_step(p, g, st, lr=1e-3)
    for k in p:
        expect = p0[k] - 1e-3 * g[k] / (np.abs(g[k]) + 1e-8)
        assert np.allclose(p[k], expect, rtol=0, atol=1e-15)
    # second step with the same gradient: m_hat = g, v_hat = g^2 again
    MO.adam_step(p, g, st, lr=1e-3)
    for k in p:
        expect = p0[k] - 2e-3 * g[k] / (np.abs(g[k]) + 1e-8)
        assert np.allclose(p[k], expect, rtol=0, atol=1e-14)


def test_silu_known_values():
    assert MO.silu(0.0) == 0.0
    assert MO.silu_grad(0.0) == 0.5
    assert MO.silu(50.0) == pytest.approx(50.0, rel=1e-15)
    assert abs(MO.silu(-50.0)) < 1e-18
    z = np.linspace(-6, 6, 41)
    fd = (MO.silu(z + 1e-6) - MO.silu(z - 1e-6)) / 2e-6
    assert np.allclose(MO.silu_grad(z), fd, atol=1e-8)


def test_features_brute_force():
    d, n, t = 3, 5, 1
    v = np.random.default_rng(5).standard_normal((n,) * d)
    S = np.array([-1.5, -0.2, 0.4, 1.1])
    X = MO.features(v, t, S)
    offs = O.offsets(d, t)
    h2 = 1.0 / (n * n)
    assert X.shape == (n ** d, offs.shape[0] + 2)
    for j in [0, 7, 62, 124]:
        idx = np.unravel_index(j, (n,) * d)
        assert X[j, 0] == h2 * v[idx]
        for a, off in enumerate(offs):
            nb = tuple((idx[ax] + off[ax]) % n for ax in range(d))
            assert X[j, 1 + a] == h2 * v[nb]
        # the nearest entry of S by a scan (ties to the lower index)
        best = min(range(len(S)), key=lambda i: (abs(S[i] - v[idx]), i))
        assert X[j, -1] == h2 * S[best]


def test_targets_round_trip():
    r = np.random.default_rng(6)
    N, m, k = 10, 9, 3
    P = r.standard_normal((N, m))
    C = r.standard_normal((k, m))
    S = np.array([-1000.0, -500.0, 30.0])
    idx = r.integers(0, k, N)
    Tg = MO.targets(P, S, C, idx)
    P2, C2 = MO.split_outputs(Tg, S, idx, m)
    assert np.array_equal(P2, P)
    assert np.allclose(C2, C[idx], rtol=1e-15)


def test_residual_is_the_dropped_fraction_of_the_row():
    """rho is ||(QG)[j, mu^c]|| / ||(QG)[j, :]|| for the row of Q G that the
    stencil q builds at point j (Sec. 3), checked with the dense inverse of
    L + s I; and 0 <= rho <= 1."""
    d, n, t = 2, 16, 1
    s = (4 * (-20) + 2) * math.pi ** 2
    g, gam = O.green_kernels(d, n, s)
    offs = O.offsets(d, t)
    N = n ** d
    Gd = np.linalg.inv(O.dense_laplacian(d, n) + s * np.eye(N))
    j = np.array([3, 11])
    mu = [int(np.ravel_multi_index(tuple((j + a) % n), (n,) * d)) for a in offs]
    mask = np.ones(N, dtype=bool)
    mask[mu] = False
    r = np.random.default_rng(7)
    alpha = O.null_vector(O.gram(g, gam, offs)[3])[0]
    for q in [alpha] + [r.standard_normal(offs.shape[0]) for _ in range(5)]:
        row = q @ Gd[mu, :]
        rho_bf = np.linalg.norm(row[mask]) / np.linalg.norm(row)
        rho = MO.residual(q, g, gam, offs)
        assert rho == pytest.approx(rho_bf, rel=1e-7, abs=1e-12)
        assert 0.0 <= rho <= 1.0 + 1e-12
