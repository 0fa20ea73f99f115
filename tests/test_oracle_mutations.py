"""Plausible mistakes planted in the oracle (on the CPU) must each make one of
its pins fail. This checks that the pins constrain the oracle, not only that
the oracle passes them."""
import math

import numpy as np
import pytest

from oracle import lsp_oracle as O
from tests import test_oracle_pins as pins

PI2 = math.pi ** 2
_orig = {name: getattr(O, name) for name in dir(O) if not name.startswith("__")}


def _symbol_missing_4(d, n):
    return _orig["symbol"](d, n) / 4.0


def _ps_apply_wrong_sign(v, u):
    d, n = u.ndim, u.shape[0]
    return np.fft.ifftn(_orig["symbol"](d, n) * np.fft.fftn(u)) - v * u


def _lap1d_wrong_diag(n):
    L = _orig["laplacian_1d_dense"](n)
    np.fill_diagonal(L, math.pi ** 2 * (n * n + 1) / 3.0)
    return L


def _green_wrong_sign(d, n, s):
    return _orig["green_kernels"](d, n, -s)


def _gram_plus(g, gam, offs):
    Gmm, A1, A2, M = _orig["gram"](g, gam, offs)
    return Gmm, A1, A2, A1 + A2


def _null_largest(M):
    w, V = np.linalg.eigh(M)
    a = O.normalise_sign(V[:, -1])
    return a, w, math.sqrt(max(w[0], 0.0)), 1.0


def _snap_round(s):
    m = round(s / (4 * PI2))
    return (4 * m + 2) * PI2


def _assign_upper(v, S):
    flat = v.reshape(-1)
    d = np.abs(S[None, :] - flat[:, None])
    return (len(S) - 1 - np.argmin(d[:, ::-1], axis=1)).astype(np.int32).reshape(v.shape)


def _assign_argmax(v, S):
    flat = v.reshape(-1)
    return np.argmax(np.abs(S[None, :] - flat[:, None]), axis=1).astype(np.int32).reshape(v.shape)


def _assemble_centre_only(v, S, alpha, C, idx, offs):
    d = v.ndim
    flat_idx = idx.reshape(-1)
    s_j = S[flat_idx]
    vj = v.reshape(-1)
    return alpha[flat_idx] + C[flat_idx] * (vj - s_j)[:, None]


def _shift_list_left_edges(v, num_shifts):
    vmin, vmax = float(np.min(v)), float(np.max(v))
    width = (vmax - vmin) / num_shifts
    out = []
    for i in range(num_shifts):
        s = O.snap_shift(vmin + i * width)
        if not out or s != out[-1]:
            out.append(s)
    return np.asarray(out)


def _global_midrange(v):
    return 0.5 * (float(np.min(v)) + float(np.max(v)))


def _global_ignores_resonance(v):
    return float(np.mean(v))


def _global_always_snaps(v):
    return O.snap_shift(float(np.mean(v)))


def _tmap_vertex_one(d, n, b, tmax):
    t = _orig["nd_tmap"](d, n, b, tmax)
    coords = np.stack(np.unravel_index(np.arange(n ** d), (n,) * d), axis=-1)
    vert = np.all(coords % b == 0, axis=1).reshape(t.shape)
    return np.where(vert, 1, t)


def _tmap_edge_full(d, n, b, tmax):
    coords = np.stack(np.unravel_index(np.arange(n ** d), (n,) * d), axis=-1)
    r = coords % b
    dist = np.minimum(r, b - r)
    t = np.where(np.all(r == 0, axis=1), b, dist.max(axis=1))
    return np.minimum(t, tmax).reshape((n,) * d)


MUTANTS = [
    ("symbol", _symbol_missing_4, lambda: pins.test_plane_waves_are_eigenvectors(2, 8)),
    ("ps_apply", _ps_apply_wrong_sign, lambda: pins.test_ps_apply_matches_dense(2, 8, 1)),
    ("laplacian_1d_dense", _lap1d_wrong_diag, lambda: pins.test_laplacian_1d_spectrum(8)),
    ("green_kernels", _green_wrong_sign,
     lambda: pins.test_green_kernel_is_first_column_of_inverse(2, 8, -7)),
    ("gram", _gram_plus, lambda: pins.test_gram_identity(2, 16, 1, -20)),
    ("null_vector", _null_largest,
     lambda: pins.test_null_vector_is_the_optimal_stencil(2, 16, 1, -20)),
    ("snap_shift", _snap_round, pins.test_snap_is_nearest_of_form),
    ("assign_shifts", _assign_upper, pins.test_assign_shifts_bruteforce),
    ("assign_shifts", _assign_argmax, pins.test_assign_shifts_bruteforce),
    ("assemble", _assemble_centre_only, pins.test_P_row_formula_dense),
    ("shift_list", _shift_list_left_edges, pins.test_shift_list_spreads_evenly),
    ("global_shift", _global_midrange, lambda: pins.test_global_setup_dense_definition(2, 8, 1)),
    ("global_shift", _global_ignores_resonance,
     lambda: pins.test_global_shift_moves_off_resonance(5)),
    ("global_shift", _global_always_snaps, pins.test_global_shift_keeps_non_resonant_mean),
    ("nd_tmap", _tmap_vertex_one, pins.test_nd_tmap_matches_fig3),
    ("nd_tmap", _tmap_edge_full, pins.test_nd_tmap_matches_fig3),
]


@pytest.mark.parametrize("name,mutant,pin", MUTANTS, ids=[f"{m[0]}-{m[1].__name__}" for m in MUTANTS])
def test_planted_mistake_is_caught(monkeypatch, name, mutant, pin):
    monkeypatch.setattr(O, name, mutant)
    with pytest.raises(AssertionError):
        pin()
