"""The seeded input recipes have the structure their descriptions state
(CPU only). They hold no arithmetic of the method; these checks keep the
stand-ins for the paper's field families honest."""
import math

import numpy as np
import pytest

from paper_1607_02560_amd import workloads as W


def _omega(n):
    return 2.0 * math.pi * n / 8.0


def test_helm2d_cross_has_two_speeds_in_a_cross():
    p = W.helm2d_cross(64)
    c = _omega(64) / np.sqrt(-p.v)
    vals = np.unique(np.round(c, 12))
    assert np.allclose(vals, [0.7, 1.0])
    slow = np.isclose(c, 0.7)
    # rows and columns through the centre are slow; a corner point is not
    assert slow[32].all() and slow[:, 32].all() and not slow[10, 10]
    assert slow.sum() == 2 * 64 * 7 - 7 * 7  # two bands of 7 grid lines, overlap counted once


def test_helm3d_cross_is_three_cylinders():
    p = W.helm3d_cross(32)
    c = _omega(32) / np.sqrt(-p.v)
    slow = np.isclose(c, 0.7)
    assert slow[:, 16, 16].all() and slow[16, :, 16].all() and slow[16, 16, :].all()
    assert not slow[4, 4, 4] and not slow[4, 4, 16]
    assert np.allclose(np.unique(np.round(c, 12)), [0.7, 1.0])


def test_helm3d_gauss_is_slowest_at_the_centre():
    p = W.helm3d_gauss(32)
    c = _omega(32) / np.sqrt(-p.v)
    assert c[16, 16, 16] == pytest.approx(0.7) and c.max() == pytest.approx(1.0, abs=1e-6)
    assert np.argmin(c) == np.ravel_multi_index((16, 16, 16), c.shape)


@pytest.mark.parametrize("d,n,per_axis", [(2, 128, 8), (3, 32, 4)])
def test_lattice_has_a_vacancy_at_the_centre(d, n, per_axis):
    p = W.schrod2d_lattice(n) if d == 2 else W.schrod3d_lattice(n)
    background = -2.4 * n * n
    bump = n * n * (4.0 - 2.4)
    step = n // per_axis
    centre = (n // 2,) * d
    # the vacancy sits at the background value; every other lattice site is a bump
    assert p.v[centre] == pytest.approx(background, rel=1e-4)
    for idx in np.ndindex(*([per_axis] * d)):
        site = tuple(i * step for i in idx)
        if site != centre:
            assert p.v[site] == pytest.approx(bump, rel=1e-3)


@pytest.mark.parametrize("name", ["schrod2d_lattice_n128", "schrod3d_wells_n32",
                                  "schrod3d_lattice_n32"])
def test_schrodinger_scaling_resolves_every_oscillation(name):
    """Sec. 5's scaling: v >= -E/h^2 with E = 2.4, so the local wavenumber
    sqrt(-v) never exceeds sqrt(2.4)/h and an oscillation spans > 4 points."""
    p = W.make(name)
    n2 = p.n * p.n
    assert p.v.min() >= -2.4 * n2 * (1 + 1e-12)
    points_per_oscillation = 2 * math.pi / math.sqrt(-p.v.min() / n2)
    assert points_per_oscillation > 4.0


@pytest.mark.parametrize("name", sorted(W.CONFIGS))
def test_configs_are_seeded_and_finite(name):
    a, b = W.make(name), W.make(name)
    assert np.array_equal(a.v, b.v) and np.array_equal(a.f, b.f)
    assert np.all(np.isfinite(a.v)) and a.v.dtype == np.float64 and a.f.dtype == np.complex128
    assert a.v.shape == (a.n,) * a.d and a.num_shifts >= 1
