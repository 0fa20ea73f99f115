"""Seeded synthetic inputs for the periodic problem (-Delta + v) u = f on [0,1)^d.

This module only *describes problems*: velocity fields, potentials and
right-hand sides sampled on the grid hJ (Section 2, grid J and h = 1/n).
It holds none of the preconditioner's arithmetic, so both the HIP path and
the FP64 oracle take their inputs from here.

The paper does not give the parameters of its own fields (Section 5 only
names "a Gaussian profile", "random Gaussians", ...). The recipes below
are stand-ins with the same structure:

  helm2d_gauss   2D Helmholtz, c = 1 - 0.3 exp(-|x-x0|^2/0.02),
                 omega for 8 points per wavelength at c = 1, 3x3 stencil,
                 |S| = 2 at n <= 32 and n/16 above.
  schrod2d_wells 2D Schroedinger-type, 16 Gaussian wells of depth
                 U[5,20] n^2 and width U[0.02,0.05], minus E = 0.5 max depth.
  helm2d_random  2D Helmholtz, c a smooth random field in [0.8,1.2]
                 (Fourier modes 0 < |k| <= 8), omega = 2 pi n / 8.
  helm3d_random  3D analogue of helm2d_random.
  batch2d        64 problems of uneven n drawn from {64,128,256,512}.

and one stand-in for each remaining field family of Sec. 5:

  helm2d_cross     2D Helmholtz, constant c = 1 background with a cross of
                   c = 0.7: the two bands |x - 1/2| < 0.05, |y - 1/2| < 0.05.
  helm3d_gauss     3D Helmholtz, c = 1 - 0.3 exp(-|x-x0|^2/0.02).
  helm3d_cross     3D Helmholtz, c = 0.7 inside three cylinders of radius
                   0.05 along the three axes through the centre, else 1.
  schrod2d_lattice 2D Schroedinger, an 8 x 8 array of equal Gaussians at
                   (i, j)/8 with the one at the centre missing.
  schrod3d_wells   3D Schroedinger, 16 Gaussians at random centres.
  schrod3d_lattice 3D analogue of schrod2d_lattice (4 x 4 x 4, centre missing).

The Schroedinger stand-ins follow Sec. 5's scaling v = (v_ext(x/h) - E)/h^2
with E = 2.4: v_ext >= 0 is a sum of Gaussian bumps A_i exp(-|y - y_i|^2 /
(2 s_i^2)) in grid units y = x/h, so -h^2 v <= E and every oscillation spans
at least 2 pi / sqrt(2.4) > 4 grid points. The lattices use A = 4, s = 2 grid
points (1.5 in 3D); the random bumps A ~ U[2, 6], s ~ U[1.5, 3].
(schrod2d_wells above is the deliberately harder deep-well case, outside that
scaling.)

Layout: C order, the last axis varies fastest; point j = (j_1,...,j_d) sits
at x = h j. Potentials are float64, right-hand sides complex128.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Problem", "grid_coords", "periodic_sqdist", "smooth_random_c",
    "helm2d_gauss", "schrod2d_wells", "helm2d_random", "helm3d_random",
    "batch2d", "gaussian_source", "random_field_v", "make", "CONFIGS",
    "helm2d_cross", "helm3d_gauss", "helm3d_cross", "schrod2d_lattice", "schrod3d_wells",
    "schrod3d_lattice",
]


@dataclasses.dataclass
class Problem:
    name: str
    d: int
    n: int
    v: np.ndarray          # float64, shape (n,)*d
    f: np.ndarray          # complex128, shape (n,)*d
    t: int                 # neighbourhood radius (Section 4.2, mu^t)
    num_shifts: int        # requested |S| (Section 4.1)
    omega: float | None = None

    @property
    def N(self) -> int:
        return self.n ** self.d


def grid_coords(d: int, n: int):
    """Coordinates x = h j on hJ, as a list of d broadcastable arrays."""
    h = 1.0 / n
    ax = np.arange(n, dtype=np.float64) * h
    out = []
    for i in range(d):
        shape = [1] * d
        shape[i] = n
        out.append(ax.reshape(shape))
    return out


def periodic_sqdist(d: int, n: int, centre) -> np.ndarray:
    """Squared minimum-image distance on the unit torus to `centre`."""
    xs = grid_coords(d, n)
    acc = np.zeros((n,) * d)
    for i in range(d):
        dx = np.abs(xs[i] - centre[i])
        dx = np.minimum(dx, 1.0 - dx)
        acc = acc + dx * dx
    return acc


def gaussian_source(d: int, n: int, centre, sigma: float) -> np.ndarray:
    """exp(-|x - centre|^2 / (2 sigma^2)) as complex128 (a point-like source)."""
    r2 = periodic_sqdist(d, n, centre)
    return np.exp(-r2 / (2.0 * sigma * sigma)).astype(np.complex128)


def _half_space_modes(d: int, kmax: float):
    """Integer wave vectors with 0 < |k| <= kmax, one of each +-k pair."""
    r = int(math.floor(kmax))
    rng1 = range(-r, r + 1)
    modes = []
    if d == 2:
        for a in rng1:
            for b in rng1:
                k = (a, b)
                if 0 < a * a + b * b <= kmax * kmax and k > (0, 0):
                    modes.append(k)
    else:
        for a in rng1:
            for b in rng1:
                for c in rng1:
                    k = (a, b, c)
                    if 0 < a * a + b * b + c * c <= kmax * kmax and k > (0, 0, 0):
                        modes.append(k)
    return modes


def smooth_random_c(d: int, n: int, seed: int, lo=0.8, hi=1.2, kmax=8.0) -> np.ndarray:
    """psi = sum a_k cos(2 pi k.x) + b_k sin(2 pi k.x) over 0<|k|<=kmax,
    a_k, b_k ~ N(0,1); then c = lo + (hi-lo)(psi - min psi)/(max psi - min psi)."""
    rng = np.random.default_rng(seed)
    modes = _half_space_modes(d, kmax)
    ab = rng.standard_normal((len(modes), 2))
    h = 1.0 / n
    j = np.arange(n, dtype=np.float64)
    psi = np.zeros((n,) * d)
    # exp(2 pi i k.x) = prod_axes exp(2 pi i k_a x_a): separable evaluation
    for (k, (a, b)) in zip(modes, ab):
        e = None
        for ax in range(d):
            ph = np.exp(2j * np.pi * k[ax] * j * h)
            shape = [1] * d
            shape[ax] = n
            ph = ph.reshape(shape)
            e = ph if e is None else e * ph
        psi = psi + a * e.real + b * e.imag
    pmin, pmax = psi.min(), psi.max()
    return lo + (hi - lo) * (psi - pmin) / (pmax - pmin)


def helm2d_gauss(n: int = 32, seed: int = 0, num_shifts=None) -> Problem:
    """2D Helmholtz, Gaussian-profile velocity, 3x3 stencils; |S| = 2 at
    n <= 32 (the small configuration) and n/16 above, the ratio of Sec. 5."""
    d = 2
    c = 1.0 - 0.3 * np.exp(-periodic_sqdist(d, n, (0.5, 0.5)) / 0.02)
    omega = 2.0 * np.pi * n / 8.0
    v = -(omega / c) ** 2
    f = gaussian_source(d, n, (0.3, 0.3), 0.05)
    if num_shifts is None:
        num_shifts = 2 if n <= 32 else n // 16
    return Problem("helm2d_gauss", d, n, np.ascontiguousarray(v), f, t=1,
                   num_shifts=num_shifts, omega=omega)


def schrod2d_wells(n: int = 256, seed: int = 0, wells: int = 16) -> Problem:
    """2D Schroedinger-type potential: -sum D_i exp(-|x-c_i|^2/(2 w_i^2)) - E."""
    d = 2
    rng = np.random.default_rng(seed)
    centres = rng.random((wells, d))
    depth = rng.uniform(5.0, 20.0, wells) * n * n
    width = rng.uniform(0.02, 0.05, wells)
    v = np.zeros((n,) * d)
    for i in range(wells):
        v -= depth[i] * np.exp(-periodic_sqdist(d, n, centres[i]) / (2.0 * width[i] ** 2))
    v -= 0.5 * depth.max()
    rng_f = np.random.default_rng(seed + 1)
    f = (rng_f.standard_normal((n,) * d) + 1j * rng_f.standard_normal((n,) * d)) / np.sqrt(2.0)
    return Problem("schrod2d_wells", d, n, np.ascontiguousarray(v), f, t=2,
                   num_shifts=16)


def helm2d_random(n: int = 1024, seed: int = 0, t: int = 2, num_shifts=None) -> Problem:
    """2D Helmholtz, smooth random c in [0.8,1.2], omega = 2 pi n / 8."""
    d = 2
    c = smooth_random_c(d, n, seed)
    omega = 2.0 * np.pi * n / 8.0
    v = -(omega / c) ** 2
    f = gaussian_source(d, n, (0.5, 0.5), 0.05)
    return Problem("helm2d_random", d, n, np.ascontiguousarray(v), f, t=t,
                   num_shifts=num_shifts if num_shifts else max(1, n // 16), omega=omega)


def helm3d_random(n: int = 64, seed: int = 0, t: int = 1, num_shifts=None) -> Problem:
    """3D Helmholtz, smooth random c in [0.8,1.2], omega = 2 pi n / 8."""
    d = 3
    c = smooth_random_c(d, n, seed)
    omega = 2.0 * np.pi * n / 8.0
    v = -(omega / c) ** 2
    f = gaussian_source(d, n, (0.5, 0.5, 0.5), 0.05)
    return Problem("helm3d_random", d, n, np.ascontiguousarray(v), f, t=t,
                   num_shifts=num_shifts if num_shifts else max(1, n // 4), omega=omega)


def batch2d(count: int = 64, seed: int = 0, sizes=(64, 128, 256, 512)):
    """`count` independent 2D Helmholtz problems, n drawn uniformly from `sizes`;
    problem p uses field seed p and |S_p| = n_p / 16."""
    rng = np.random.default_rng(seed)
    ns = rng.choice(np.asarray(sizes), size=count)
    return [helm2d_random(int(n_p), seed=p, t=2, num_shifts=int(n_p) // 16)
            for p, n_p in enumerate(ns)]


def _helmholtz(name: str, d: int, n: int, c: np.ndarray, t: int, num_shifts: int) -> Problem:
    omega = 2.0 * np.pi * n / 8.0
    v = -(omega / c) ** 2
    f = gaussian_source(d, n, (0.5,) * d, 0.05)
    return Problem(name, d, n, np.ascontiguousarray(v), f, t=t, num_shifts=num_shifts,
                   omega=omega)


def _band_distance(d: int, n: int, axis: int) -> np.ndarray:
    """Periodic distance of the grid points from the plane x_axis = 1/2."""
    x = np.arange(n) / n - 0.5
    x = np.minimum(np.abs(x), 1.0 - np.abs(x))
    shape = [1] * d
    shape[axis] = n
    return np.broadcast_to(x.reshape(shape), (n,) * d)


def helm2d_cross(n: int = 128, seed: int = 0, t: int = 1, num_shifts=None) -> Problem:
    """2D Helmholtz, constant background with a cross-shaped slow region."""
    d = 2
    cross = (_band_distance(d, n, 0) < 0.05) | (_band_distance(d, n, 1) < 0.05)
    c = np.where(cross, 0.7, 1.0)
    return _helmholtz("helm2d_cross", d, n, c, t, num_shifts or max(1, n // 16))


def helm3d_gauss(n: int = 32, seed: int = 0, t: int = 1, num_shifts=None) -> Problem:
    """3D Helmholtz, constant background with a Gaussian profile at the centre."""
    d = 3
    c = 1.0 - 0.3 * np.exp(-periodic_sqdist(d, n, (0.5, 0.5, 0.5)) / 0.02)
    return _helmholtz("helm3d_gauss", d, n, c, t, num_shifts or max(1, n // 4))


def helm3d_cross(n: int = 32, seed: int = 0, t: int = 1, num_shifts=None) -> Problem:
    """3D Helmholtz, three slow cylinders along the axes through the centre."""
    d = 3
    r = [_band_distance(d, n, a) for a in range(d)]
    cyl = ((r[1] ** 2 + r[2] ** 2 < 0.05 ** 2) | (r[0] ** 2 + r[2] ** 2 < 0.05 ** 2)
           | (r[0] ** 2 + r[1] ** 2 < 0.05 ** 2))
    c = np.where(cyl, 0.7, 1.0)
    return _helmholtz("helm3d_cross", d, n, c, t, num_shifts or max(1, n // 4))


def _bumps(d: int, n: int, centres, height, width_grid, energy: float = 2.4) -> np.ndarray:
    """v = n^2 (v_ext - energy), v_ext a sum of Gaussian bumps whose widths
    are given in grid points (Sec. 5: v_ext is a function of x/h)."""
    v_ext = np.zeros((n,) * d)
    for c, A, s in zip(centres, height, width_grid):
        w = s / n
        v_ext += A * np.exp(-periodic_sqdist(d, n, c) / (2.0 * w * w))
    return n * n * (v_ext - energy)


def _lattice_centres(d: int, per_axis: int):
    """Centres k / per_axis (k = 0..per_axis-1 per axis; per_axis even, so one
    centre is the domain's centre) without the centre one."""
    assert per_axis % 2 == 0
    ticks = np.arange(per_axis) / per_axis
    grids = np.meshgrid(*([ticks] * d), indexing="ij")
    pts = np.stack([g.reshape(-1) for g in grids], axis=1)
    keep = np.any(np.abs(pts - 0.5) > 1e-12, axis=1)
    assert keep.sum() == per_axis ** d - 1
    return pts[keep]


def _random_rhs(d: int, n: int, seed: int) -> np.ndarray:
    rng_f = np.random.default_rng(seed)
    return (rng_f.standard_normal((n,) * d) + 1j * rng_f.standard_normal((n,) * d)) / np.sqrt(2.0)


def schrod2d_lattice(n: int = 128, seed: int = 0, t: int = 2, num_shifts=None) -> Problem:
    """2D Schroedinger: an 8 x 8 lattice of equal bumps, the centre one missing."""
    d = 2
    cen = _lattice_centres(d, 8)
    v = _bumps(d, n, cen, [4.0] * len(cen), [2.0] * len(cen))
    return Problem("schrod2d_lattice", d, n, np.ascontiguousarray(v), _random_rhs(d, n, seed + 1),
                   t=t, num_shifts=num_shifts or max(1, n // 16))


def schrod3d_wells(n: int = 32, seed: int = 0, t: int = 1, num_shifts=None) -> Problem:
    """3D Schroedinger: 16 Gaussian bumps at random centres."""
    d = 3
    rng = np.random.default_rng(seed)
    centres = rng.random((16, d))
    height = rng.uniform(2.0, 6.0, 16)
    width = rng.uniform(1.5, 3.0, 16)
    v = _bumps(d, n, centres, height, width)
    return Problem("schrod3d_wells", d, n, np.ascontiguousarray(v), _random_rhs(d, n, seed + 1),
                   t=t, num_shifts=num_shifts or max(1, n // 4))


def schrod3d_lattice(n: int = 32, seed: int = 0, t: int = 1, num_shifts=None) -> Problem:
    """3D Schroedinger: a 4 x 4 x 4 lattice of equal bumps, the centre one missing."""
    d = 3
    cen = _lattice_centres(d, 4)
    v = _bumps(d, n, cen, [4.0] * len(cen), [1.5] * len(cen))
    return Problem("schrod3d_lattice", d, n, np.ascontiguousarray(v), _random_rhs(d, n, seed + 1),
                   t=t, num_shifts=num_shifts or max(1, n // 4))


def random_field_v(d: int, n: int, seed: int, lo: float, hi: float) -> np.ndarray:
    """Uniform random potential in [lo, hi] (for tests of host logic and edge cases)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, (n,) * d)


CONFIGS = {
    "helm2d_gauss_n32": lambda: helm2d_gauss(32),
    "schrod2d_wells_n256": lambda: schrod2d_wells(256),
    "helm2d_random_n1024": lambda: helm2d_random(1024),
    "helm3d_random_n64": lambda: helm3d_random(64),
    "helm2d_cross_n128": lambda: helm2d_cross(128),
    "helm3d_gauss_n32": lambda: helm3d_gauss(32),
    "helm3d_cross_n32": lambda: helm3d_cross(32),
    "schrod2d_lattice_n128": lambda: schrod2d_lattice(128),
    "schrod3d_wells_n32": lambda: schrod3d_wells(32),
    "schrod3d_lattice_n32": lambda: schrod3d_lattice(32),
}


def make(name: str) -> Problem:
    return CONFIGS[name]()
