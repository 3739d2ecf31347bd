"""Seeded synthetic inputs shared by the oracle and the GPU path.

This module only draws random numbers and evaluates the prescribed initial
fields at given points.  It contains none of the discretisation: no shape
functions, quadrature, assembly or solver arithmetic.  Both the oracle and the
HIP path receive the same arrays from here; each side builds its own mesh and
passes its own node coordinates in.

Workload recipes (unit domain [0,1]^d, integer node coordinates scaled by
2^-max_level):

* multi-drop pressure problem (3D, uniform level 7): 8 drops with radius
  U[0.05, 0.15] and centre U[R, 1-R]^3, Cn = 0.01, density ratio 1000.  The
  phase field is -1 + sum_d [1 + tanh((R_d - |x - c_d|)/(sqrt(2) Cn))] so that
  the drops are the phi = +1 (heavy, rho = 1) phase.
* right-hand side f = sum_k a_k cos(l_k pi x) cos(m_k pi y) cos(n_k pi z),
  a_k ~ N(0,1), (l,m,n)_k ~ U{0..4}^3 without (0,0,0).
* rising bubble (3D adaptive): centre (0.5, 0.3, 0.5), radius 0.15, the bubble
  is the light phase: phi = tanh((|x - c| - R)/(sqrt(2) Cn)).
* 2D drop (uniform 64x64): phi = tanh((0.25 - |x - (0.5,0.5)|)/(sqrt(2) Cn)).
"""
from __future__ import annotations

import numpy as np

SQRT2 = float(np.sqrt(2.0))


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def normal_vector(seed: int, n: int) -> np.ndarray:
    """Seeded N(0,1) vector of length n (float64)."""
    return rng(seed).standard_normal(n)


def drops(seed: int, n_drops: int = 8, rmin: float = 0.05, rmax: float = 0.15, dim: int = 3):
    """Radii R_d ~ U[rmin, rmax] and centres c_d ~ U[R_d, 1 - R_d]^dim."""
    g = rng(seed)
    radii = g.uniform(rmin, rmax, size=n_drops)
    centres = np.empty((n_drops, dim))
    for k in range(n_drops):
        centres[k] = g.uniform(radii[k], 1.0 - radii[k], size=dim)
    return centres, radii


def phi_drops(x: np.ndarray, centres: np.ndarray, radii: np.ndarray, cn: float) -> np.ndarray:
    """Multi-drop phase field at points x (n, dim)."""
    out = np.full(x.shape[0], -1.0)
    for c, r in zip(centres, radii):
        dist = np.sqrt(((x - c[None, :]) ** 2).sum(axis=1))
        out += 1.0 + np.tanh((r - dist) / (SQRT2 * cn))
    return out


def phi_bubble(x: np.ndarray, centre=(0.5, 0.3, 0.5), radius: float = 0.15, cn: float = 0.01) -> np.ndarray:
    """Light bubble (phi = -1 inside) in the heavy phase."""
    c = np.asarray(centre, dtype=np.float64)[: x.shape[1]]
    dist = np.sqrt(((x - c[None, :]) ** 2).sum(axis=1))
    return np.tanh((dist - radius) / (SQRT2 * cn))


def phi_drop2d(x: np.ndarray, centre=(0.5, 0.5), radius: float = 0.25, cn: float = 0.02) -> np.ndarray:
    """Heavy drop (phi = +1 inside) in 2D."""
    c = np.asarray(centre, dtype=np.float64)
    dist = np.sqrt(((x - c[None, :]) ** 2).sum(axis=1))
    return np.tanh((radius - dist) / (SQRT2 * cn))


def rhs_modes(seed: int, n_modes: int = 8, kmax: int = 4, dim: int = 3):
    """Amplitudes a_k ~ N(0,1) and integer wave numbers in U{0..kmax}^dim minus 0."""
    g = rng(seed)
    amps = g.standard_normal(n_modes)
    waves = np.zeros((n_modes, dim), dtype=np.int64)
    for k in range(n_modes):
        while True:
            w = g.integers(0, kmax + 1, size=dim)
            if w.any():
                break
        waves[k] = w
    return amps, waves


def rhs_field(x: np.ndarray, amps: np.ndarray, waves: np.ndarray) -> np.ndarray:
    """f(x) = sum_k a_k prod_d cos(w_kd pi x_d) at points x (n, dim)."""
    out = np.zeros(x.shape[0])
    for a, w in zip(amps, waves):
        term = np.full(x.shape[0], a)
        for d in range(x.shape[1]):
            term = term * np.cos(w[d] * np.pi * x[:, d])
        out += term
    return out


def unit_coords(ijk: np.ndarray, max_level: int) -> np.ndarray:
    """Integer node coordinates (units of 2^-max_level) to unit-domain floats."""
    return np.asarray(ijk, dtype=np.float64) / float(1 << max_level)


# ---- incomplete (carved) octree: the paper's 3D Rayleigh-Taylor column
# The 1 x 8 x 1 box is the part x < 1/8, z < 1/8 of the unit root cube
# (carve level 3, extent (1, 8, 1)); physical lengths are 8 x unit ones.
RT_CARVE_LEVEL = 3
RT_EXTENT = (1, 8, 1)


def phi_rt(x: np.ndarray, cn: float, l: float = 6.0, amp: float = 0.05) -> np.ndarray:
    """phi = tanh(sqrt2 (x2 - l - g(x)) / Cn), g = amp (cos 2 pi x1 + cos 2 pi x3)
    in physical units (unit coordinates x times 8); 2D: g = amp cos 2 pi x1."""
    X = 8.0 * np.asarray(x, dtype=np.float64)
    g = amp * np.cos(2 * np.pi * X[:, 0])
    if X.shape[1] == 3:
        g = g + amp * np.cos(2 * np.pi * X[:, 2])
    return np.tanh(SQRT2 * (X[:, 1] - l - g) / cn)


def rt_slab_meets(lo_y: float, hi_y: float, width: float, l: float = 6.0) -> bool:
    """Refinement predicate of the Rayleigh-Taylor meshes: the octant's
    vertical extent (unit coordinates) meets the slab |8 y - l| <= width."""
    return 8.0 * lo_y <= l + width and 8.0 * hi_y >= l - width
