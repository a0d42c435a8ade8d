"""Seeded synthetic inputs: permeability fields, right-hand sides, manufactured data.

This module holds no arithmetic of the method (no discretisation, no local
solves, no coupling).  It only draws or evaluates problem data, and both the
HIP path and the oracle receive its arrays as inputs.

Cell ``(ix, iy)`` of an ``nx x ny`` grid has id ``iy * nx + ix`` (x fastest);
cell (0, 0) touches the corner x = 0, y = 0.  On an ``nx x ny x nz`` grid cell
``(ix, iy, iz)`` has id ``(iz * ny + iy) * nx + ix``.  Arrays are float64,
length n.

Field recipes (stand-ins for the paper's workloads; the paper's SPE10 layers
and inclusion geometries are not reproduced):

* Gaussian random field: white noise from ``numpy.random.Generator(PCG64(seed))``
  on a grid padded by ceil(3 * ell) cells per side, convolved along each axis
  with the kernel exp(-2 t^2 / ell^2) normalised to unit L2 norm, then cropped.
  This gives unit variance and covariance exp(-r^2 / ell^2).
* Log-normal K = exp(sigma * G).
* 3-D Gaussian random field: the same recipe on an (nz, ny, nx) array, one
  correlation length on every axis, convolved along x, then y, then z.
* Channel facies: chi = [G(ell_x, ell_y) > 0]; K = k_hi on chi, k_lo elsewhere.
* Mixture (contrast 1e8): channel facies chi = [G1(160, 24) > 0] at a facies
  contrast of 1e4 times a log-normal factor, K_raw = exp(G2) * (chi + 1e-4
  (1 - chi)) with G2 of correlation 32, then ln K stretched affinely so that
  the field spans exactly the contrast: K = exp(ln(contrast) (ln K_raw -
  min) / (max - min)), so max K = 1 and min K = 1 / contrast.  (A facies
  contrast of the full 1e8 at this 50 % channel fraction leaves the shale
  cells nearly disconnected, close to the percolation threshold: there the
  restarted GMRES of the method stalls at 2048^2 and above.)
* Thin inclusions (stand-in for the paper's inclusion fields, Section 4.3):
  background K = 1 with straight segments one cell thick, horizontal or
  vertical with equal probability, lengths uniform in [0.15, 0.45] of the
  grid side, start cells uniform (``Generator(PCG64(seed))``).  High
  inclusions have K = contrast, low ones 1 / contrast; the combined field
  draws the high segments first and the low ones after them (written over
  any crossing), so its contrast ratio is contrast^2.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.signal import fftconvolve


def _kernel(ell: float) -> np.ndarray:
    half = int(math.ceil(3.0 * ell))
    t = np.arange(-half, half + 1, dtype=np.float64)
    k = np.exp(-2.0 * t * t / (ell * ell))
    return k / np.sqrt(np.sum(k * k))


def gaussian_field(nx: int, ny: int, ell_x: float, ell_y: float | None = None,
                   seed: int = 0) -> np.ndarray:
    """Unit-variance Gaussian field with Gaussian covariance, shape (ny, nx)."""
    if ell_y is None:
        ell_y = ell_x
    px = int(math.ceil(3.0 * ell_x))
    py = int(math.ceil(3.0 * ell_y))
    rng = np.random.Generator(np.random.PCG64(seed))
    w = rng.standard_normal((ny + 2 * py, nx + 2 * px))
    kx = _kernel(ell_x)
    ky = _kernel(ell_y)
    g = fftconvolve(w, kx[None, :], mode="same", axes=1)
    g = fftconvolve(g, ky[:, None], mode="same", axes=0)
    return np.ascontiguousarray(g[py:py + ny, px:px + nx])


def lognormal_K(nx: int, ny: int, sigma: float, ell: float, seed: int) -> np.ndarray:
    return np.exp(sigma * gaussian_field(nx, ny, ell, ell, seed)).ravel()


def gaussian_field3(nx: int, ny: int, nz: int, ell: float, seed: int) -> np.ndarray:
    """Unit-variance 3-D Gaussian field with Gaussian covariance, shape (nz, ny, nx)."""
    pad = int(math.ceil(3.0 * ell))
    rng = np.random.Generator(np.random.PCG64(seed))
    w = rng.standard_normal((nz + 2 * pad, ny + 2 * pad, nx + 2 * pad))
    k = _kernel(ell)
    g = fftconvolve(w, k[None, None, :], mode="same", axes=2)
    g = fftconvolve(g, k[None, :, None], mode="same", axes=1)
    g = fftconvolve(g, k[:, None, None], mode="same", axes=0)
    return np.ascontiguousarray(g[pad:pad + nz, pad:pad + ny, pad:pad + nx])


def lognormal_K3(nx: int, ny: int, nz: int, sigma: float, ell: float, seed: int) -> np.ndarray:
    return np.exp(sigma * gaussian_field3(nx, ny, nz, ell, seed)).ravel()


def channel_K(nx: int, ny: int, ell_x: float, ell_y: float, seed: int,
              k_hi: float = 1.0, k_lo: float = 1e-6) -> np.ndarray:
    chi = gaussian_field(nx, ny, ell_x, ell_y, seed) > 0.0
    return np.where(chi, k_hi, k_lo).astype(np.float64).ravel()


def mixture_K(nx: int, ny: int, seed_channels: int, seed_lognormal: int,
              contrast: float = 1e8, facies_contrast: float = 1e4) -> np.ndarray:
    chi = (gaussian_field(nx, ny, 160.0, 24.0, seed_channels) > 0.0).astype(np.float64)
    g2 = gaussian_field(nx, ny, 32.0, 32.0, seed_lognormal)
    lraw = g2 + np.log(chi + (1.0 / facies_contrast) * (1.0 - chi))
    lo, hi = lraw.min(), lraw.max()
    return np.exp(np.log(contrast) * ((lraw - lo) / (hi - lo) - 1.0)).ravel()


def _segments(rng: np.random.Generator, nx: int, ny: int, count: int) -> list:
    """count thin straight segments as lists of cell ids."""
    out = []
    for _ in range(count):
        horizontal = rng.random() < 0.5
        side = nx if horizontal else ny
        length = int(rng.integers(int(0.15 * side), int(0.45 * side) + 1))
        if horizontal:
            x0, y = int(rng.integers(0, nx - length + 1)), int(rng.integers(0, ny))
            out.append([y * nx + x for x in range(x0, x0 + length)])
        else:
            x, y0 = int(rng.integers(0, nx)), int(rng.integers(0, ny - length + 1))
            out.append([y * nx + x for y in range(y0, y0 + length)])
    return out


def inclusions_K(nx: int, ny: int, kind: str, seed: int, count: int = 24,
                 contrast: float = 1e4) -> np.ndarray:
    """Thin high ('high'), low ('low') or both kinds ('both') of inclusions on
    a background K = 1, count segments per kind."""
    if kind not in ("high", "low", "both"):
        raise ValueError(kind)
    rng = np.random.Generator(np.random.PCG64(seed))
    K = np.ones(nx * ny)
    if kind in ("high", "both"):
        for seg in _segments(rng, nx, ny, count):
            K[seg] = contrast
    if kind in ("low", "both"):
        for seg in _segments(rng, nx, ny, count):
            K[seg] = 1.0 / contrast
    return K


def dirichlet_left_right(nx: int, ny: int, left: float = 1.0, right: float = 0.0):
    """Boundary data of the paper's Dirichlet left/right problems (pressure
    `left` at x = 0, `right` at x = 1, no flow on the other sides, no source):
    (f, g) with g the W, E, S, N face values in the order of the ABI."""
    g = np.concatenate([np.full(ny, left), np.full(ny, right), np.zeros(nx), np.zeros(nx)])
    return np.zeros(nx * ny), g


def corner_sources(nx: int, ny: int) -> np.ndarray:
    """Point injector +1 in cell (0, 0) and producer -1 in cell (nx-1, ny-1)."""
    b = np.zeros(nx * ny)
    b[0] = 1.0
    b[nx * ny - 1] = -1.0
    return b


def corner_sources3(nx: int, ny: int, nz: int) -> np.ndarray:
    """Point injector +1 in cell (0, 0, 0) and producer -1 in the opposite corner cell."""
    b = np.zeros(nx * ny * nz)
    b[0] = 1.0
    b[-1] = -1.0
    return b


def random_pairs(nx: int, ny: int, nrhs: int, seed: int) -> np.ndarray:
    """nrhs right-hand sides e_inj - e_prod with distinct uniform cells, shape (nrhs, n)."""
    n = nx * ny
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.zeros((nrhs, n))
    for r in range(nrhs):
        a, b = rng.choice(n, size=2, replace=False)
        out[r, a] = 1.0
        out[r, b] = -1.0
    return out


def random_vector(n: int, seed: int, zero_mean: bool = False) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    v = rng.standard_normal(n)
    if zero_mean:
        v -= v.mean()
    return v


def cell_centres(nx: int, ny: int, lx: float = 1.0, ly: float | None = None):
    """Cell-centre coordinates (x, y) as flat arrays, square cells of side lx / nx."""
    h = lx / nx
    ix = np.arange(nx)
    iy = np.arange(ny)
    X, Y = np.meshgrid((ix + 0.5) * h, (iy + 0.5) * h)
    return X.ravel(), Y.ravel()


# Manufactured problems of the paper's Section 4 (unit square).
def manufactured(case: str):
    """Return (K(x, y), f(x, y), p(x, y)) callables for case 'const' or 'var'."""
    pi = math.pi
    if case == "const":
        return (lambda x, y: np.ones_like(x),
                lambda x, y: 8 * pi * pi * np.cos(2 * pi * x) * np.cos(2 * pi * y),
                lambda x, y: np.cos(2 * pi * x) * np.cos(2 * pi * y))
    if case == "var":
        return (lambda x, y: 1.0 + np.sin(pi * x) * np.sin(pi * y),
                lambda x, y: 2 * pi * pi * np.cos(pi * x) * np.cos(pi * y)
                * (1.0 + 2.0 * np.sin(pi * x) * np.sin(pi * y)),
                lambda x, y: np.cos(pi * x) * np.cos(pi * y))
    raise ValueError(case)
