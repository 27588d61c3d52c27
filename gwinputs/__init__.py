"""Seeded synthetic inputs shared by the CPU oracle and the HIP path.

This module only *generates inputs*: grids, conductivity fields, boundary
heads and well layouts.  It contains none of the solver's arithmetic
(no assembly, no AMG, no Krylov), so both sides can take their inputs
from here without sharing any of the method's code.

The paper's own aquifer models (a 2D field-scale geothermal doublet model and
its 10-layer 3D extension, Benchmarking Examples section) and their lognormal
K realizations (variance of ln K equal to 10) are not published with the
paper.  The generator below stands in for them: a stationary Gaussian ln K
field with exponential covariance, drawn by circulant embedding (Dietrich &
Newsam 1997), which is the spectral method used for such fields.

Array layout everywhere: cell (i, j, k) lives at flat index
``i + nx * (j + ny * k)`` (x fastest); a numpy field therefore has shape
``(nz, ny, nx)`` in C order.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Tuple

import numpy as np

__all__ = [
    "Grid", "Well", "Problem", "lognormal_field", "four_well_layout",
    "homogeneous_slab", "heterogeneous_aquifer", "serve_stream", "doublet_layout",
    "paper_like_aquifer",
]

K_GEO_DEFAULT = 1.0e-4   # geometric-mean conductivity [m/s]
H_WEST_DEFAULT = 10.0    # fixed head on the x = 0 face [m]
H_EAST_DEFAULT = 0.0     # fixed head on the x = L face [m]
PHI_DEFAULT = 0.25       # porosity used in the travel-time equation
K_PAPER = 6.38e-5        # K_mean of the paper's benchmark models [m/s]


@dataclasses.dataclass(frozen=True)
class Grid:
    nx: int
    ny: int
    nz: int
    dx: float = 1.0
    dy: float = 1.0
    dz: float = 1.0

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz


@dataclasses.dataclass(frozen=True)
class Well:
    """Point sink in cell (ix, iy, iz); ``q`` > 0 is a pumping rate [m^3/s]."""
    ix: int
    iy: int
    iz: int
    q: float


@dataclasses.dataclass
class Problem:
    """One confined-aquifer flow problem plus what travel time needs."""
    grid: Grid
    K: np.ndarray                      # float64, shape (n,), natural order
    h_west: float = H_WEST_DEFAULT
    h_east: float = H_EAST_DEFAULT
    wells: List[Well] = dataclasses.field(default_factory=list)
    phi: float = PHI_DEFAULT
    label: str = ""


def _min_image_lags(m: int) -> np.ndarray:
    a = np.arange(m, dtype=np.float64)
    return np.minimum(a, m - a)


def lognormal_field(shape_xyz: Tuple[int, int, int], sigma2: float,
                    corr_len: float, seed: int,
                    k_geo: float = K_GEO_DEFAULT,
                    return_clip: bool = False):
    """ln K = ln(k_geo) + Y with Y ~ N(0, C), C(r) = sigma2 * exp(-r / corr_len).

    r is the Euclidean lag measured in cells.  Circulant embedding on a grid
    padded to twice the model size in every direction:

    1. c = covariance at the periodic minimum-image lags of the padded grid;
    2. Lambda = Re(FFT(c)), negative eigenvalues clipped to zero;
    3. eps ~ N(0, 1) on the padded grid from ``numpy.random.default_rng(seed)``;
    4. Y = IFFT(sqrt(Lambda) * FFT(eps)), cropped to the model grid.

    With unnormalized forward FFT F and IFFT = F^H / M, Cov(Y) = F^H Lambda F / M,
    which is the circulant whose first column is c.

    Returns K flattened in natural order (x fastest); optionally also the
    fraction of clipped (negative) eigenvalues.
    """
    nx, ny, nz = (int(s) for s in shape_xyz)
    if sigma2 == 0.0:
        K = np.full(nx * ny * nz, float(k_geo))
        return (K, 0.0) if return_clip else K
    mx, my, mz = 2 * nx, 2 * ny, (2 * nz if nz > 1 else 1)
    lz = _min_image_lags(mz)[:, None, None]
    ly = _min_image_lags(my)[None, :, None]
    lx = _min_image_lags(mx)[None, None, :]
    r = np.sqrt(lx * lx + ly * ly + lz * lz)
    c = sigma2 * np.exp(-r / float(corr_len))
    lam = np.fft.rfftn(c).real
    neg = lam < 0.0
    clip_frac = float(neg.mean())
    lam[neg] = 0.0
    rng = np.random.default_rng(seed)
    eps = rng.standard_normal((mz, my, mx))
    y = np.fft.irfftn(np.sqrt(lam) * np.fft.rfftn(eps), s=(mz, my, mx), axes=(0, 1, 2))
    y = y[:nz, :ny, :nx]
    K = np.exp(np.log(k_geo) + y).reshape(-1).astype(np.float64)
    K = np.ascontiguousarray(K)
    return (K, clip_frac) if return_clip else K


def four_well_layout(grid: Grid, k_geo: float = K_GEO_DEFAULT,
                     dh: float = H_WEST_DEFAULT - H_EAST_DEFAULT,
                     share: float = 0.1) -> List[Well]:
    """Four pumping wells at (nx/4|3nx/4, ny/4|3ny/4, nz/2).

    Each pumps ``share * k_geo * (dh / L) * (W * H)``: with share 0.1 the four
    wells together take 40 % of the nominal regional through-flow.
    """
    L = grid.nx * grid.dx
    W = grid.ny * grid.dy
    H = grid.nz * grid.dz
    q = share * k_geo * (dh / L) * (W * H)
    iz = grid.nz // 2
    xs = (grid.nx // 4, (3 * grid.nx) // 4)
    ys = (grid.ny // 4, (3 * grid.ny) // 4)
    return [Well(xs[0], ys[0], iz, q), Well(xs[1], ys[0], iz, q),
            Well(xs[0], ys[1], iz, q), Well(xs[1], ys[1], iz, q)]


def homogeneous_slab(nx: int = 64, ny: int = 64, nz: int = 1,
                     k: float = K_GEO_DEFAULT) -> Problem:
    """Homogeneous confined slab, fixed heads 10 m / 0 m on the x faces."""
    g = Grid(nx, ny, nz)
    return Problem(g, np.full(g.n, float(k)), label=f"homogeneous {nx}x{ny}x{nz}")


def heterogeneous_aquifer(nx: int, ny: int, nz: int, sigma2: float,
                          corr_len: float, seed: int, wells: bool = True) -> Problem:
    """Lognormal aquifer with the four-well layout (3D cases)."""
    g = Grid(nx, ny, nz)
    K = lognormal_field((nx, ny, nz), sigma2, corr_len, seed)
    w = four_well_layout(g) if wells else []
    return Problem(g, K, wells=w,
                   label=f"lognormal {nx}x{ny}x{nz} s2={sigma2} lam={corr_len} seed={seed}")


def doublet_layout(grid: Grid, rate: float, n_screen: int = 5) -> List[Well]:
    """Four injection/production doublets (the paper's geothermal model has
    four, at positions it does not give).  Injectors at (3nx/10 | 7nx/10,
    ny/4 | 3ny/4) are screened over the lowest ``n_screen`` layers, their
    producers nx/10 cells downstream over the top ``n_screen`` layers; each
    well moves ``rate`` m^3/s, split evenly over its screened cells (q < 0
    injects)."""
    ns = max(1, min(n_screen, grid.nz))
    q = rate / ns
    wells = []
    for y in (grid.ny // 4, (3 * grid.ny) // 4):
        for x in ((3 * grid.nx) // 10, (7 * grid.nx) // 10):
            xp = min(grid.nx - 1, x + max(1, grid.nx // 10))
            wells += [Well(x, y, k, -q) for k in range(ns)]
            wells += [Well(xp, y, grid.nz - 1 - k, q) for k in range(ns)]
    return wells


def paper_like_aquifer(sigma2: float = 10.0, corr_len: float = 10.0, seed: int = 31, nz: int = 10,
                       rate: float = 0.02) -> Problem:
    """Stand-in for the paper's geothermal model (Benchmarking Examples):
    550 x 500 blocks of 20 m in every direction, ``nz`` layers (10: the 3D
    extension, 2.75M blocks; 1: the 2D model), K_mean = 6.38e-5 m/s taken as
    the geometric mean of a lognormal field of variance ``sigma2`` (10 in the
    paper; 0 gives its homogeneous case), four doublets with partially
    penetrating wells (``doublet_layout``).  The paper's boundaries are all
    no-flow, which leaves the flow matrix singular; fixed heads on the two
    x faces stand in for them."""
    g = Grid(550, 500, nz, 20.0, 20.0, 20.0)
    K = lognormal_field((g.nx, g.ny, g.nz), sigma2, corr_len, seed, k_geo=K_PAPER)
    return Problem(g, K, wells=doublet_layout(g, rate),
                   label=f"paper-like 550x500x{nz} s2={sigma2} lam={corr_len} seed={seed}")


@dataclasses.dataclass(frozen=True)
class Arrival:
    t: float          # arrival time [s] from the start of the stream
    side: int         # cubic grid side length
    sigma2: float
    corr_len: float
    seed: int


def serve_stream(n_requests: int, rate_hz: float, seed: int = 5,
                 side_min: int = 32, side_max: int = 192) -> List[Arrival]:
    """Poisson arrivals of cubic problems with uniform side length.

    Side ~ U{side_min..side_max}, sigma2 ~ U{1, 2, 4}, correlation length
    ~ U{4..16} cells; each request gets its own field seed.
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, size=n_requests)
    t = np.cumsum(gaps) - gaps[0]
    sides = rng.integers(side_min, side_max + 1, size=n_requests)
    s2 = rng.choice(np.array([1.0, 2.0, 4.0]), size=n_requests)
    lam = rng.integers(4, 17, size=n_requests)
    seeds = rng.integers(1, 2**31 - 1, size=n_requests)
    return [Arrival(float(t[i]), int(sides[i]), float(s2[i]), float(lam[i]), int(seeds[i]))
            for i in range(n_requests)]


def problem_for_arrival(a: Arrival) -> Problem:
    return heterogeneous_aquifer(a.side, a.side, a.side, a.sigma2, a.corr_len, a.seed)


def random_k(grid: Grid, seed: int, lo: float = 1e-6, hi: float = 1e-2) -> np.ndarray:
    """Log-uniform uncorrelated K (small-grid pins)."""
    rng = np.random.default_rng(seed)
    return np.exp(rng.uniform(np.log(lo), np.log(hi), size=grid.n)).astype(np.float64)


def random_vector(n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.standard_normal(n).astype(np.float64)


def _csr_from_pairs(n: int, i: np.ndarray, j: np.ndarray, w: np.ndarray, diag: np.ndarray):
    """CSR (sorted columns) of the symmetric matrix with off-diagonal
    entries (i, j, w) and (j, i, w) and the given diagonal."""
    rows = np.concatenate([i, j, np.arange(n)])
    cols = np.concatenate([j, i, np.arange(n)])
    vals = np.concatenate([w, w, diag])
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    rowptr = np.zeros(n + 1, dtype=np.int32)
    np.add.at(rowptr, rows + 1, 1)
    return np.cumsum(rowptr).astype(np.int32), cols.astype(np.int32), vals.astype(np.float64)


def random_graph_spd(n: int, deg: int, seed: int):
    """Symmetric, strictly diagonally dominant M-matrix on a random graph
    (close to 2*deg neighbours in every row, at arbitrary column distance): an
    operator with no stencil structure.  Returns (rowptr, col, val)."""
    rng = np.random.default_rng(seed)
    i = np.tile(np.arange(n), deg)
    j = np.concatenate([rng.permutation(n) for _ in range(deg)])
    i, j = np.minimum(i, j), np.maximum(i, j)
    keep = i < j
    i, j = i[keep], j[keep]
    key = np.unique(i.astype(np.int64) * n + j)
    i, j = (key // n).astype(np.int64), (key % n).astype(np.int64)
    w = -rng.uniform(0.5, 1.5, size=len(i))
    off = np.zeros(n)
    np.add.at(off, i, -w)
    np.add.at(off, j, -w)
    return _csr_from_pairs(n, i, j, w, off + rng.uniform(0.1, 1.0, size=n))


def arrow_spd(n: int, seed: int, stride: int = 2, weak: float = 0.01):
    """1-D chain (a tridiagonal M-matrix) plus weak couplings between row 0
    and every `stride`-th row: one row far longer than the rest.  Returns
    (rowptr, col, val)."""
    rng = np.random.default_rng(seed)
    ci = np.arange(n - 1)
    cw = -rng.uniform(0.5, 1.5, size=n - 1)
    aj = np.arange(stride, n, stride)
    aj = aj[aj > 1]
    aw = np.full(len(aj), -weak)
    i = np.concatenate([ci, np.zeros(len(aj), dtype=np.int64)])
    j = np.concatenate([ci + 1, aj])
    w = np.concatenate([cw, aw])
    off = np.zeros(n)
    np.add.at(off, i, -w)
    np.add.at(off, j, -w)
    return _csr_from_pairs(n, i, j, w, off + rng.uniform(0.1, 1.0, size=n))
