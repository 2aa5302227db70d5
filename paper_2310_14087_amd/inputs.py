"""Seeded synthetic problem generator shared by the oracle-side tests, the GPU tests and the bench.

This module holds none of the method's arithmetic: it only draws samples and filling points and fixes the
bandwidth and regularisers of each workload.  Every array is float64, row-major, C-contiguous.

Workloads (the paper's experiments, Section 5, use mixtures of Gaussians, quasi-random filling points and
lambda1 = 1/l, lambda2 = 1/sqrt(n_sample); the shapes below follow that recipe at the sizes this library targets):

* ``tiny``     n=100/side, d=2, N(0,I) vs N((1,1),I), l=50, sigma=1, lambda1=lambda2=1e-3, tol 1e-8.
* ``gauss500`` n=2000/side, d=5, N(0,I) vs N(m, AA^T/5 + 0.1I), m ~ U[-1,1]^5, l=500.
* ``mix1000``  n=5000/side, d=10, two 4-component unit-covariance mixtures, means ~ U[-2,2]^10, l=1000.
* ``mix1000_median``  the same draw on raw coordinates with sigma = the median pooled pairwise distance (a
               dense kernel: the coupled form of the l=1000 workload).
* ``batch``    one problem of the uneven batch: n ~ U{200..2000}, l ~ U{100..400}, d ~ U{2..10},
               N(0,I) vs N(s, I), s ~ U[-1,1]^d.
* ``mix256``   n=1000/side, d=8, two 3-component unit-covariance mixtures, means ~ U[-2,2]^8, l=256.

Filling points: x~ uniform in the bounding box of the source samples, y~ uniform in the bounding box of the
target samples (a point of X x Y, Section 3).

Bandwidth and scale:
* ``tiny``: raw coordinates, sigma = 1 (fixed by the workload's definition).
* ``gauss500``, ``mix1000_median``: raw coordinates, sigma = median of all pooled pairwise Euclidean distances.
* ``mix1000``, ``mix256``, ``batch`` (no bandwidth in their definition): the paper's own recipe (Section 5):
  samples affinely mapped into the unit cube (pooled bounding box, one common scale so the cost keeps its
  geometry), filling points uniform in the unit-cube boxes of each side, sigma^2 = 0.005.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = ["Problem", "make_problem", "make_custom", "median_pairwise_distance", "WORKLOADS"]

WORKLOADS = ("tiny", "gauss500", "mix1000", "mix1000_median", "batch", "mix256", "sweep_d2", "sweep_d5", "sweep_d10",
             "cells48")

# Seed offsets per workload: seed = base + s.
_SEED_BASE = {"tiny": 1000, "gauss500": 2000, "mix1000": 3000, "mix1000_median": 3000, "batch": 4000, "mix256": 5000, "sweep_d2": 6000,
              "sweep_d5": 7000, "sweep_d10": 8000, "cells48": 9000}


@dataclass
class Problem:
    name: str
    seed: int
    xs: np.ndarray  # n_src x d
    ys: np.ndarray  # n_tgt x d
    xf: np.ndarray  # l x d
    yf: np.ndarray  # l x d
    sigma: float
    lam1: float
    lam2: float
    tol: float
    meta: dict = field(default_factory=dict)

    @property
    def l(self) -> int:
        return self.xf.shape[0]

    @property
    def d(self) -> int:
        return self.xs.shape[1]

    @property
    def n_src(self) -> int:
        return self.xs.shape[0]

    @property
    def n_tgt(self) -> int:
        return self.ys.shape[0]


def median_pairwise_distance(xs: np.ndarray, ys: np.ndarray, chunk: int = 1024) -> float:
    """Exact median of the Euclidean distances over all unordered pairs of the pooled samples."""
    pts = np.concatenate([xs, ys], axis=0)
    n = pts.shape[0]
    sq = np.einsum("ij,ij->i", pts, pts)
    parts = []
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        blk = pts[s:e]
        d2 = sq[s:e, None] + sq[None, :] - 2.0 * blk @ pts.T
        for r in range(e - s):
            i = s + r
            row = d2[r, i + 1:]
            parts.append(row)
    d2all = np.concatenate(parts)
    np.maximum(d2all, 0.0, out=d2all)
    return float(np.sqrt(np.median(d2all)))


def _box_uniform(rng: np.random.Generator, pts: np.ndarray, l: int) -> np.ndarray:
    lo = pts.min(axis=0)
    hi = pts.max(axis=0)
    return lo + (hi - lo) * rng.random((l, pts.shape[1]))


PAPER_SIGMA = float(np.sqrt(0.005))


def _unit_cube(xs: np.ndarray, ys: np.ndarray):
    pts = np.concatenate([xs, ys], axis=0)
    lo = pts.min(axis=0)
    scale = float((pts.max(axis=0) - lo).max())
    return (xs - lo) / scale, (ys - lo) / scale


def _mixture(rng: np.random.Generator, means: np.ndarray, n: int) -> np.ndarray:
    lab = rng.integers(0, means.shape[0], size=n)
    return means[lab] + rng.standard_normal((n, means.shape[1]))


def sobol_filling(rng: np.random.Generator, l: int, d: int):
    """l filling points (x~_i, y~_i) from a scrambled Sobol sequence in [0, 1]^(2d), split into the x- and
    y-halves (the joint points of Section 5's synthetic setup)."""
    import warnings
    from scipy.stats import qmc
    with warnings.catch_warnings():  # balance is exact only for powers of two; any l is accepted
        warnings.simplefilter("ignore", UserWarning)
        pts = qmc.Sobol(d=2 * d, scramble=True, seed=rng).random(l)
    return np.ascontiguousarray(pts[:, :d]), np.ascontiguousarray(pts[:, d:])


def _sweep(rng: np.random.Generator, name: str, seed: int, d: int, l_: int, n_: int, meta: dict) -> Problem:
    """Section 5's synthetic setup: mu a mixture of 3 and nu a mixture of 5 Gaussians in R^d (equal weights,
    identity covariance, means uniform in [-2, 2]^d), the samples scaled jointly into the unit cube, l filling
    points from a 2d-dimensional Sobol sequence, sigma^2 = 0.005, lambda1 = 1/l, lambda2 = 1/sqrt(n), stop at
    |R(w)| < 0.005."""
    mx = rng.uniform(-2.0, 2.0, size=(3, d))
    my = rng.uniform(-2.0, 2.0, size=(5, d))
    xs = _mixture(rng, mx, n_)
    ys = _mixture(rng, my, n_)
    xs, ys = _unit_cube(xs, ys)
    xf, yf = sobol_filling(rng, l_, d)
    meta.update(components=(3, 5))
    return Problem(name, seed, xs, ys, xf, yf, sigma=PAPER_SIGMA, lam1=1.0 / l_, lam2=1.0 / np.sqrt(n_),
                   tol=0.005, meta=meta)


def _cells48(rng: np.random.Generator, name: str, seed: int, l_: int, n_: int, meta: dict) -> Problem:
    """Synthetic stand-in with the shapes of the single-cell comparison (48 features, 256 filling points): an
    'unperturbed' population of 6 clusters with random anisotropic covariances and a 'perturbed' one in which
    every cluster is shifted and rescaled and the cluster weights change; the samples are scaled jointly into
    the unit cube, the filling points come from a 96-dimensional Sobol sequence and the bandwidth is a third of
    the median pairwise distance (at the median itself the iteration stalls near |R| ~ 1e-5 at these sizes; no
    cell measurements are used)."""
    d, k = 48, 6
    means = rng.uniform(-1.0, 1.0, size=(k, d))
    facs = [rng.standard_normal((d, d)) / np.sqrt(d) * rng.uniform(0.2, 0.6) for _ in range(k)]
    wx = rng.dirichlet(np.ones(k))
    wy = rng.dirichlet(np.ones(k))
    shift = 0.4 * rng.standard_normal((k, d)) / np.sqrt(d) * 4.0
    scale = rng.uniform(0.7, 1.3, size=k)

    def draw(w, perturbed):
        lab = rng.choice(k, size=n_, p=w)
        z = rng.standard_normal((n_, d))
        out = np.empty((n_, d))
        for j in range(k):
            idx = lab == j
            v = z[idx] @ facs[j].T
            out[idx] = means[j] + (shift[j] + scale[j] * v if perturbed else v)
        return out

    xs = draw(wx, False)
    ys = draw(wy, True)
    xs, ys = _unit_cube(xs, ys)
    xf, yf = sobol_filling(rng, l_, d)
    meta.update(clusters=k)
    return Problem(name, seed, xs, ys, xf, yf, sigma=median_pairwise_distance(xs, ys) / 3.0, lam1=1.0 / l_,
                   lam2=1.0 / np.sqrt(n_), tol=1e-6, meta=meta)


def make_problem(name: str, s: int = 0, *, l: int | None = None, n: int | None = None) -> Problem:
    """Draw problem number ``s`` of workload ``name``.  ``l``/``n`` override the sizes (for scaled-down tests);
    the draw order is fixed so that an override changes only the affected arrays' lengths."""
    if name not in _SEED_BASE:
        raise ValueError(f"unknown workload {name!r}; expected one of {WORKLOADS}")
    seed = _SEED_BASE[name] + s
    rng = np.random.default_rng(seed)
    meta: dict = {}
    if name.startswith("sweep_d"):
        l_ = l or 500
        return _sweep(rng, name, seed, int(name[len("sweep_d"):]), l_, n or l_, meta)
    if name == "cells48":
        return _cells48(rng, name, seed, l or 256, n or 1000, meta)
    if name == "tiny":
        n_ = n or 100
        l_ = l or 50
        d = 2
        xs = rng.standard_normal((n_, d))
        ys = np.array([1.0, 1.0]) + rng.standard_normal((n_, d))
        xf = _box_uniform(rng, xs, l_)
        yf = _box_uniform(rng, ys, l_)
        return Problem(name, seed, xs, ys, xf, yf, sigma=1.0, lam1=1e-3, lam2=1e-3, tol=1e-8, meta=meta)
    if name == "gauss500":
        n_ = n or 2000
        l_ = l or 500
        d = 5
        m = rng.uniform(-1.0, 1.0, size=d)
        A = rng.standard_normal((d, d))
        cov = A @ A.T / 5.0 + 0.1 * np.eye(d)
        L = np.linalg.cholesky(cov)
        xs = rng.standard_normal((n_, d))
        ys = m + rng.standard_normal((n_, d)) @ L.T
    elif name in ("mix1000", "mix1000_median"):
        n_ = n or 5000
        l_ = l or 1000
        d = 10
        mx = rng.uniform(-2.0, 2.0, size=(4, d))
        my = rng.uniform(-2.0, 2.0, size=(4, d))
        xs = _mixture(rng, mx, n_)
        ys = _mixture(rng, my, n_)
    elif name == "mix256":
        n_ = n or 1000
        l_ = l or 256
        d = 8
        mx = rng.uniform(-2.0, 2.0, size=(3, d))
        my = rng.uniform(-2.0, 2.0, size=(3, d))
        xs = _mixture(rng, mx, n_)
        ys = _mixture(rng, my, n_)
    else:  # batch
        n_draw = int(rng.integers(200, 2001))
        l_draw = int(rng.integers(100, 401))
        n_ = n or n_draw
        l_ = l or l_draw
        d = int(rng.integers(2, 11))
        shift = rng.uniform(-1.0, 1.0, size=d)
        xs = rng.standard_normal((n_, d))
        ys = shift + rng.standard_normal((n_, d))
    if name in ("gauss500", "mix1000_median"):
        xf = _box_uniform(rng, xs, l_)
        yf = _box_uniform(rng, ys, l_)
        sigma = median_pairwise_distance(xs, ys)
    else:
        xs, ys = _unit_cube(xs, ys)
        xf = _box_uniform(rng, xs, l_)
        yf = _box_uniform(rng, ys, l_)
        sigma = PAPER_SIGMA
    lam1 = 1.0 / l_
    lam2 = 1.0 / np.sqrt(n_)
    return Problem(name, seed, xs, ys, xf, yf, sigma=sigma, lam1=lam1, lam2=lam2, tol=1e-6, meta=meta)


def make_custom(seed: int, n: int, d: int, l: int, *, sigma: float = 1.0, lam1: float = 1e-3,
                lam2: float = 1e-3, shift: float = 1.0, tol: float = 1e-8) -> Problem:
    """Small free-form problem for edge-case tests: N(0,I) vs N(shift*1, I)."""
    rng = np.random.default_rng(seed)
    xs = rng.standard_normal((n, d))
    ys = shift + rng.standard_normal((n, d))
    xf = _box_uniform(rng, xs, l)
    yf = _box_uniform(rng, ys, l)
    return Problem("custom", seed, xs, ys, xf, yf, sigma=sigma, lam1=lam1, lam2=lam2, tol=tol)
