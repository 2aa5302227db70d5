"""Inputs of Section 5's synthetic sweep (and the 48-feature stand-in) and the oracle on them (no GPU)."""
import numpy as np
import pytest

from oracle import kot_oracle as ko
from paper_2310_14087_amd.inputs import PAPER_SIGMA, make_problem, sobol_filling


def test_sobol_filling_is_a_stratified_net():
    """A scrambled Sobol set of 2^m points puts exactly one point in every interval [j/2^m, (j+1)/2^m) of every
    coordinate (each one-dimensional projection is a (0, m, 1)-net); i.i.d. uniform points almost never do."""
    xf, yf = sobol_filling(np.random.default_rng(3), 256, 5)
    pts = np.concatenate([xf, yf], axis=1)
    assert pts.shape == (256, 10) and pts.min() >= 0.0 and pts.max() < 1.0
    for k in range(10):
        assert len(np.unique(np.floor(pts[:, k] * 256).astype(int))) == 256
    u = np.random.default_rng(3).random(256)
    assert len(np.unique(np.floor(u * 256).astype(int))) < 256
    xf2, _ = sobol_filling(np.random.default_rng(3), 256, 5)
    assert np.array_equal(xf, xf2)


@pytest.mark.parametrize("d", [2, 5, 10])
def test_sweep_problem_settings(d):
    """Section 5: mixtures of 3 and 5 Gaussians, filling points from a 2d-dimensional Sobol sequence,
    sigma^2 = 0.005, lambda1 = 1/l, lambda2 = 1/sqrt(n), stop at |R| < 0.005."""
    p = make_problem(f"sweep_d{d}", 0, l=96, n=150)
    assert p.meta["components"] == (3, 5)
    assert p.xs.shape == (150, d) and p.ys.shape == (150, d) and p.xf.shape == (96, d) and p.yf.shape == (96, d)
    assert abs(p.sigma ** 2 - 0.005) < 1e-15 and p.sigma == PAPER_SIGMA
    assert p.lam1 == 1.0 / 96 and abs(p.lam2 - 1.0 / np.sqrt(150)) < 1e-15 and p.tol == 0.005
    both = np.concatenate([p.xs, p.ys])
    assert both.min() >= 0.0 and both.max() <= 1.0 + 1e-12


def test_cells48_shapes():
    p = make_problem("cells48", 0, l=64, n=120)
    assert p.d == 48 and p.l == 64 and p.n_src == 120 and p.sigma > 0.0


@pytest.mark.parametrize("name", ["sweep_d5", "sweep_d10"])
def test_oracle_reaches_the_sweep_tolerance(name):
    p = make_problem(name, 1, l=64, n=64)
    core = ko.setup(p.xs, p.ys, p.xf, p.yf, p.sigma, p.lam1, p.lam2)
    r = ko.solve(core, ko.Params(tol=p.tol))
    assert r["status"] == "converged" and r["residual"] < 0.005
    _, _, rn, _ = ko.residual(core, r["gamma"], r["X"])
    assert abs(rn - r["residual"]) <= 1e-12 * max(1.0, rn)
