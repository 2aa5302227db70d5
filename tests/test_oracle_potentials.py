"""Pins of the potentials / transport-map oracle (CPU).  Each ties it to something other than itself:
the estimator of Section 3 through the reproducing property, the dual data (Q, z) through the constraint of
Eq. (3.2), finite differences, and a one-sample closed form."""
import numpy as np
import pytest

from oracle import kot_oracle as ko
from oracle import potentials as po
from paper_2310_14087_amd.inputs import make_custom, make_problem


def _solved(name="mix256", l=60, n=150, seed=2):
    p = make_problem(name, seed, l=l, n=n)
    core = ko.setup(p.xs, p.ys, p.xf, p.yf, p.sigma, p.lam1, p.lam2)
    res = ko.solve(core, ko.Params(tol=1e-9))
    return p, core, res


def test_potentials_reproduce_the_estimator():
    """<u^, w_mu_hat> = mean of u^ over the source samples; the sum with v^ is the solver's OT estimate."""
    p, core, res = _solved()
    g = res["gamma"]
    u = po.potential(p.xs, p.xs, p.xf, g, p.sigma, p.lam2)
    v = po.potential(p.ys, p.ys, p.yf, g, p.sigma, p.lam2)
    assert abs(u.mean() + v.mean() - res["ot"]) <= 1e-10 * max(1.0, abs(res["ot"]))


@pytest.mark.parametrize("seed", [0, 3])
def test_constraint_identity(seed):
    """c_i/2 - u^(x~_i) - v^(y~_i) = ((Q gamma - z)/(2 lambda2))_i for any gamma (the value Phi(X) takes at a
    stationary point), and it is >= 0 up to the tolerance at the solution (X PSD)."""
    p = make_custom(seed, 40, 3, 25, sigma=0.8, lam1=1e-2, lam2=1e-2)
    core = ko.setup(p.xs, p.ys, p.xf, p.yf, p.sigma, p.lam1, p.lam2)
    g = np.random.default_rng(seed).standard_normal(p.l) * 1e-2
    c = ((p.xf - p.yf) ** 2).sum(axis=1)
    lhs = 0.5 * c - po.potential(p.xf, p.xs, p.xf, g, p.sigma, p.lam2) - po.potential(p.yf, p.ys, p.yf, g, p.sigma, p.lam2)
    rhs = (core.Q @ g - core.z) / (2 * p.lam2)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-10, atol=1e-10 * np.abs(rhs).max())


def test_constraint_nonnegative_at_solution():
    p, core, res = _solved()
    g = res["gamma"]
    c = ((p.xf - p.yf) ** 2).sum(axis=1)
    slack = 0.5 * c - po.potential(p.xf, p.xs, p.xf, g, p.sigma, p.lam2) - po.potential(p.yf, p.ys, p.yf, g, p.sigma, p.lam2)
    assert slack.min() >= -10 * res["residual"] * max(1.0, np.abs(slack).max())


def test_gradient_finite_differences():
    p, core, res = _solved(l=40, n=80)
    g = res["gamma"]
    rng = np.random.default_rng(7)
    q = p.xs[:5] + 0.01 * rng.standard_normal((5, p.d))
    grad = po.potential_grad(q, p.xs, p.xf, g, p.sigma, p.lam2)
    h = 1e-6
    for k in range(p.d):
        e = np.zeros(p.d)
        e[k] = h
        fd = (po.potential(q + e, p.xs, p.xf, g, p.sigma, p.lam2) - po.potential(q - e, p.xs, p.xf, g, p.sigma, p.lam2)) / (2 * h)
        np.testing.assert_allclose(grad[:, k], fd, rtol=1e-6, atol=1e-7 * np.abs(grad).max())


def test_one_sample_closed_form():
    """One sample, one filling point, gamma = 0: u^(x) = exp(-|x - x1|^2/(2 s^2)) / (2 lam2) and
    T(x) = x - k (x1 - x) / (s^2 2 lam2)."""
    x1 = np.array([[0.3, -0.2]])
    xf = np.array([[5.0, 5.0]])
    q = np.array([[0.0, 0.1], [1.0, -1.0]])
    s, lam2 = 0.7, 0.25
    k = np.exp(-((q - x1) ** 2).sum(axis=1) / (2 * s * s))
    np.testing.assert_allclose(po.potential(q, x1, xf, np.zeros(1), s, lam2), k / (2 * lam2), rtol=1e-14)
    np.testing.assert_allclose(po.transport_map(q, x1, xf, np.zeros(1), s, lam2),
                               q - k[:, None] * (x1 - q) / (s * s) / (2 * lam2), rtol=1e-14)
