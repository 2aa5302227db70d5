"""Pins of the oracle's Jacobi-preconditioned CG for the Schur system of Algorithm 1 (no GPU).

Section 4.3 solves the Schur system by CG or symmetric QMR; the diagonal preconditioner is an addition.  The
oracle's diagonal is written as a closed form (schur_diag) and is pinned here against the operator itself, probed
with unit vectors.
"""
import numpy as np
import pytest

from oracle import kot_oracle as ko
from paper_2310_14087_amd.inputs import make_custom, make_problem


def _state(seed, l=14, n=40):
    p = make_custom(seed, n=n, d=3, l=l, sigma=0.7, lam1=0.02, lam2=0.05)
    core = ko.setup(p.xs, p.ys, p.xf, p.yf, p.sigma, p.lam1, p.lam2)
    rng = np.random.default_rng(seed + 100)
    g = 0.05 * rng.standard_normal(l)
    B = rng.standard_normal((l, l))
    X = (B @ B.T) / l
    return core, g, X


@pytest.mark.parametrize("seed,mu", [(1, 0.3), (2, 0.01), (3, 2.0)])
def test_schur_diag_matches_unit_probes(seed, mu):
    """M_ii = e_i^T M e_i with M applied by the plain dense schur_matvec (T in its P (Psi o P^T S P) P^T form)."""
    core, g, X = _state(seed)
    _, _, _, (s, P) = ko.residual(core, g, X)
    assert 0 < int(np.sum(s > 0)) < core.l  # both eigen-sets present: every block of Psi contributes
    Psi = ko.psi_matrix(s, mu)
    d = ko.schur_diag(core, P, Psi, mu)
    brute = np.array([ko.schur_matvec(core, P, Psi, mu, e)[i] for i, e in enumerate(np.eye(core.l))])
    np.testing.assert_allclose(d, brute, rtol=1e-12, atol=1e-12 * np.abs(brute).max())


def test_pcg_unit_preconditioner_is_cg():
    """With D = I the preconditioned recurrences reduce to plain CG: same iterate, count and residual."""
    rng = np.random.default_rng(7)
    A = rng.standard_normal((30, 30))
    A = A @ A.T + 3 * np.eye(30)
    b = rng.standard_normal(30)
    stop = lambda res, x: res <= 1e-9
    x1, it1, r1 = ko.cg(lambda v: A @ v, b, stop, 50)
    x2, it2, r2 = ko.pcg(lambda v: A @ v, b, np.ones(30), stop, 50)
    assert it1 == it2
    np.testing.assert_allclose(x2, x1, rtol=1e-13, atol=1e-15)
    assert abs(r1 - r2) <= 1e-12 * max(r1, 1e-300) + 1e-300


def test_pcg_solves_badly_scaled_system():
    """A badly row/column-scaled SPD system: PCG with its diagonal reaches the exact solution (np.linalg.solve)
    in far fewer iterations than CG, whose count is capped."""
    rng = np.random.default_rng(11)
    n = 60
    C = rng.standard_normal((n, n))
    C = C @ C.T / n + np.eye(n)
    s = 10.0 ** rng.uniform(-3, 3, n)
    A = (s[:, None] * C) * s[None, :]
    b = rng.standard_normal(n)
    x_ref = np.linalg.solve(A, b)
    stop = lambda res, x: res <= 1e-10 * np.linalg.norm(b)
    xp, itp, _ = ko.pcg(lambda v: A @ v, b, 1.0 / np.diag(A), stop, 500)
    _, itc, _ = ko.cg(lambda v: A @ v, b, stop, 500)
    np.testing.assert_allclose(xp, x_ref, rtol=1e-6, atol=1e-8 * np.abs(x_ref).max())
    assert itp < 60 and itp * 4 < itc


def test_solve_with_jacobi_reaches_the_same_minimizer():
    """Eq. (3.4) has a unique minimizer: the preconditioned solver reaches the same gamma and OT estimate."""
    p = make_problem("mix256", 1, l=64, n=300)
    core = ko.setup(p.xs, p.ys, p.xf, p.yf, p.sigma, p.lam1, p.lam2)
    a = ko.solve(core, ko.Params(tol=1e-9))
    b = ko.solve(core, ko.Params(tol=1e-9, precond="jacobi"))
    assert a["status"] == "converged" and b["status"] == "converged"
    np.testing.assert_allclose(b["gamma"], a["gamma"], atol=1e-6 * np.abs(a["gamma"]).max())
    assert abs(b["ot"] - a["ot"]) <= 1e-7 * abs(a["ot"])


@pytest.mark.parametrize("scaled", [False, True])
def test_sqmr_true_residual_and_solution(scaled):
    """Symmetric QMR: the carried residual s_k equals b - A x_k at every step, and the iterate reaches
    np.linalg.solve (plain, and with the diagonal preconditioner on a badly scaled system)."""
    rng = np.random.default_rng(5)
    n = 40
    C = rng.standard_normal((n, n))
    A = C @ C.T / n + 0.2 * np.eye(n)
    if scaled:
        sc = 10.0 ** rng.uniform(-2, 2, n)
        A = (sc[:, None] * A) * sc[None, :]
    b = rng.standard_normal(n)
    dinv = 1.0 / np.diag(A) if scaled else None
    seen = []

    def stop(res, x):
        seen.append((res, x.copy()))
        return res <= 1e-11 * np.linalg.norm(b)

    x, it, res = ko.sqmr(lambda v: A @ v, b, dinv, stop, 400)
    for rk, xk in seen:
        assert abs(rk - np.linalg.norm(b - A @ xk)) <= 1e-8 * np.linalg.norm(b)
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=0, atol=1e-8 * np.abs(np.linalg.solve(A, b)).max())


def test_sqmr_one_step_is_the_minimal_residual_point():
    """After one step the QMR iterate minimizes |b - A x| over x in span{b} (exact arithmetic identity)."""
    rng = np.random.default_rng(9)
    A = rng.standard_normal((12, 12))
    A = A @ A.T + np.eye(12)
    b = rng.standard_normal(12)
    x, it, _ = ko.sqmr(lambda v: A @ v, b, None, lambda r_, x_: False, 1)
    Ab = A @ b
    t = float(b @ Ab) / float(Ab @ Ab)
    assert it == 1
    np.testing.assert_allclose(x, t * b, rtol=1e-12, atol=1e-14)


def test_solve_with_sqmr_reaches_the_same_minimizer():
    p = make_problem("mix256", 1, l=64, n=300)
    core = ko.setup(p.xs, p.ys, p.xf, p.yf, p.sigma, p.lam1, p.lam2)
    a = ko.solve(core, ko.Params(tol=1e-9))
    b = ko.solve(core, ko.Params(tol=1e-9, schur_solver="sqmr", precond="jacobi"))
    assert a["status"] == "converged" and b["status"] == "converged"
    np.testing.assert_allclose(b["gamma"], a["gamma"], atol=1e-6 * np.abs(a["gamma"]).max())
    assert abs(b["ot"] - a["ot"]) <= 1e-7 * abs(a["ot"])
