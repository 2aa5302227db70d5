"""The diagonal-factor path (the sparsity of K, Remark 4.5): when every off-diagonal entry of K + eps I is at
most kdiag_tol times its largest diagonal entry, the setup takes R = diag(sqrt(K_ii + eps)) and the products
with R become diagonal scalings.  Checked against the oracle running Algorithm 2 on the same dropped data, and
against the factorized path where the dropped entries are below rounding's reach."""
import numpy as np
import pytest

from oracle import kot_oracle as ko
from paper_2310_14087_amd.inputs import make_problem

pytestmark = pytest.mark.gpu


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")


def _n(t):
    return t.detach().cpu().numpy()


def _dropped_core(p, eps=1e-10):
    """The oracle's dual data with the off-diagonal entries of K + eps I dropped: R = diag(sqrt(K_ii + eps))."""
    core = ko.setup(p.xs, p.ys, p.xf, p.yf, p.sigma, p.lam1, p.lam2, eps=eps)
    K = core.extra["K"] + eps * np.eye(p.l)
    return core, ko.core_from_arrays(core.Q, core.z, np.diag(np.sqrt(np.diag(K))), p.lam1, p.lam2, core.q2,
                                     core.wsum)


@pytest.mark.parametrize("iters", [3, 5])
def test_forced_diagonal_factor_matches_oracle_on_dropped_data(gpu_ctx, iters):
    """kdiag_tol = 1 takes the path on the dense 'tiny' kernel (every Gaussian entry is at most the diagonal):
    the trajectory is the oracle's Algorithm 2 on R = diag(sqrt(K_ii + eps)), with converged inner solves.
    (From the sixth iteration on, each Schur system of these dropped data takes 175-210 CG iterations to reach
    the 1e-13 stop, and the trial of iteration 5 is accepted on one side and rejected on the other, so the
    comparison stops at five.)"""
    from paper_2310_14087_amd import kotssn
    p = make_problem("tiny", 0)
    print(f"[case] kot_solve tiny forced diagonal factor, {iters} iterations", flush=True)
    _, core_d = _dropped_core(p)
    ref = ko.solve(core_d, ko.Params(tol=p.tol, max_iter=iters, cg_max_iter=400, tau=1e-13, kappa=1e-13))
    prm = kotssn.default_params(sigma=p.sigma, lambda1=p.lam1, lambda2=p.lam2, tol=p.tol, max_iter=iters,
                                cg_max_iter=400, tau=1e-13, kappa=1e-13, kdiag_tol=1.0)
    gamma, X, r = gpu_ctx.solve(_t(p.xs), _t(p.ys), _t(p.xf), _t(p.yf), prm, want_X=True)
    assert r.kdiag == 1
    hist = np.array([h["res"] for h in ref["history"]])
    assert r.iters == ref["iters"]
    np.testing.assert_allclose(r.res_hist, hist, rtol=1e-6)
    np.testing.assert_allclose(_n(gamma), ref["gamma"], atol=1e-6 * np.abs(ref["gamma"]).max())
    np.testing.assert_allclose(_n(X), ref["X"], atol=1e-6 * max(1e-30, np.abs(ref["X"]).max()))
    assert abs(r.ot - ref["ot"]) <= 1e-6 * abs(ref["ot"])


def test_forced_diagonal_factor_with_lifted_start(gpu_ctx):
    """The lifted start X0 = R^-T diag(y) R^-1 is diag(y / r^2) on the diagonal path: the first residuals
    match the oracle's from the same closed-form start on the dropped data."""
    from paper_2310_14087_amd import kotssn
    p = make_problem("mix256", 2, l=60, n=200)
    print("[case] kot_solve mix256 l=60 forced diagonal factor, closed-form start", flush=True)
    core, core_d = _dropped_core(p)
    g0 = np.maximum(core.z / np.diag(core.Q), -p.lam1)
    y = (core.Q @ g0 - core.z) / (2 * p.lam2)
    act = (g0 <= -0.9 * p.lam1) & (y > 0)
    yy = np.where(act, y, 0.0)
    if act.any():
        yy[yy < 0.02 * yy[act].mean()] = 0.0
    r = np.diag(core_d.R)
    X0 = np.diag(yy / r ** 2)
    _, _, rn_lift, _ = ko.residual(core_d, g0, X0)
    rn_cold = np.linalg.norm(core.z) / (2 * p.lam2)
    gs, Xs = (g0, X0) if rn_lift <= rn_cold else (np.zeros(p.l), np.zeros((p.l, p.l)))
    ref = ko.solve(core_d, ko.Params(tol=p.tol, max_iter=3), gamma0=gs, X0=Xs)
    prm = kotssn.default_params(sigma=p.sigma, lambda1=p.lam1, lambda2=p.lam2, tol=p.tol, max_iter=3,
                                closed_start=1, kdiag_tol=1.0)
    gamma, _, res = gpu_ctx.solve(_t(p.xs), _t(p.ys), _t(p.xf), _t(p.yf), prm)
    assert res.kdiag == 1 and res.warm_used == (1 if rn_lift <= rn_cold else 0)
    hist = np.array([h["res"] for h in ref["history"]])
    np.testing.assert_allclose(res.res_hist[:2], hist[:2], rtol=1e-8)


@pytest.mark.parametrize("name,l,n,seed", [("mix1000", 150, 600, 0), ("mix256", 64, 300, 1)])
@pytest.mark.parametrize("start", ["cold", "closed"])
def test_detected_on_decoupled_workloads(gpu_ctx, name, l, n, seed, start):
    """At sigma^2 = 0.005 on the unit cube K is the identity to about 1e-14: the default kdiag_tol (1e-12)
    takes the diagonal path, and the solve agrees with the factorized one (kdiag_tol = 0) and the oracle."""
    from paper_2310_14087_amd import kotssn
    p = make_problem(name, seed, l=l, n=n)
    print(f"[case] kot_solve {name} l={l} diagonal path vs factorized, {start} start", flush=True)
    core = ko.setup(p.xs, p.ys, p.xf, p.yf, p.sigma, p.lam1, p.lam2)
    off = np.abs(core.extra["K"] - np.diag(np.diag(core.extra["K"]))).max()
    assert off <= 1e-12
    kw = dict(sigma=p.sigma, lambda1=p.lam1, lambda2=p.lam2, tol=p.tol, closed_start=1 if start == "closed" else 0)
    gd, _, rd = gpu_ctx.solve(_t(p.xs), _t(p.ys), _t(p.xf), _t(p.yf), kotssn.default_params(**kw))
    gf, _, rf = gpu_ctx.solve(_t(p.xs), _t(p.ys), _t(p.xf), _t(p.yf), kotssn.default_params(kdiag_tol=0.0, **kw))
    assert rd.kdiag == 1 and rf.kdiag == 0
    assert rd.status == kotssn.KOT_OK and rf.status == kotssn.KOT_OK
    assert rd.residual <= p.tol and rf.residual <= p.tol
    assert abs(rd.ot - rf.ot) <= 1e-9 * abs(rf.ot)
    np.testing.assert_allclose(_n(gd), _n(gf), atol=1e-8 * np.abs(_n(gf)).max())
    ref = ko.solve(core, ko.Params(tol=p.tol))
    assert abs(rd.ot - ref["ot"]) <= 1e-6 * abs(ref["ot"])


@pytest.mark.parametrize("name,l,n", [("tiny", 50, 100), ("gauss500", 60, 240), ("mix1000_median", 80, 400)])
def test_not_taken_on_coupled_workloads(gpu_ctx, name, l, n):
    from paper_2310_14087_amd import kotssn
    p = make_problem(name, 0, l=l, n=n) if name != "tiny" else make_problem(name, 0)
    print(f"[case] kot_solve {name} l={p.l}: dense kernel, factorized path", flush=True)
    prm = kotssn.default_params(sigma=p.sigma, lambda1=p.lam1, lambda2=p.lam2, tol=p.tol, max_iter=1)
    _, _, r = gpu_ctx.solve(_t(p.xs), _t(p.ys), _t(p.xf), _t(p.yf), prm)
    assert r.kdiag == 0


def test_setup_returns_the_diagonal_factor(gpu_ctx):
    from paper_2310_14087_amd import kotssn
    p = make_problem("mix1000", 0, l=150, n=600)
    print("[case] kot_setup mix1000 l=150 diagonal factor", flush=True)
    core = ko.setup(p.xs, p.ys, p.xf, p.yf, p.sigma, p.lam1, p.lam2)
    prm = kotssn.default_params(sigma=p.sigma, lambda1=p.lam1, lambda2=p.lam2)
    Q, z, R, wsum, q2 = gpu_ctx.setup(_t(p.xs), _t(p.ys), _t(p.xf), _t(p.yf), prm)
    Rg = _n(R)
    assert np.all(Rg == np.diag(np.diag(Rg)))
    np.testing.assert_allclose(np.diag(Rg) ** 2, np.diag(core.extra["K"]) + 1e-10, rtol=1e-15)
    np.testing.assert_allclose(Rg, core.R, atol=1e-12)


def test_closed_form_fallback_on_diagonal_path(gpu_ctx):
    """closed_start = 2 on the diagonal path: a rejected given start is replaced by the closed-form start, whose
    lift is the diagonal diag(y / r^2); the solve is the closed_start = 1 solve bit for bit."""
    from paper_2310_14087_amd import kotssn
    p = make_problem("mix1000", 2, l=150, n=600)
    print("[case] kot_solve mix1000 l=150 diagonal path, rejected start replaced by the closed-form start", flush=True)
    args = (_t(p.xs), _t(p.ys), _t(p.xf), _t(p.yf))
    base = dict(sigma=p.sigma, lambda1=p.lam1, lambda2=p.lam2, tol=p.tol)
    bad = _t(np.full(p.l, 100.0 * p.lam1))
    gf, Xf, rf = gpu_ctx.solve(*args, kotssn.default_params(closed_start=2, **base), gamma0=bad, want_X=True)
    gc, Xc, rc = gpu_ctx.solve(*args, kotssn.default_params(closed_start=1, **base), want_X=True)
    assert rf.kdiag == 1 and rc.kdiag == 1
    assert rf.warm_used == 2 and rc.warm_used == 1
    assert rf.status == kotssn.KOT_OK and (rf.iters, rf.ot) == (rc.iters, rc.ot)
    assert np.array_equal(_n(gf), _n(gc)) and np.array_equal(_n(Xf), _n(Xc))
