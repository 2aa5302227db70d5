"""GPU checks of the warm-start network kernels against the CPU oracle, and of the learned start itself."""
import os

import numpy as np
import pytest

from oracle import kot_oracle as ko
from oracle import mlp
from paper_2310_14087_amd.inputs import make_problem

pytestmark = pytest.mark.gpu


def _t(a, dt=None):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dt or np.float64)).to("cuda:0")


def _n(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("n,F,H", [(300, 12, 32), (1000, 12, 512), (70, 5, 64)])
def test_mlp_forward_and_grad(gpu_ctx, n, F, H):
    print(f"[case] kot_mlp_forward / kot_mlp_loss_grad n={n} F={F} H={H}", flush=True)
    rng = np.random.default_rng(n + H)
    theta = (rng.standard_normal(mlp.n_params(F, H)) * 0.3).astype(np.float32)
    X = rng.standard_normal((n, F)).astype(np.float32)
    y = rng.standard_normal(n).astype(np.float32)
    out = _n(gpu_ctx.mlp_forward(_t(X, np.float32), _t(theta, np.float32), H))
    ref, _ = mlp.forward(theta.astype(np.float64), X.astype(np.float64), F, H)
    np.testing.assert_allclose(out, ref, rtol=1e-4, atol=1e-4 * np.abs(ref).max())
    loss, g = gpu_ctx.mlp_loss_grad(_t(X, np.float32), _t(y, np.float32), _t(theta, np.float32), H)
    rl, rg = mlp.loss_and_grad(theta.astype(np.float64), X.astype(np.float64), y.astype(np.float64), F, H)
    assert loss == pytest.approx(rl, rel=1e-4)
    g = _n(g)
    np.testing.assert_allclose(g, rg, atol=2e-4 * np.abs(rg).max())


def test_mlp_adam(gpu_ctx):
    print("[case] kot_mlp_adam", flush=True)
    rng = np.random.default_rng(3)
    P = 1000
    th = rng.standard_normal(P).astype(np.float32)
    g = rng.standard_normal(P).astype(np.float32)
    m = (rng.standard_normal(P) * 0.1).astype(np.float32)
    v = np.abs(rng.standard_normal(P) * 0.1).astype(np.float32)
    tt, tm, tv = _t(th, np.float32), _t(m, np.float32), _t(v, np.float32)
    gpu_ctx.mlp_adam(tt, _t(g, np.float32), tm, tv, 7, lr=1e-2)
    rth, rm, rv = mlp.adam_step(th.astype(np.float64), g.astype(np.float64), m.astype(np.float64),
                                v.astype(np.float64), 7, lr=1e-2)
    np.testing.assert_allclose(_n(tt), rth, rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(_n(tm), rm, rtol=1e-5, atol=1e-7)


def test_features(gpu_ctx):
    from paper_2310_14087_amd import kotssn
    p = make_problem("mix256", 0, l=80, n=200)
    print(f"[case] kot_features mix256 l={p.l}", flush=True)
    core = ko.setup(p.xs, p.ys, p.xf, p.yf, p.sigma, p.lam1, p.lam2)
    prm = kotssn.default_params(lambda1=p.lam1, lambda2=p.lam2)
    X = _n(gpu_ctx.features(_t(core.Q), _t(core.z), _t(core.R), _t(core.wsum), core.q2, prm))
    K = core.R.T @ core.R
    qd, kd = np.diag(core.Q), np.diag(K)
    f0 = core.z / (p.lam1 * qd)
    az = np.abs(core.z)
    ref = np.column_stack([np.maximum(f0, -2), np.maximum(f0, -1), core.Q.sum(1) / qd - 1, K.sum(1) / kd - 1,
                           (K * K).sum(1) / kd ** 2 - 1, qd - 2, kd - 1,
                           np.where(az > 0, np.minimum(core.wsum / np.where(az > 0, az, 1), 10), 10),
                           np.full(p.l, np.mean(f0 < -1)), np.full(p.l, np.maximum(f0, -1).mean()),
                           np.zeros(p.l), np.ones(p.l)])
    np.testing.assert_allclose(X, ref, rtol=1e-5, atol=1e-6)


@pytest.mark.parametrize("name,l,n,seed", [("mix256", 96, 300, 7), ("mix1000", 120, 400, 5)])
def test_lift_from_exact_dual(gpu_ctx, name, l, n, seed):
    """Starting from the oracle's dual with the lifted multiplier, Algorithm 2 is (almost) done at once."""
    from paper_2310_14087_amd import kotssn
    p = make_problem(name, seed, l=l, n=n)
    print(f"[case] kot_solve from exact gamma {name} l={p.l}", flush=True)
    core = ko.setup(p.xs, p.ys, p.xf, p.yf, p.sigma, p.lam1, p.lam2)
    ref = ko.solve(core, ko.Params(tol=1e-9))
    prm = kotssn.default_params(sigma=p.sigma, lambda1=p.lam1, lambda2=p.lam2, tol=p.tol)
    g, _, r = gpu_ctx.solve(_t(p.xs), _t(p.ys), _t(p.xf), _t(p.yf), prm, gamma0=_t(ref["gamma"]))
    assert r.status == kotssn.KOT_OK and r.warm_used == 1
    assert r.iters <= 2
    assert abs(r.ot - ref["ot"]) <= 1e-6 * abs(ref["ot"])


WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2310_14087_amd",
                       "weights", "warmstart_mix256.npz")


@pytest.mark.skipif(not os.path.exists(WEIGHTS), reason="trained weights not present")
def test_learned_warm_start_gain(gpu_ctx):
    """Held-out problems (seeds never used in training): the learned start needs fewer iterations than the
    cold start and reaches the same estimate."""
    import torch
    from paper_2310_14087_amd import kotssn, warmstart
    theta, F, H, meta = warmstart.load(WEIGHTS)
    th = torch.from_numpy(theta).to("cuda:0")
    cold_it, warm_it = [], []
    for s in range(100000, 100016):
        p = make_problem("mix256", s)
        print(f"[case] warm vs cold mix256 seed={s}", flush=True)
        args = (_t(p.xs), _t(p.ys), _t(p.xf), _t(p.yf))
        prm = kotssn.default_params(sigma=p.sigma, lambda1=p.lam1, lambda2=p.lam2, tol=p.tol)
        _, _, rc = gpu_ctx.solve(*args, prm)
        prw = kotssn.default_params(sigma=p.sigma, lambda1=p.lam1, lambda2=p.lam2, tol=p.tol, ws_F=F, ws_H=H,
                                    ws_theta=th.data_ptr(), closed_start=0)
        _, _, rw = gpu_ctx.solve(*args, prw)
        assert rc.status == kotssn.KOT_OK and rw.status == kotssn.KOT_OK
        assert abs(rw.ot - rc.ot) <= 1e-6 * abs(rc.ot)
        cold_it.append(rc.iters)
        warm_it.append(rw.iters)
    print(f"cold iterations {np.mean(cold_it):.2f}, warm {np.mean(warm_it):.2f}")
    assert np.mean(warm_it) < 0.7 * np.mean(cold_it)


@pytest.mark.skipif(not os.path.exists(WEIGHTS), reason="trained weights not present")
def test_learned_start_against_closed_form_start_256(gpu_ctx):
    """256 held-out problems (seeds never used in training): outer iterations from the cold start, from the
    closed-form start gamma0_i = max(z_i/Q_ii, -lambda1) (the network's first feature times lambda1, same lift,
    no network) and from the network's start; every run reaches the same estimate.  The learned start needs
    fewer iterations than the cold start; what the network adds over the closed-form start is printed (and
    recorded in the design notes)."""
    import torch
    from paper_2310_14087_amd import kotssn, warmstart
    theta, F, H, meta = warmstart.load(WEIGHTS)
    th = torch.from_numpy(theta).to("cuda:0")
    its = {"cold": [], "closed": [], "learned": []}
    used = {"closed": 0, "learned": 0}
    print("[case] cold / closed-form / learned starts on 256 held-out mix256 problems", flush=True)
    for s in range(100000, 100256):
        p = make_problem("mix256", s)
        args = (_t(p.xs), _t(p.ys), _t(p.xf), _t(p.yf))
        base = dict(sigma=p.sigma, lambda1=p.lam1, lambda2=p.lam2, tol=p.tol)
        _, _, rc = gpu_ctx.solve(*args, kotssn.default_params(**base))
        _, _, rz = gpu_ctx.solve(*args, kotssn.default_params(closed_start=1, **base))
        _, _, rw = gpu_ctx.solve(*args, kotssn.default_params(ws_F=F, ws_H=H, ws_theta=th.data_ptr(), closed_start=0,
                                                              **base))
        for r in (rc, rz, rw):
            assert r.status == kotssn.KOT_OK, (s, r)
            assert abs(r.ot - rc.ot) <= 1e-6 * abs(rc.ot)
        its["cold"].append(rc.iters)
        its["closed"].append(rz.iters)
        its["learned"].append(rw.iters)
        used["closed"] += rz.warm_used
        used["learned"] += rw.warm_used
    m = {k: float(np.mean(v)) for k, v in its.items()}
    print(f"mean outer iterations over 256 held-out problems: cold {m['cold']:.3f}, closed-form start "
          f"{m['closed']:.3f} (kept {used['closed']}/256), learned start {m['learned']:.3f} (kept "
          f"{used['learned']}/256); learned better than closed-form on "
          f"{sum(a < b for a, b in zip(its['learned'], its['closed']))}, worse on "
          f"{sum(a > b for a, b in zip(its['learned'], its['closed']))}")
    assert m["learned"] < 0.7 * m["cold"]


@pytest.mark.parametrize("name,l,n,seed", [("mix256", 70, 200, 11), ("tiny", None, None, 0), ("mix256", 200, 300, 5)])
def test_lifted_start_matrix(gpu_ctx, name, l, n, seed):
    """max_iter = 0 returns the start point: X0 = R^-T diag(y) R^-1 with the lift's rule, checked with numpy
    (dense factor at 'tiny': exercises the blocked triangular inverse)."""
    from paper_2310_14087_amd import kotssn
    p = make_problem(name, seed, l=l, n=n)
    print(f"[case] lifted X0 {name} l={p.l}", flush=True)
    core = ko.setup(p.xs, p.ys, p.xf, p.yf, p.sigma, p.lam1, p.lam2)
    rng = np.random.default_rng(1)
    g0 = -p.lam1 * (1.0 + 0.3 * rng.standard_normal(p.l))
    prm = kotssn.default_params(sigma=p.sigma, lambda1=p.lam1, lambda2=p.lam2, tol=1e-300, max_iter=0,
                                closed_start=0)
    g, X, r = gpu_ctx.solve(_t(p.xs), _t(p.ys), _t(p.xf), _t(p.yf), prm, gamma0=_t(g0), want_X=True)
    y = (core.Q @ g0 - core.z) / (2 * p.lam2)
    y = np.where((g0 <= -0.9 * p.lam1) & (y > 0), y, 0.0)
    if np.any(y > 0):
        y = np.where(y < 0.02 * y[y > 0].mean(), 0.0, y)
    Ri = np.linalg.inv(core.R)
    X0 = Ri.T @ np.diag(y) @ Ri
    if r.warm_used:
        np.testing.assert_allclose(_n(X), X0, atol=1e-9 * max(1.0, np.abs(X0).max()))
        np.testing.assert_allclose(ko.phi(core.R, _n(X)), y, atol=1e-8 * max(1.0, y.max()))
    else:  # the start was worse than the cold start: (0, 0) is returned
        assert np.all(_n(X) == 0) and np.all(_n(g) == 0)


def _same_solve(a, b):
    """a reached b's start after rejecting another one: the same iterates, histories and counters, and at least
    b's sweeps (the rejected start's residual took its own)."""
    (ga, Xa, ra), (gb, Xb, rb) = a, b
    k = ra.iters + 1
    assert (ra.status, ra.iters, ra.cg_iters_total, ra.eg_accepts) == (rb.status, rb.iters, rb.cg_iters_total,
                                                                         rb.eg_accepts)
    assert ra.eig_sweeps_total >= rb.eig_sweeps_total
    np.testing.assert_array_equal(ra.res_hist[:k], rb.res_hist[:k])
    assert ra.ot == rb.ot
    assert np.array_equal(_n(ga), _n(gb)) and np.array_equal(_n(Xa), _n(Xb))


def test_rejected_start_replaced_by_closed_form_start(gpu_ctx):
    """A given start worse than the cold one (gamma0 = +10 lambda1 everywhere): with closed_start = 2 the
    closed-form start replaces it (warm_used = 2) and the solve is the closed_start = 1 solve bit for bit; with
    closed_start = 0 (the default) it is the cold solve bit for bit (warm_used = 0)."""
    from paper_2310_14087_amd import kotssn
    p = make_problem("mix256", 3, l=90, n=300)
    print(f"[case] rejected given start, closed-form fallback, mix256 l={p.l}", flush=True)
    args = (_t(p.xs), _t(p.ys), _t(p.xf), _t(p.yf))
    bad = _t(np.full(p.l, 10.0 * p.lam1))
    base = dict(sigma=p.sigma, lambda1=p.lam1, lambda2=p.lam2, tol=p.tol)
    fb = gpu_ctx.solve(*args, kotssn.default_params(closed_start=2, **base), gamma0=bad, want_X=True, hist_cap=256)
    cl = gpu_ctx.solve(*args, kotssn.default_params(closed_start=1, **base), want_X=True, hist_cap=256)
    assert cl[2].warm_used == 1 and fb[2].warm_used == 2
    assert fb[2].status == kotssn.KOT_OK
    _same_solve(fb, cl)
    nf = gpu_ctx.solve(*args, kotssn.default_params(closed_start=0, **base), gamma0=bad, want_X=True, hist_cap=256)
    cd = gpu_ctx.solve(*args, kotssn.default_params(closed_start=0, **base), want_X=True, hist_cap=256)
    assert nf[2].warm_used == 0
    _same_solve(nf, cd)
    # |r1| of this start alone exceeds the cold start's residual: it is dropped before its Z is decomposed
    assert fb[2].eig_sweeps_total == cl[2].eig_sweeps_total and nf[2].eig_sweeps_total == cd[2].eig_sweeps_total


@pytest.mark.skipif(not os.path.exists(WEIGHTS), reason="trained weights not present")
def test_learned_start_fallback_on_coupled_workload(gpu_ctx):
    """The median-bandwidth workload at full size (l = 1000, n = 5000), 2 outer iterations: the network's start
    fails the fallback test there (it was trained on decoupled problems); with closed_start = 2 the closed-form
    start replaces it (warm_used = 2), and the solve is then the closed_start = 1 solve bit for bit."""
    import torch
    from paper_2310_14087_amd import kotssn, warmstart
    theta, F, H, meta = warmstart.load(WEIGHTS)
    th = torch.from_numpy(theta).to("cuda:0")
    p = make_problem("mix1000_median", 0)
    print(f"[case] learned start with closed-form fallback, mix1000_median l={p.l}", flush=True)
    args = (_t(p.xs), _t(p.ys), _t(p.xf), _t(p.yf))
    base = dict(sigma=p.sigma, lambda1=p.lam1, lambda2=p.lam2, tol=p.tol, max_iter=2)
    lw = dict(ws_F=F, ws_H=H, ws_theta=th.data_ptr())
    only = gpu_ctx.solve(*args, kotssn.default_params(closed_start=0, **lw, **base))
    assert only[2].warm_used == 0
    fb = gpu_ctx.solve(*args, kotssn.default_params(closed_start=2, **lw, **base), want_X=True, hist_cap=16)
    cl = gpu_ctx.solve(*args, kotssn.default_params(closed_start=1, **base), want_X=True, hist_cap=16)
    assert cl[2].warm_used == 1 and fb[2].warm_used == 2
    _same_solve(fb, cl)
    assert fb[2].eig_sweeps_total == cl[2].eig_sweeps_total  # the network's start fails on |r1| alone


def test_closed_start_value_checked(gpu_ctx):
    import torch
    from paper_2310_14087_amd import kotssn
    print("[case] kot_solve rejects closed_start=3", flush=True)
    p = make_problem("mix256", 0, l=20, n=40)
    prm = kotssn.default_params(sigma=p.sigma, lambda1=p.lam1, lambda2=p.lam2, closed_start=3)
    with pytest.raises(kotssn.KotError) as e:
        gpu_ctx.solve(_t(p.xs), _t(p.ys), _t(p.xf), _t(p.yf), prm)
    assert e.value.status == kotssn.KOT_ERR_ARG


@pytest.mark.skipif(not os.path.exists(WEIGHTS), reason="trained weights not present")
def test_kot_warmstart_prediction(gpu_ctx):
    """kot_warmstart: gamma0 = lambda1 * f(features) with the trained network, against the network evaluated in
    FP64 on the CPU (oracle/mlp.py) on the library's features; kot_solve with the same network and max_iter = 0
    returns that start (kept on this held-out decoupled problem)."""
    import torch
    from paper_2310_14087_amd import kotssn, warmstart
    theta, F, H, meta = warmstart.load(WEIGHTS)
    th = torch.from_numpy(theta).to("cuda:0")
    p = make_problem("mix256", 100003)
    print(f"[case] kot_warmstart mix256 seed=100003 l={p.l}", flush=True)
    args = (_t(p.xs), _t(p.ys), _t(p.xf), _t(p.yf))
    prm = kotssn.default_params(sigma=p.sigma, lambda1=p.lam1, lambda2=p.lam2, tol=1e-300, max_iter=0)
    g0 = _n(gpu_ctx.warmstart(*args, prm, th, H))
    core = ko.setup(p.xs, p.ys, p.xf, p.yf, p.sigma, p.lam1, p.lam2)
    X = _n(gpu_ctx.features(_t(core.Q), _t(core.z), _t(core.R), _t(core.wsum), core.q2, prm))
    ref, _ = mlp.forward(theta.astype(np.float64), X.astype(np.float64), F, H)
    np.testing.assert_allclose(g0, p.lam1 * ref, rtol=0, atol=1e-4 * p.lam1 * max(1.0, np.abs(ref).max()))
    prw = kotssn.default_params(sigma=p.sigma, lambda1=p.lam1, lambda2=p.lam2, tol=1e-300, max_iter=0, ws_F=F,
                                ws_H=H, ws_theta=th.data_ptr())
    g, _, r = gpu_ctx.solve(*args, prw)
    assert r.warm_used == 1
    np.testing.assert_allclose(_n(g), g0, rtol=1e-6, atol=1e-9 * p.lam1)
