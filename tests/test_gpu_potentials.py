"""Potentials and transport map through the C-ABI against the CPU oracle (Section 3, maximizers of Eq. 3.2)."""
import numpy as np
import pytest

from oracle import kot_oracle as ko
from oracle import potentials as po
from paper_2310_14087_amd.inputs import make_custom, make_problem

pytestmark = pytest.mark.gpu


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")


def _n(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("d,l,n,m", [(2, 30, 50, 1), (8, 70, 300, 257), (10, 40, 120, 600), (17, 33, 90, 100),
                                     (40, 20, 64, 31)])
def test_potentials_match_oracle(gpu_ctx, d, l, n, m):
    """Any gamma: u, v, T elementwise (ragged query counts, every padded dimension class)."""
    from paper_2310_14087_amd import kotssn
    p = make_custom(d * 100 + l, n, d, l, sigma=0.9 + 0.1 * d ** 0.5, lam1=1e-2, lam2=3e-2)
    print(f"[case] kot_potentials d={d} l={l} n={n} m={m}", flush=True)
    rng = np.random.default_rng(d + m)
    g = rng.standard_normal(l) * 1e-2
    xq = p.xs[rng.integers(0, n, size=m)] + 0.3 * rng.standard_normal((m, d))
    yq = p.ys[rng.integers(0, n, size=m)] + 0.3 * rng.standard_normal((m, d))
    prm = kotssn.default_params(sigma=p.sigma, lambda1=p.lam1, lambda2=p.lam2)
    u, v, T = gpu_ctx.potentials(_t(p.xs), _t(p.ys), _t(p.xf), _t(p.yf), prm, _t(g), _t(xq), _t(yq))
    ou = po.potential(xq, p.xs, p.xf, g, p.sigma, p.lam2)
    ov = po.potential(yq, p.ys, p.yf, g, p.sigma, p.lam2)
    oT = po.transport_map(xq, p.xs, p.xf, g, p.sigma, p.lam2)
    np.testing.assert_allclose(_n(u), ou, rtol=1e-12, atol=1e-13 * np.abs(ou).max())
    np.testing.assert_allclose(_n(v), ov, rtol=1e-12, atol=1e-13 * np.abs(ov).max())
    np.testing.assert_allclose(_n(T), oT, rtol=1e-12, atol=1e-12 * np.abs(oT - xq).max())


def test_potentials_of_a_solve_reproduce_the_estimate(gpu_ctx):
    """mean u(xs) + mean v(ys) = OT estimate of the same solve (reproducing property), and the constraint slack
    c_i/2 - u(xf_i) - v(yf_i) is nonnegative at the solution."""
    from paper_2310_14087_amd import kotssn
    p = make_problem("mix256", 7, l=96, n=400)
    print("[case] kot_solve + kot_potentials mix256 l=96", flush=True)
    args = (_t(p.xs), _t(p.ys), _t(p.xf), _t(p.yf))
    prm = kotssn.default_params(sigma=p.sigma, lambda1=p.lam1, lambda2=p.lam2, tol=1e-9)
    gamma, _, r = gpu_ctx.solve(*args, prm)
    assert r.status == kotssn.KOT_OK
    u, v, _ = gpu_ctx.potentials(*args, prm, gamma, xq=args[0], yq=args[1], want_map=False)
    est = _n(u).mean() + _n(v).mean()
    assert abs(est - r.ot) <= 1e-10 * max(1.0, abs(r.ot))
    uf, vf, _ = gpu_ctx.potentials(*args, prm, gamma, xq=args[2], yq=args[3], want_map=False)
    slack = 0.5 * ((p.xf - p.yf) ** 2).sum(axis=1) - _n(uf) - _n(vf)
    assert slack.min() >= -1e-6 * max(1.0, np.abs(slack).max())


def test_potentials_one_side_and_empty(gpu_ctx):
    from paper_2310_14087_amd import kotssn
    p = make_custom(5, 80, 3, 25)
    print("[case] kot_potentials one side / m=0", flush=True)
    g = np.random.default_rng(1).standard_normal(25) * 1e-3
    prm = kotssn.default_params(sigma=p.sigma, lambda1=p.lam1, lambda2=p.lam2)
    args = (_t(p.xs), _t(p.ys), _t(p.xf), _t(p.yf))
    u, v, T = gpu_ctx.potentials(*args, prm, _t(g), yq=_t(p.ys[:9]))
    assert u is None and T is None
    np.testing.assert_allclose(_n(v), po.potential(p.ys[:9], p.ys, p.yf, g, p.sigma, p.lam2), rtol=1e-12)
    u, v, T = gpu_ctx.potentials(*args, prm, _t(g), xq=_t(np.zeros((0, 3))), want_map=False)
    assert u.shape[0] == 0
