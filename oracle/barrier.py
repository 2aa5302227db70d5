"""Independent generic convex solver for Eq. (3.4): log-barrier path following with damped Newton steps.

TEST INFRASTRUCTURE ONLY (see ``kot_oracle``).  It does not use the residual map, the eigendecomposition or
any piece of Algorithms 1-2; it is the textbook barrier method (Boyd & Vandenberghe, Section 11.3) on

    min_gamma  f(gamma) = gamma^T Q gamma/(4 lambda2) - gamma^T z/(2 lambda2)
    s.t.       S(gamma) = sum_i gamma_i Phi_i Phi_i^T + lambda1 I  >= 0,

minimising f - t log det S for a decreasing sequence of t.  Feasibility is kept by Cholesky-tested
backtracking.  At a central point X = t S^{-1} is a dual multiplier; the duality gap is t * l.
"""
from __future__ import annotations

import numpy as np

__all__ = ["barrier_solve"]


def _S(R, lam1, g):
    return (R * g[None, :]) @ R.T + lam1 * np.eye(R.shape[0])


def _is_pd(S):
    try:
        np.linalg.cholesky(0.5 * (S + S.T))
        return True
    except np.linalg.LinAlgError:
        return False


def barrier_solve(Q, z, R, lam1, lam2, t0: float = 1.0, t_end: float = 1e-12, shrink: float = 0.2,
                  newton_tol: float = 1e-13, max_newton: int = 200):
    l = Q.shape[0]
    g = np.zeros(l)                      # S = lam1 I > 0: strictly feasible
    t = t0

    def obj(gv, tv):
        S = _S(R, lam1, gv)
        sign, logdet = np.linalg.slogdet(S)
        if sign <= 0:
            return np.inf
        return gv @ Q @ gv / (4 * lam2) - gv @ z / (2 * lam2) - tv * logdet

    newton_total = 0
    while True:
        for _ in range(max_newton):
            S = _S(R, lam1, g)
            Sinv = np.linalg.inv(S)
            G = R.T @ Sinv @ R                                  # G_ij = Phi_i^T S^-1 Phi_j
            grad = (Q @ g - z) / (2 * lam2) - t * np.diag(G)
            H = Q / (2 * lam2) + t * G * G
            step = -np.linalg.solve(H, grad)
            dec = float(-grad @ step)                            # Newton decrement squared
            if dec / 2 <= newton_tol * max(1.0, abs(obj(g, t))):
                break
            s = 1.0
            f0 = obj(g, t)
            while True:
                gn = g + s * step
                if _is_pd(_S(R, lam1, gn)) and obj(gn, t) <= f0 - 0.25 * s * dec:
                    break
                s *= 0.5
                if s < 1e-20:
                    break
            g = g + s * step
            newton_total += 1
            if s < 1e-20:
                break
        if t <= t_end:
            break
        t = max(t * shrink, t_end)
    S = _S(R, lam1, g)
    X = t * np.linalg.inv(S)
    return dict(gamma=g, X=0.5 * (X + X.T), t=t, gap=t * l, newton_steps=newton_total)
