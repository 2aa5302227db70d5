"""Brute-force dense forms for tiny l (l <= 8): test infrastructure only (see ``kot_oracle``).

* ``jacobian_dense``: the (l + l^2) x (l + l^2) matrix of the element of the generalized Jacobian of the
  residual map Eq. (4.2) built column by column from the directional derivative of each block:
  d r1 = Q dg/(2 lambda2) - Phi(dX),  d r2 = dX - M(Z)[dX - Phi*(dg)],  with M(Z)[S] = P(Omega o P^T S P)P^T
  (Section 4.2).  No Schur complement, no T operator, no CG.
* ``newton_dense``: the exact solution of (J + mu I) dw = -r by a dense LU solve.
* ``proj_jacobian_fd``: central finite differences of the PSD projection along a symmetric direction.
"""
from __future__ import annotations

import numpy as np

from . import kot_oracle as ko

__all__ = ["jacobian_dense", "newton_dense", "proj_jacobian_fd", "m_apply"]


def m_apply(P, Om, S):
    return P @ (Om * (P.T @ S @ P)) @ P.T


def jacobian_dense(core: ko.Core, eig):
    s, P = eig
    l = core.l
    Om = ko.omega_matrix(s)
    n = l + l * l
    J = np.zeros((n, n))
    for c in range(n):
        dg = np.zeros(l)
        dX = np.zeros((l, l))
        if c < l:
            dg[c] = 1.0
        else:
            dX.flat[c - l] = 1.0
        d1 = core.Q @ dg / (2 * core.lam2) - ko.phi(core.R, dX)
        d2 = dX - m_apply(P, Om, dX - ko.phi_star(core.R, dg))
        J[:l, c] = d1
        J[l:, c] = d2.ravel()
    return J


def newton_dense(core: ko.Core, r1, r2, eig, mu):
    l = core.l
    J = jacobian_dense(core, eig)
    rhs = -np.concatenate([r1, r2.ravel()])
    sol = np.linalg.solve(J + mu * np.eye(J.shape[0]), rhs)
    return sol[:l], sol[l:].reshape(l, l)


def proj_jacobian_fd(Z, S, h=1e-6):
    return (ko.proj_psd(Z + h * S) - ko.proj_psd(Z - h * S)) / (2 * h)
