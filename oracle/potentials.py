"""CPU FP64 oracle of the Kantorovich potentials and the transport map recovered from the dual solution.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import or call this module.  It shares no code with the HIP library.

Section 3: the empirical problem Eq. (3.2) maximizes over ``u, v, A`` with the equality constraints at the
filling points.  Its Lagrangian with multipliers ``gamma_i`` on the constraints is stationary in ``u`` when
``w_mu_hat - 2 lambda2 u - sum_i gamma_i phi_X(x~_i) = 0``, so the maximizers are

    u^(x) = (w_mu_hat(x) - sum_i gamma_i k_X(x~_i, x)) / (2 lambda2),
    v^(y) = (w_nu_hat(y) - sum_i gamma_i k_Y(y~_i, y)) / (2 lambda2),

with ``w_mu_hat(x) = (1/n) sum_j k_X(x_j, x)``.  Pairing them with the embeddings (reproducing property)
gives back the estimator of Section 3, ``<u^, w_mu_hat> + <v^, w_nu_hat> = (q^2 - gamma^T (w_mu + w_nu)) /
(2 lambda2)``.  For the cost ``|x - y|^2 / 2`` the map pushing mu forward is ``T(x) = x - grad u^(x)``
(the gradient of the convex ``|x|^2/2 - u``), the reading used for the maps the paper plots in Section 5.

Gaussian kernel ``k(a, b) = exp(-|a - b|^2 / (2 sigma^2))``, so ``grad_x k(a, x) = k(a, x) (a - x) / sigma^2``.
"""
from __future__ import annotations

import numpy as np

__all__ = ["kernel_rows", "potential", "potential_grad", "transport_map"]


def kernel_rows(q: np.ndarray, pts: np.ndarray, sigma: float) -> np.ndarray:
    """k(pts_j, q_i) for every query row i and point j, squared distances summed coordinate by coordinate."""
    d2 = np.zeros((q.shape[0], pts.shape[0]))
    for k in range(q.shape[1]):
        diff = q[:, k][:, None] - pts[:, k][None, :]
        d2 += diff * diff
    return np.exp(-d2 / (2.0 * sigma * sigma))


def potential(q: np.ndarray, samples: np.ndarray, fill: np.ndarray, gamma: np.ndarray, sigma: float,
              lam2: float) -> np.ndarray:
    """u^(q) (or v^ with the target samples and the y-parts of the filling points), one value per query row."""
    w = kernel_rows(q, samples, sigma).mean(axis=1)
    s = kernel_rows(q, fill, sigma) @ gamma
    return (w - s) / (2.0 * lam2)


def potential_grad(q: np.ndarray, samples: np.ndarray, fill: np.ndarray, gamma: np.ndarray, sigma: float,
                   lam2: float) -> np.ndarray:
    """grad u^(q): (1/n) sum_j k(x_j, q)(x_j - q)/sigma^2 - sum_i gamma_i k(x~_i, q)(x~_i - q)/sigma^2, / (2 lam2)."""
    ks = kernel_rows(q, samples, sigma) / samples.shape[0]      # m x n
    kf = kernel_rows(q, fill, sigma) * gamma[None, :]            # m x l
    gw = ks @ samples - ks.sum(axis=1)[:, None] * q
    gs = kf @ fill - kf.sum(axis=1)[:, None] * q
    return (gw - gs) / (sigma * sigma) / (2.0 * lam2)


def transport_map(q: np.ndarray, samples: np.ndarray, fill: np.ndarray, gamma: np.ndarray, sigma: float,
                  lam2: float) -> np.ndarray:
    """T(q) = q - grad u^(q)."""
    return q - potential_grad(q, samples, fill, gamma, sigma, lam2)
