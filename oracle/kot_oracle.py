"""CPU FP64 oracle of the semismooth Newton (SSN) method for kernel-based OT (Lin, Cuturi, Jordan 2023).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import or call this module.  It shares no code with the HIP library and imports nothing from
the product package; the two meet only in the seeded input arrays.

Everything is plain numpy float64, written from the paper's definitions in the paper's order:

* Section 3 (finite-dimensional dual data): Gram matrices, mean embeddings, ``q^2``, ``z``, the kernel ``K`` on
  X x Y and its upper Cholesky factor ``R`` (columns ``Phi_i``), Eq. (3.4) and the estimator below it.
* Section 4.1: the operators ``Phi``/``Phi*``, the min-max form Eq. (4.1) and the residual map Eq. (4.2).
* Section 4.2: the spectral decomposition Eq. (4.4), the PSD projection and the Jacobian weight ``Omega``.
* Section 4.3: the inexactness rule Eq. (4.5), Algorithm 1 (Schur-complement Newton direction, Lemma 4.3),
  the weight ``Psi`` of the operator ``T`` applied in its plain dense form ``P (Psi o (P^T S P)) P^T``,
  and the adaptive ``theta`` rule.
* Section 4.4: Algorithm 2 (extragradient safeguard + regularized SSN + accept test).

Readings where the paper is silent or inconsistent (each is listed in the design notes):

* Gaussian kernel ``k(a, b) = exp(-|a - b|^2 / (2 sigma^2))`` for k_X, k_Y, and k_XY on the concatenated
  point, so ``K = K_X o K_Y``; one bandwidth for all three.
* ``q^2`` uses the squared norm of both mean embeddings (the dual-data definition omits one square).
* ``K`` is factored with a jitter: ``R^T R = K + eps I`` (eps = 1e-10 by default).
* Residual norm ``|R(w)| = |r1|_2 + |r2|_F`` (the pair norm of Section 4.3), absolute tolerance.
* Cold start ``gamma0 = 0, X0 = 0, theta0 = 1``; ``tau = kappa = 0.5``; ``theta`` clipped to [1e-6, 1e6].
* Eq. (4.5) is checked on the CG residual of the Schur system (the second block row of the full residual
  vanishes identically when the X-direction is formed as in Algorithm 1) against ``tau*min(1, kappa|r||a~1|)``
  (``|a~1| <= |dw|``, so the test is at least as strict).  CG stops at 20 iterations with its last iterate.
* The constants of Section 5: alpha1=1e-6, alpha2=1, beta0=0.5, beta2=5, and beta1 = 1/1.2: Section 5 prints
  beta1 = 1.2 and the theta rule's text asks for beta1 > 1, while Algorithm 2's input line asks for beta1 < 1.
  With 1.2, mu = theta |r| settles near alpha2 = 1 and the decoupled l = 1000 instances do not reach 1e-6 in
  200 iterations (1/1.2: 10 iterations).  ``Params(beta1=1.2)`` runs the printed value.
* Accept test as printed in Algorithm 2: w_{k+1} is the SSN trial when |R(trial)| <= |R(v_{k+1})|, else
  v_{k+1}.  ``Params(null_step=True)`` is an opt-in variant that keeps w_k when the trial is worse than w_k
  and w_k also beats v_{k+1}.
* Extragradient: Korpelevich steps on the monotone operator of Eq. (4.1),
  ``F(gamma, X) = ((Q gamma - z)/(2 lambda2) - Phi(X),  Phi*(gamma) + lambda1 I)`` with projection onto
  ``R^l x S^l_+``; default step ``0.5 / (|Q|_inf/(2 lambda2) + sqrt(|K o K|_inf))`` (a bound on 1/L).
* ``alpha = {i : sigma_i > 0}`` strictly.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict

import numpy as np

__all__ = [
    "Params", "Core", "gaussian_gram", "mean_embedding", "mean_gram", "setup", "core_from_arrays",
    "phi", "phi_star", "eig_sym", "proj_psd", "residual", "pair_norm", "pair_dot", "omega_matrix",
    "psi_matrix", "t_apply", "schur_matvec", "schur_diag", "cg", "pcg", "sqmr", "ssn_direction", "eg_operator", "eg_step",
    "default_eg_step", "theta_update", "solve", "ot_estimate", "kkt_report",
]


# ----------------------------------------------------------------------------------------------------------------
# Parameters (Algorithm 2 inputs and the Section 5 constants)
# ----------------------------------------------------------------------------------------------------------------
@dataclass
class Params:
    tol: float = 1e-6
    max_iter: int = 200
    cg_max_iter: int = 20          # Remark 4.5: CG capped at 20 iterations
    tau: float = 0.5               # Eq. (4.5)
    kappa: float = 0.5             # Eq. (4.5)
    alpha1: float = 1e-6           # Section 5 constants
    alpha2: float = 1.0
    beta0: float = 0.5
    beta1: float = 1.0 / 1.2       # reading: Algorithm 2 requires beta1 < 1; Section 5 prints 1.2
    beta2: float = 5.0
    theta0: float = 1.0
    theta_min: float = 1e-6
    theta_max: float = 1e6
    eg_step: float = 0.0           # 0 => default bound-based step
    safeguard: str = "eg"          # "eg" (Algorithm 2 as written), "none" (pure regularized SSN) or "eg_only"
                                   # (pure extragradient, the comparison method of Appendix F)
    null_step: bool = False        # False: Algorithm 2's accept test as printed; True: keep w_k when it beats
                                   # both the trial and v_{k+1} (opt-in variant)
    eps_jitter: float = 1e-10
    precond: str = "none"          # "none" (CG as the paper runs it) or "jacobi" (diagonal preconditioner of the
                                   # Schur system; an addition, the paper names none)
    schur_solver: str = "cg"       # "cg" (the paper's choice) or "sqmr" (symmetric QMR, the other solver it names)


@dataclass
class Core:
    """Finite-dimensional data of Eq. (3.4): ``Q, z, R`` (R^T R = K + eps I), ``q2`` and ``wsum = w_mu + w_nu``
    at the filling points (for the estimator), and the regularisers."""
    Q: np.ndarray
    z: np.ndarray
    R: np.ndarray
    q2: float
    wsum: np.ndarray
    lam1: float
    lam2: float
    extra: dict = field(default_factory=dict)

    @property
    def l(self) -> int:
        return self.Q.shape[0]


# ----------------------------------------------------------------------------------------------------------------
# Section 3: kernels and dual data
# ----------------------------------------------------------------------------------------------------------------
def _sqdist(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Squared distances as sum_k (a_k - b_k)^2 (no |a|^2+|b|^2-2ab expansion)."""
    diff = A[:, None, :] - B[None, :, :]
    return np.sum(diff * diff, axis=2)


def gaussian_gram(A: np.ndarray, B: np.ndarray, sigma: float, chunk: int = 256) -> np.ndarray:
    """k(a_i, b_j) = exp(-|a_i - b_j|^2 / (2 sigma^2))."""
    out = np.empty((A.shape[0], B.shape[0]))
    for s in range(0, A.shape[0], chunk):
        out[s:s + chunk] = np.exp(-_sqdist(A[s:s + chunk], B) / (2.0 * sigma * sigma))
    return out


def mean_embedding(samples: np.ndarray, pts: np.ndarray, sigma: float) -> np.ndarray:
    """w_hat(p_i) = (1/n) sum_j k(x_j, p_i)   (Section 3, embedding at the filling points)."""
    return gaussian_gram(pts, samples, sigma).mean(axis=1)


def mean_gram(samples: np.ndarray, sigma: float, chunk: int = 128) -> float:
    """|w_hat|^2 = (1/n^2) sum_{i,j} k(x_i, x_j)   (Section 3)."""
    n = samples.shape[0]
    tot = 0.0
    for s in range(0, n, chunk):
        tot += float(np.sum(gaussian_gram(samples[s:s + chunk], samples, sigma)))
    return tot / (n * n)


def setup(xs, ys, xf, yf, sigma: float, lam1: float, lam2: float, eps: float = 1e-10) -> Core:
    """Dual data of Eq. (3.4) from samples and filling points (Section 3)."""
    KX = gaussian_gram(xf, xf, sigma)
    KY = gaussian_gram(yf, yf, sigma)
    Q = KX + KY
    K = KX * KY                                   # Gaussian on the concatenated (x, y)
    wmu = mean_embedding(xs, xf, sigma)
    wnu = mean_embedding(ys, yf, sigma)
    c = np.sum((xf - yf) ** 2, axis=1)
    z = wmu + wnu - lam2 * c
    q2 = mean_gram(xs, sigma) + mean_gram(ys, sigma)
    L = np.linalg.cholesky(K + eps * np.eye(K.shape[0]))   # K + eps I = L L^T
    R = L.T                                               # upper triangular, R^T R = K + eps I
    return Core(Q=Q, z=z, R=R, q2=q2, wsum=wmu + wnu, lam1=lam1, lam2=lam2,
                extra=dict(KX=KX, KY=KY, K=K, wmu=wmu, wnu=wnu, c=c, eps=eps))


def core_from_arrays(Q, z, R, lam1, lam2, q2=0.0, wsum=None) -> Core:
    Q = np.asarray(Q, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    if wsum is None:
        wsum = np.zeros_like(z)
    return Core(Q=Q, z=z, R=R, q2=float(q2), wsum=np.asarray(wsum, dtype=np.float64), lam1=lam1, lam2=lam2)


# ----------------------------------------------------------------------------------------------------------------
# Section 4.1: operators and residual map
# ----------------------------------------------------------------------------------------------------------------
def phi(R: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Phi(X)_i = <X, Phi_i Phi_i^T> = Phi_i^T X Phi_i, Phi_i = R[:, i]."""
    return np.sum(R * (X @ R), axis=0)


def phi_star(R: np.ndarray, g: np.ndarray) -> np.ndarray:
    """Phi*(gamma) = sum_i gamma_i Phi_i Phi_i^T = R diag(gamma) R^T."""
    return (R * g[None, :]) @ R.T


def eig_sym(Z: np.ndarray):
    """Z = P diag(s) P^T, s ascending (Eq. 4.4)."""
    s, P = np.linalg.eigh(0.5 * (Z + Z.T))
    return s, P


def proj_psd(Z: np.ndarray, eig=None) -> np.ndarray:
    """Projection onto S^l_+: P_alpha Sigma_alpha P_alpha^T with alpha = {sigma_i > 0} (Section 4.2)."""
    s, P = eig if eig is not None else eig_sym(Z)
    a = s > 0
    Pa = P[:, a]
    return (Pa * s[a][None, :]) @ Pa.T


def pair_norm(g: np.ndarray, X: np.ndarray) -> float:
    """|w| = |gamma|_2 + |X|_F (Section 4.3)."""
    return float(np.linalg.norm(g) + np.linalg.norm(X))


def pair_dot(g1, X1, g2, X2) -> float:
    return float(g1 @ g2 + np.sum(X1 * X2))


def residual(core: Core, g: np.ndarray, X: np.ndarray):
    """Eq. (4.2): r1 = (Q g - z)/(2 lambda2) - Phi(X); r2 = X - Pi(X - (Phi*(g) + lambda1 I)).
    Returns (r1, r2, norm, (s, P)) with (s, P) the spectral data of Z = X - Phi*(g) - lambda1 I."""
    l = core.l
    r1 = (core.Q @ g - core.z) / (2.0 * core.lam2) - phi(core.R, X)
    Z = X - phi_star(core.R, g) - core.lam1 * np.eye(l)
    s, P = eig_sym(Z)
    r2 = X - proj_psd(Z, (s, P))
    return r1, r2, pair_norm(r1, r2), (s, P)


# ----------------------------------------------------------------------------------------------------------------
# Section 4.2-4.3: Jacobian weights and the operator T
# ----------------------------------------------------------------------------------------------------------------
def omega_matrix(s: np.ndarray) -> np.ndarray:
    """Omega: 1 on alpha x alpha, eta_ij = s_i/(s_i - s_j) on alpha x alpha-bar (and transpose), 0 elsewhere."""
    l = s.shape[0]
    a = s > 0
    Om = np.zeros((l, l))
    for i in range(l):
        for j in range(l):
            if a[i] and a[j]:
                Om[i, j] = 1.0
            elif a[i] and not a[j]:
                Om[i, j] = s[i] / (s[i] - s[j])
            elif a[j] and not a[i]:
                Om[i, j] = s[j] / (s[j] - s[i])
    return Om


def psi_matrix(s: np.ndarray, mu: float) -> np.ndarray:
    """Psi = Omega/(mu + 1 - Omega) entrywise: 1/mu on alpha x alpha, xi = eta/(mu + 1 - eta) on the
    off-diagonal blocks, 0 on alpha-bar x alpha-bar (Section 4.3)."""
    a = s > 0
    sa = s[:, None]
    sb = s[None, :]
    with np.errstate(divide="ignore", invalid="ignore"):
        eta_ij = sa / (sa - sb)          # valid where i in alpha, j in alpha-bar
        eta_ji = sb / (sb - sa)          # valid where j in alpha, i in alpha-bar
    Psi = np.zeros_like(eta_ij)
    aa = a[:, None] & a[None, :]
    ab = a[:, None] & ~a[None, :]
    ba = ~a[:, None] & a[None, :]
    Psi[aa] = 1.0 / mu
    Psi[ab] = eta_ij[ab] / (mu + 1.0 - eta_ij[ab])
    Psi[ba] = eta_ji[ba] / (mu + 1.0 - eta_ji[ba])
    return Psi


def t_apply(P: np.ndarray, Psi: np.ndarray, S: np.ndarray) -> np.ndarray:
    """T[S] = P (Psi o (P^T S P)) P^T  (plain dense form)."""
    return P @ (Psi * (P.T @ S @ P)) @ P.T


def schur_matvec(core: Core, P, Psi, mu: float, v: np.ndarray) -> np.ndarray:
    """(Q/(2 lambda2) + mu I + Phi T Phi*) v  (Algorithm 1, second step)."""
    return core.Q @ v / (2.0 * core.lam2) + mu * v + phi(core.R, t_apply(P, Psi, phi_star(core.R, v)))


def schur_diag(core: Core, P, Psi, mu: float) -> np.ndarray:
    """Diagonal of the Schur operator M = Q/(2 lambda2) + mu I + Phi T Phi* of Algorithm 1.

    With b = P^T R_i (R_i the i-th column of R), (Phi T Phi* e_i)_i = R_i^T P (Psi o (b b^T)) P^T R_i
    = sum_{r,s} Psi_rs b_r^2 b_s^2, so M_ii = Q_ii/(2 lambda2) + mu + [(B o B)^T Psi (B o B)]_ii, B = P^T R.
    """
    B = P.T @ core.R
    B2 = B * B
    return np.diag(core.Q) / (2.0 * core.lam2) + mu + np.einsum("ri,rs,si->i", B2, Psi, B2)


def pcg(matvec, b: np.ndarray, dinv: np.ndarray, stop, max_iter: int):
    """Preconditioned conjugate gradients with the diagonal preconditioner D (dinv = 1/diag(D)) from x = 0:
    z = D^-1 r, alpha = r.z / p.Ap, beta = r'.z' / r.z, p = z + beta p.  ``stop(res_norm, x)`` sees the
    unpreconditioned residual, as Eq. (4.5) asks."""
    x = np.zeros_like(b)
    r = b.copy()
    z = dinv * r
    p = z.copy()
    rr = float(r @ r)
    rz = float(r @ z)
    it = 0
    while it < max_iter:
        if stop(math.sqrt(rr), x):
            break
        Ap = matvec(p)
        pAp = float(p @ Ap)
        if pAp <= 0.0:
            break
        alpha = rz / pAp
        x = x + alpha * p
        r = r - alpha * Ap
        z = dinv * r
        rz_new = float(r @ z)
        p = z + (rz_new / rz) * p
        rz = rz_new
        rr = float(r @ r)
        it += 1
    return x, it, math.sqrt(rr)


def sqmr(matvec, b: np.ndarray, dinv, stop, max_iter: int):
    """Symmetric QMR (Freund and Nachtigal's simplified QMR for symmetric systems) with the symmetric diagonal
    preconditioner D (dinv = 1/diag(D), or None for none), from x = 0.

    Lanczos-type vectors: r (the BCG residual), q the search direction, rho = r^T D^-1 r.  Quasi-minimal
    residual: theta_k = |r_k|_{D^-1} / tau_{k-1}, c_k = 1/sqrt(1 + theta_k^2), tau_k = tau_{k-1} theta_k c_k,
    d_k = c_k^2 theta_{k-1}^2 d_{k-1} + c_k^2 alpha_k q_{k-1}, x_k = x_{k-1} + d_k.  The true residual
    s_k = b - A x_k is carried by s_k = s_{k-1} - A d_k with A d_k formed by the same recurrence, and
    ``stop(|s_k|, x_k)`` decides termination (Eq. 4.5)."""
    dv = np.ones_like(b) if dinv is None else dinv
    x = np.zeros_like(b)
    d = np.zeros_like(b)
    e = np.zeros_like(b)          # A d
    s = b.copy()                  # b - A x
    r = b.copy()
    q = dv * r
    rho = float(r @ q)
    tau = math.sqrt(rho)
    theta = 0.0
    it = 0
    while it < max_iter:
        if stop(float(np.linalg.norm(s)), x):
            break
        t = matvec(q)
        sigma = float(q @ t)
        if sigma <= 0.0 or rho <= 0.0:
            break
        alpha = rho / sigma
        r = r - alpha * t
        u = dv * r
        rho_new = float(r @ u)
        theta_old = theta
        theta = math.sqrt(rho_new) / tau
        c2 = 1.0 / (1.0 + theta * theta)
        tau = tau * theta * math.sqrt(c2)
        d = (c2 * theta_old * theta_old) * d + (c2 * alpha) * q
        e = (c2 * theta_old * theta_old) * e + (c2 * alpha) * t
        x = x + d
        s = s - e
        q = u + (rho_new / rho) * q
        rho = rho_new
        it += 1
    return x, it, float(np.linalg.norm(s))


def cg(matvec, b: np.ndarray, stop, max_iter: int):
    """Conjugate gradients from x = 0; ``stop(res_norm, x)`` decides termination (Eq. 4.5)."""
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = float(r @ r)
    it = 0
    while it < max_iter:
        if stop(math.sqrt(rr), x):
            break
        Ap = matvec(p)
        pAp = float(p @ Ap)
        if pAp <= 0.0:
            break
        alpha = rr / pAp
        x = x + alpha * p
        r = r - alpha * Ap
        rr_new = float(r @ r)
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
    return x, it, math.sqrt(rr)


def ssn_direction(core: Core, r1, r2, eig, mu: float, prm: Params):
    """Algorithm 1: Newton direction of Eq. (4.3) via the Schur complement of Lemma 4.3."""
    s, P = eig
    Psi = psi_matrix(s, mu)
    T = lambda S: t_apply(P, Psi, S)
    a1 = -r1 - phi(core.R, r2 + T(r2)) / (mu + 1.0)
    a2 = -r2
    rnorm = pair_norm(r1, r2)
    mv = lambda v: schur_matvec(core, P, Psi, mu, v)
    stop = lambda res, x: res <= prm.tau * min(1.0, prm.kappa * rnorm * float(np.linalg.norm(x)))
    if prm.precond not in ("none", "jacobi"):
        raise ValueError(f"unknown preconditioner {prm.precond!r}")
    dinv = 1.0 / schur_diag(core, P, Psi, mu) if prm.precond == "jacobi" else None
    if prm.schur_solver == "sqmr":
        at1, it, res = sqmr(mv, a1, dinv, stop, prm.cg_max_iter)
    elif prm.schur_solver != "cg":
        raise ValueError(f"unknown Schur-system solver {prm.schur_solver!r}")
    elif dinv is not None:
        at1, it, res = pcg(mv, a1, dinv, stop, prm.cg_max_iter)
    else:
        at1, it, res = cg(mv, a1, stop, prm.cg_max_iter)
    at2 = (a2 + T(a2)) / (mu + 1.0)
    dg = at1
    dX = at2 - T(phi_star(core.R, at1))
    return dg, dX, dict(cg_iters=it, cg_res=res, alpha=int(np.sum(s > 0)))


# ----------------------------------------------------------------------------------------------------------------
# Section 4.4: extragradient safeguard on Eq. (4.1)
# ----------------------------------------------------------------------------------------------------------------
def eg_operator(core: Core, g, X):
    """F(gamma, X) = ((Q g - z)/(2 lambda2) - Phi(X),  Phi*(g) + lambda1 I)."""
    Fg = (core.Q @ g - core.z) / (2.0 * core.lam2) - phi(core.R, X)
    FX = phi_star(core.R, g) + core.lam1 * np.eye(core.l)
    return Fg, FX


def default_eg_step(core: Core) -> float:
    """0.5 / Lhat, Lhat = |Q|_inf/(2 lambda2) + sqrt(|K o K|_inf) with K = R^T R  (bounds the Lipschitz
    constant of F: |Phi|^2 = |Phi Phi*| and Phi(Phi*(v)) = (K o K) v)."""
    K = core.R.T @ core.R
    qn = float(np.max(np.sum(np.abs(core.Q), axis=1)))
    kn = float(np.max(np.sum(np.abs(K * K), axis=1)))
    return 0.5 / (qn / (2.0 * core.lam2) + math.sqrt(kn))


def eg_step(core: Core, g, X, eta: float):
    """One Korpelevich step: v_half = Pi_C(v - eta F(v)), v+ = Pi_C(v - eta F(v_half)), C = R^l x S^l_+."""
    Fg, FX = eg_operator(core, g, X)
    gh = g - eta * Fg
    Xh = proj_psd(X - eta * FX)
    Fg2, FX2 = eg_operator(core, gh, Xh)
    gn = g - eta * Fg2
    Xn = proj_psd(X - eta * FX2)
    return gn, Xn


def theta_update(theta: float, rho: float, dw2: float, prm: Params) -> float:
    """Adaptive theta rule of Section 4.3 (rho = -<R(w + dw), dw>)."""
    if rho >= prm.alpha2 * dw2:
        return max(prm.theta_min, prm.beta0 * theta)
    if rho >= prm.alpha1 * dw2:
        return prm.beta1 * theta
    return min(prm.theta_max, prm.beta2 * theta)


def ot_estimate(core: Core, g: np.ndarray) -> float:
    """OT_hat = q^2/(2 lambda2) - (1/(2 lambda2)) sum_i gamma_i (w_mu(x~_i) + w_nu(y~_i))  (Section 3)."""
    return (core.q2 - float(g @ core.wsum)) / (2.0 * core.lam2)


def solve(core: Core, prm: Params | None = None, gamma0=None, X0=None, record: bool = True):
    """Algorithm 2 (EG-safeguarded regularized SSN).  Returns a dict with gamma, X, ot, residual, iters,
    status ('converged' / 'max_iter') and the per-iteration history."""
    prm = prm or Params()
    l = core.l
    g = np.zeros(l) if gamma0 is None else np.array(gamma0, dtype=np.float64)
    X = np.zeros((l, l)) if X0 is None else np.array(X0, dtype=np.float64)
    vg, vX = g.copy(), X.copy()
    theta = prm.theta0
    eta = prm.eg_step if prm.eg_step > 0 else default_eg_step(core)
    r1, r2, rn, eig = residual(core, g, X)
    rv = rn
    hist = []
    status = "max_iter"
    k = 0
    for k in range(prm.max_iter + 1):
        if record:
            hist.append(dict(k=k, res=rn, res_v=rv, theta=theta))
        if not np.isfinite(rn):
            status = "numeric"
            break
        if rn <= prm.tol:
            status = "converged"
            break
        if k == prm.max_iter:
            break
        if prm.safeguard == "eg_only":
            g, X = eg_step(core, g, X, eta)
            r1, r2, rn, eig = residual(core, g, X)
            rv = rn
            continue
        # (1) safeguard sequence: one EG step on v
        if prm.safeguard == "eg":
            vg, vX = eg_step(core, vg, vX, eta)
            vr1, vr2, rv, veig = residual(core, vg, vX)
        # (2) one regularized SSN step on w
        mu = theta * rn
        dg, dX, info = ssn_direction(core, r1, r2, eig, mu, prm)
        gt, Xt = g + dg, X + dX
        tr1, tr2, trn, teig = residual(core, gt, Xt)
        rho = -pair_dot(tr1, tr2, dg, dX)
        dw2 = pair_norm(dg, dX) ** 2
        theta = theta_update(theta, rho, dw2, prm)
        # (3) accept test
        accept = prm.safeguard != "eg" or trn <= rv
        if prm.null_step and trn > rn and (prm.safeguard != "eg" or rn <= rv):
            accept = None                       # null step: w_{k+1} = w_k
        elif accept:
            g, X, r1, r2, rn, eig = gt, Xt, tr1, tr2, trn, teig
        else:
            g, X, r1, r2, rn, eig = vg.copy(), vX.copy(), vr1, vr2, rv, veig
        if record:
            hist[-1].update(mu=mu, cg_iters=info["cg_iters"], cg_res=info["cg_res"], alpha=info["alpha"],
                            trial_res=trn, accepted_ssn=bool(accept), rho=rho)
    return dict(gamma=g, X=X, ot=ot_estimate(core, g), residual=rn, iters=k, status=status,
                history=hist, eg_step=eta, params=asdict(prm))


# ----------------------------------------------------------------------------------------------------------------
# Proposition 4.1: KKT report at a point
# ----------------------------------------------------------------------------------------------------------------
def kkt_report(core: Core, g: np.ndarray, X: np.ndarray) -> dict:
    """Stationarity |(Qg - z)/(2 lambda2) - Phi(X)|, dual feasibility lambda_min(Phi*(g) + lambda1 I),
    lambda_min(X) and complementarity <X, Phi*(g) + lambda1 I>."""
    S = phi_star(core.R, g) + core.lam1 * np.eye(core.l)
    stat = (core.Q @ g - core.z) / (2.0 * core.lam2) - phi(core.R, X)
    return dict(stationarity=float(np.linalg.norm(stat)),
                lmin_S=float(np.linalg.eigvalsh(0.5 * (S + S.T))[0]),
                lmin_X=float(np.linalg.eigvalsh(0.5 * (X + X.T))[0]),
                compl=float(np.sum(X * S)))
