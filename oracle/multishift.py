"""Several shifts of one right-hand side, and the spectral bounds of M M^dagger (oracle, test-only).

Sec. 5.1 uses shifted operators M M^dagger + mu^2; Sec. 6.1 models the solver time by
the extreme eigenvalues lambda_min, lambda_max of M M^dagger (eq. (solver_time_eqn)),
and the tuning section places the Hasenbusch masses geometrically between them
(eq. (mu_i_eqn)).  The paper promises multi-shift solvers without giving one; the
reading here is the shared-Krylov CG for shifted systems (Jegerlehner's CG-M):

* `solve_shifts`   - the plain definition x_s = (A_0 + sigma_s)^{-1} b, one solve per
                     shift (A_0 = M M^dag + mu_0^2, sigma_s = mu_s^2 - mu_0^2);
* `cg_multishift`  - CG on A_0 with the shifted iterates carried along by the
                     recurrences zeta, alpha^s, beta^s (method oracle);
* `ritz_extremes`  - the Lanczos tridiagonal matrix that the CG coefficients define
                     (diagonal 1/alpha_k + beta_{k-1}/alpha_{k-1}, off-diagonal
                     sqrt(beta_k)/alpha_k) and its extreme eigenvalues;
* `spectrum_extremes` - the extreme eigenvalues of A by dense eigh or ARPACK;
* `hasenbusch_masses` - eq. (mu_i_eqn).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from .operator import Lattice, NormalOperator
from .solve import solve


def solve_shifts(lat: Lattice, phi, mu2s, b, tol: float = 1e-13):
    return [solve(lat, phi, float(m), b, tol=tol)[0] for m in mu2s]


def cg_multishift(Aop, b, sigmas, tol: float = 1e-12, maxiter: int = 100000):
    """CG on A_0 x = b carrying x_s = (A_0 + sigma_s)^{-1} b (sigma_s >= 0).

    Returns (xs, alphas, betas, iterations); each shifted system stops updating once
    its residual |zeta_s| |r| is below tol |b|."""
    b = np.asarray(b, dtype=np.complex128).ravel()
    ns = len(sigmas)
    bn = float(np.linalg.norm(b))
    x = np.zeros_like(b)
    r = b.copy()
    p = b.copy()
    xs = [np.zeros_like(b) for _ in range(ns)]
    ps = [b.copy() for _ in range(ns)]
    z_prev = np.ones(ns)      # zeta_{k-1}
    z_cur = np.ones(ns)       # zeta_k
    live = [True] * ns
    a_prev, b_prev = 1.0, 0.0  # alpha_{k-1}, beta_{k-1}
    rr = float(np.vdot(r, r).real)
    alphas, betas = [], []
    k = 0
    while np.sqrt(rr) > tol * bn and k < maxiter:
        q = Aop(p)
        a = rr / float(np.vdot(p, q).real)
        x = x + a * p
        r = r - a * q
        rr_new = float(np.vdot(r, r).real)
        beta = rr_new / rr
        for s in range(ns):
            if not live[s]:
                continue
            sg = float(sigmas[s])
            z_next = z_cur[s] * z_prev[s] * a_prev / (
                a * b_prev * (z_prev[s] - z_cur[s]) + z_prev[s] * a_prev * (1.0 + sg * a))
            a_s = a * z_next / z_cur[s]
            b_s = beta * (z_next / z_cur[s]) ** 2
            xs[s] = xs[s] + a_s * ps[s]
            ps[s] = z_next * r + b_s * ps[s]
            z_prev[s], z_cur[s] = z_cur[s], z_next
            if abs(z_next) * np.sqrt(rr_new) <= tol * bn:
                live[s] = False
        p = r + beta * p
        alphas.append(a)
        betas.append(beta)
        a_prev, b_prev = a, beta
        rr = rr_new
        k += 1
    return xs, np.array(alphas), np.array(betas), k


def lanczos_tridiagonal(alphas, betas) -> np.ndarray:
    """The k x k Lanczos matrix of the CG coefficients alpha_0..alpha_{k-1}, beta_0..beta_{k-1}."""
    a = np.asarray(alphas, dtype=np.float64)
    bt = np.asarray(betas, dtype=np.float64)
    k = len(a)
    T = np.zeros((k, k))
    for j in range(k):
        T[j, j] = 1.0 / a[j] + (bt[j - 1] / a[j - 1] if j > 0 else 0.0)
        if j + 1 < k:
            T[j, j + 1] = T[j + 1, j] = np.sqrt(bt[j]) / a[j]
    return T


def ritz_extremes(alphas, betas):
    ev = np.linalg.eigvalsh(lanczos_tridiagonal(alphas, betas))
    return float(ev[0]), float(ev[-1])


def spectrum_extremes(lat: Lattice, phi, mu2: float = 0.0, dense_limit: int = 3000):
    A = NormalOperator(lat, phi, mu2)
    if lat.n <= dense_limit:
        ev = np.linalg.eigvalsh(A.dense())
        return float(ev[0]), float(ev[-1])
    op = spla.LinearOperator((lat.n, lat.n), matvec=A, dtype=np.complex128)
    lmax = float(spla.eigsh(op, k=1, which="LA", return_eigenvectors=False, tol=1e-10)[0])
    lmin = float(spla.eigsh(op, k=1, sigma=0.0, which="LM", return_eigenvectors=False, tol=1e-10,
                            OPinv=spla.LinearOperator((lat.n, lat.n), dtype=np.complex128,
                                                      matvec=lambda v: solve(lat, phi, mu2, v)[0]))[0])
    return lmin, lmax


def hasenbusch_masses(lmin: float, lmax: float, n: int):
    """eq. (mu_i_eqn): mu_i = lambda_min (lambda_max / lambda_min)^((i+1)/(n+1)), i = 0..n-1."""
    return [lmin * (lmax / lmin) ** ((i + 1) / (n + 1)) for i in range(n)]
