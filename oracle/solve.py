"""Solutions of (M M^dagger + mu^2) x = b (oracle, test-only).

Sec. 3 of the paper: M M^dagger is Hermitian positive definite, so the solution
is unique and CG applies; the paper's double-precision CG stops at a relative
tolerance.  The shift mu^2 is the Hasenbusch mass shift of Sec. 5.1.

* `solve_dense` - LU solve of the dense matrix (the plain definition, small N);
* `cg`          - textbook conjugate gradients in complex128 on the sparse
                  operator, stopped on the recursive residual and then certified
                  by the true residual ||b - A x|| / ||b|| recomputed in FP64
                  (restarted from x if the certificate fails);
* `solve`       - picks one of the two and returns x with its certificate;
* `fgmres_alg_a1` - the flexible GMRES of Appendix A (Algorithm A.1) with a
                  single-precision CG preconditioner emulated in NumPy complex64.
                  This is a method oracle for the structure and iteration counts
                  of the mixed solver, not the parity target (the parity target
                  is the unique solution above).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .operator import Lattice, NormalOperator, build_M


def solve_dense(A: np.ndarray, b: np.ndarray) -> np.ndarray:
    return np.linalg.solve(A, b)


def _norm(v) -> float:
    return float(np.sqrt(np.vdot(v, v).real))


def cg(Aop, b: np.ndarray, tol: float = 1e-13, maxiter: int = 100000, x0=None):
    """Conjugate gradients (Hestenes-Stiefel) on a Hermitian positive-definite operator.

    Returns (x, iterations, true relative residual)."""
    b = np.asarray(b, dtype=np.complex128)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    bnorm = _norm(b)
    if bnorm == 0.0:
        return np.zeros_like(b), 0, 0.0
    it = 0
    while True:
        r = b - Aop(x)
        if _norm(r) <= tol * bnorm or it >= maxiter:
            return x, it, _norm(r) / bnorm
        p = r.copy()
        rr = np.vdot(r, r).real
        while it < maxiter:
            q = Aop(p)
            alpha = rr / np.vdot(p, q).real
            x = x + alpha * p
            r = r - alpha * q
            rr_new = np.vdot(r, r).real
            it += 1
            if np.sqrt(rr_new) <= tol * bnorm:
                break
            p = r + (rr_new / rr) * p
            rr = rr_new
        # loop back: certify with the true residual, restart from x if needed


def true_rel_residual(lat: Lattice, phi, mu2: float, b, x, A: NormalOperator | None = None) -> float:
    """||b - (M M^dagger + mu^2) x|| / ||b|| in FP64."""
    A = NormalOperator(lat, phi, mu2) if A is None else A
    bf = np.asarray(b, dtype=np.complex128).ravel()
    xf = np.asarray(x, dtype=np.complex128).ravel()
    return _norm(bf - A(xf)) / _norm(bf)


def solve(lat: Lattice, phi, mu2: float, b, tol: float = 1e-13, dense_limit: int = 2500, A=None):
    """x = (M M^dagger + mu^2)^{-1} b for one right-hand side.

    Dense LU for N <= dense_limit, else CG certified to `tol`.  Returns
    (x shaped like b, true relative residual)."""
    A = NormalOperator(lat, phi, mu2) if A is None else A
    bf = np.asarray(b, dtype=np.complex128).ravel()
    if lat.n <= dense_limit:
        x = solve_dense(A.dense(), bf)
    else:
        x, _, _ = cg(A, bf, tol=tol)
    return x.reshape(np.shape(b)), true_rel_residual(lat, phi, mu2, bf, x, A)


# ----------------------------------------------------------------------------
# Method oracle: Algorithm A.1 (flexible GMRES, spCG preconditioner).
# ----------------------------------------------------------------------------

def _spcg_c64(A32, mu2, v: np.ndarray, tol: float, maxiter: int):
    """Single-precision CG with x0 = 0, stopped on the recursive residual (complex64
    storage and arithmetic, float32 accumulation).  Returns (z, iterations)."""
    b = v.astype(np.complex64)
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = np.float32(np.vdot(r, r).real)
    stop = np.float32(tol) ** 2 * rr
    it = 0
    while it < maxiter and rr > stop:
        q = A32(p)
        alpha = np.float32(rr / np.float32(np.vdot(p, q).real))
        x = x + alpha * p
        r = r - alpha * q
        rr_new = np.float32(np.vdot(r, r).real)
        p = r + np.float32(rr_new / rr) * p
        rr = rr_new
        it += 1
    return x, it


def fgmres_alg_a1(lat: Lattice, phi, mu2: float, b, TOL: float = 1e-10, m: int = 10, a: float = 5.0,
                  inner_floor: float = 1e-5, inner_maxiter: int = 5000, max_outer: int = 50,
                  record: list | None = None):
    """Flexible GMRES of Appendix A with spCG preconditioning, read as follows.

    * The initial spCG and every inner spCG start from zero and stop at the relative
      recursive residual tau = max(TOL * a * |b| / ERR, inner_floor) (ERR = |b| for
      the initial solve); the floor keeps the request reachable in single precision.
    * h and y are complex; h_ij = v_i^H w (classical Gram-Schmidt: all projections
      first, then one subtraction).
    * ERR, the residual estimate the step's inner tolerance and the cycle's break
      test use, is after each Arnoldi step the least-squares residual
      min_y |(|r|, 0, ...) - h y| of the steps so far: the residual of the best
      iterate of the cycle.  The printed update ERR <- ERR * |w| is that quantity
      when each step's inner solve meets its tolerance (|w| is then the reduction the
      solve achieved); after an unpreconditioned step (z_j = v_j) the product no
      longer tracks the residual and ends cycles early.
    * The small least-squares problem min |(|r|, 0, ...) - h y| is solved with
      numpy's lstsq; the update runs over the Arnoldi steps actually completed.
    * Outer test: recomputed FP64 true residual |b - A x| <= TOL |b|.

    Returns (x, info) with info = dict(outer=number of restart cycles,
    arnoldi=Arnoldi steps, inner_solves, inner_iters, true_rel_resid).  A list passed
    as `record` receives, per restart cycle, the cycle's start x0, its vectors v_j
    and z_j, the values TOL a |b| / ERR of the inner-solve test and ERR after each step
    (for tests of the cycle's minimal-residual property, of the residual estimate and
    of how close the inner-solve test came to 1)."""
    M = build_M(lat, phi)
    A = NormalOperator(lat, phi, mu2, M=M)
    M32 = M.astype(np.complex64)
    M32h = M32.conj().T.tocsr()
    mu2_32 = np.float32(mu2)

    def A32(x):
        return M32 @ (M32h @ x) + mu2_32 * x

    bf = np.asarray(b, dtype=np.complex128).ravel()
    bnorm = _norm(bf)
    info = dict(outer=0, arnoldi=0, inner_solves=0, inner_iters=0)
    z0, its = _spcg_c64(A32, mu2, bf, max(TOL * a, inner_floor), inner_maxiter)
    info["inner_solves"] += 1
    info["inner_iters"] += its
    x = z0.astype(np.complex128)
    r = bf - A(x)
    ERR = _norm(r)
    w = r.copy()
    while ERR > TOL * bnorm and info["outer"] < max_outer:
        rnorm = ERR
        V, Z, ratios, errs = [], [], [], []
        H = np.zeros((m + 1, m), dtype=np.complex128)
        k = 0
        for j in range(m):
            if ERR < TOL * bnorm:
                break
            wn = _norm(w)
            if wn == 0.0:
                break
            V.append(w / wn)
            ratio = TOL * a * bnorm / ERR
            ratios.append(ratio)
            if ratio < 1.0:
                z, its = _spcg_c64(A32, mu2, V[j], max(ratio, inner_floor), inner_maxiter)
                info["inner_solves"] += 1
                info["inner_iters"] += its
                Z.append(z.astype(np.complex128))
            else:
                Z.append(V[j].copy())
            w = A(Z[j])
            for i in range(j + 1):
                H[i, j] = np.vdot(V[i], w)
            for i in range(j + 1):
                w = w - H[i, j] * V[i]
            H[j + 1, j] = _norm(w)
            e1 = np.zeros(j + 2, dtype=np.complex128)
            e1[0] = rnorm
            yj = np.linalg.lstsq(H[: j + 2, : j + 1], e1, rcond=None)[0]
            ERR = _norm(e1 - H[: j + 2, : j + 1] @ yj)
            errs.append(ERR)
            k = j + 1
            info["arnoldi"] += 1
        if k == 0:
            break
        rhs = np.zeros(k + 1, dtype=np.complex128)
        rhs[0] = rnorm
        y = np.linalg.lstsq(H[: k + 1, :k], rhs, rcond=None)[0]
        if record is not None:
            record.append(dict(x0=x.copy(), V=[v.copy() for v in V[:k]], Z=[z.copy() for z in Z[:k]],
                               ratio=list(ratios[:k]), err=list(errs[:k])))
        for i in range(k):
            x = x + y[i] * Z[i]
        r = bf - A(x)
        ERR = _norm(r)
        w = r.copy()
        info["outer"] += 1
    info["true_rel_resid"] = _norm(bf - A(x)) / bnorm
    return x.reshape(np.shape(b)), info
