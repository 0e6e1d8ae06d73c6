"""Conjugate gradient on the normal equations (Sec. 2.2, algorithm "alg. cg").

D is not Hermitian, but gamma_5 D gamma_5 = D^dag (Sec. 2.2), so CG runs on a
Hermitian positive-definite normal operator.  The paper's listing solves
D D^dag y = eta and sets psi = D^dag y (CGNE, ``cgne``); the default here is
the other normal form, D^dag D x = D^dag b (CGNR, ``cgnr``).  Both reach the
unique x = D^{-1} b.

Readings of the printed listing:
* |.| in the step lengths is the squared 2-norm, so for CGNR
  alpha = ||r||^2 / ||D p||^2 (= <r, r> / <p, D^dag D p>) and
  beta = ||r_new||^2 / ||r_old||^2.
* The initial residual is that of the normal equations: x0 = 0 gives
  r0 = b' = D^dag b; a warm start x0 gives r0 = b' - D^dag D x0.
* Stopping: ||r|| <= tol * ||b'|| (2-norms, relative) instead of the
  listing's absolute r_min, plus an iteration cap.

``matvec`` and ``matvec_dag`` are callables on canonical arrays, so the same
routine runs with the stencil or with a dense matrix.
"""
from __future__ import annotations

import numpy as np


def _dot_re(a, b):
    return float(np.sum(np.asarray(a, np.float64) * np.asarray(b, np.float64)))


def cgnr(matvec, matvec_dag, b: np.ndarray, tol: float = 1e-10, max_iter: int = 20000,
         x0: np.ndarray | None = None):
    """Return (x, iterations, info) for D^dag D x = D^dag b.

    info holds 'rel_resid' (||r_k|| / ||b'|| by the recurrence), 'history'
    of ||r_k||^2, 'alphas' and 'betas' (for a Lanczos condition estimate),
    and 'converged'.
    """
    b = np.asarray(b, dtype=np.float64)
    bp = matvec_dag(b)
    bnorm2 = _dot_re(bp, bp)
    if x0 is None:
        x = np.zeros_like(b)
        r = bp.copy()
    else:
        x = np.array(x0, dtype=np.float64)
        r = bp - matvec_dag(matvec(x))
    p = r.copy()
    rr = _dot_re(r, r)
    hist = [rr]
    alphas, betas = [], []
    it = 0
    target = (tol ** 2) * bnorm2
    while rr > target and it < max_iter:
        t = matvec(p)
        tt = _dot_re(t, t)  # <p, D^dag D p> = ||D p||^2
        alpha = rr / tt
        x = x + alpha * p
        r = r - alpha * matvec_dag(t)
        rr_new = _dot_re(r, r)
        beta = rr_new / rr
        p = r + beta * p
        rr = rr_new
        it += 1
        hist.append(rr)
        alphas.append(alpha)
        betas.append(beta)
    info = {
        "rel_resid": float(np.sqrt(rr / bnorm2)) if bnorm2 > 0 else 0.0,
        "history": hist,
        "alphas": alphas,
        "betas": betas,
        "converged": rr <= target,
        "bnorm2": bnorm2,
    }
    return x, it, info


def cgne(matvec, matvec_dag, b: np.ndarray, tol: float = 1e-10, max_iter: int = 20000):
    """Return (x, iterations, info) for the paper's form of Sec. 2.2: CG on
    D D^dag y = b, then x = D^dag y.

    Step lengths as read for CGNR, with the roles of D and D^dag exchanged:
    alpha = ||r||^2 / ||D^dag p||^2, r -= alpha D (D^dag p), beta =
    ||r_new||^2 / ||r_old||^2.  r is the residual of D x = b itself, so the
    stop is ||b - D x|| <= tol * ||b||.  Starts from y = 0.
    """
    b = np.asarray(b, dtype=np.float64)
    bnorm2 = _dot_re(b, b)
    y = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = bnorm2
    alphas, betas = [], []
    it = 0
    target = (tol ** 2) * bnorm2
    while rr > target and it < max_iter:
        t = matvec_dag(p)
        tt = _dot_re(t, t)  # <p, D D^dag p> = ||D^dag p||^2
        alpha = rr / tt
        y = y + alpha * p
        r = r - alpha * matvec(t)
        rr_new = _dot_re(r, r)
        beta = rr_new / rr
        p = r + beta * p
        rr = rr_new
        it += 1
        alphas.append(alpha)
        betas.append(beta)
    x = matvec_dag(y)
    info = {
        "rel_resid": float(np.sqrt(rr / bnorm2)) if bnorm2 > 0 else 0.0,
        "alphas": alphas,
        "betas": betas,
        "converged": rr <= target,
        "bnorm2": bnorm2,
    }
    return x, it, info


def lanczos_condition(alphas, betas) -> float:
    """Estimate cond(D^dag D) from CG's alpha/beta (the Lanczos tridiagonal).

    T has diagonal 1/a_k + b_{k-1}/a_{k-1} and off-diagonal sqrt(b_k)/a_k.
    """
    n = len(alphas)
    if n == 0:
        return 1.0
    T = np.zeros((n, n))
    for k in range(n):
        T[k, k] = 1.0 / alphas[k] + (betas[k - 1] / alphas[k - 1] if k > 0 else 0.0)
        if k + 1 < n:
            T[k, k + 1] = T[k + 1, k] = np.sqrt(betas[k]) / alphas[k]
    ev = np.linalg.eigvalsh(T)
    return float(ev[-1] / ev[0])
