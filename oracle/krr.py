"""Kernel ridge regression by preconditioned conjugate gradients with a
low-rank preconditioner (Section 3.2), written plainly in FP64 numpy.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The system is (A + mu I) beta = y with A the kernel matrix of the training
points; the preconditioner is P = F F^* + mu I for a rank-k factor F (the
output of a pivoted partial Cholesky method), applied through the Woodbury
identity P^{-1} r = (r - F (mu I + F^* F)^{-1} F^* r) / mu.  PCG is the
textbook iteration (Golub and Van Loan, Alg. 11.5.1) from beta = 0, stopped
when |r| <= tol |y|.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import cho_factor, cho_solve

from .kernels import kernel_block


def kernel_matvec(X: np.ndarray, kernel: int, sigma: float, v: np.ndarray, mu: float, chunk: int = 2048):
    """(A + mu I) v, regenerating A a block of rows at a time."""
    N = X.shape[0]
    out = np.empty(N)
    for r0 in range(0, N, chunk):
        R = np.arange(r0, min(r0 + chunk, N))
        out[R] = kernel_block(X, R, slice(None), kernel, sigma) @ v
    return out + mu * v


def woodbury_apply(F: np.ndarray, mu: float):
    """r -> (F F^* + mu I)^{-1} r through the k x k system mu I + F^* F."""
    k = F.shape[1]
    if k == 0:
        return lambda r: r / mu
    M = cho_factor(mu * np.eye(k) + F.T @ F, lower=True)
    return lambda r: (r - F @ cho_solve(M, F.T @ r)) / mu


def pcg(apply_A, apply_Pinv, y: np.ndarray, tol: float, max_iter: int):
    """Returns (beta, iterations, relative residual |y - A beta| / |y| as
    tracked by the recurrence)."""
    beta = np.zeros_like(y)
    r = y.copy()
    ny = np.linalg.norm(y)
    z = apply_Pinv(r)
    p = z.copy()
    rz = r @ z
    it = 0
    rel = np.linalg.norm(r) / ny
    while it < max_iter and rel > tol:
        q = apply_A(p)
        alpha = rz / (p @ q)
        beta += alpha * p
        r -= alpha * q
        it += 1
        rel = np.linalg.norm(r) / ny
        if rel <= tol:
            break
        z = apply_Pinv(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return beta, it, rel


def krr_pcg(X, kernel: int, sigma: float, mu: float, y, F, tol: float = 1e-8, max_iter: int = 1000):
    """Solve (A + mu I) beta = y by PCG with P = F F^* + mu I."""
    X = np.asarray(X, dtype=np.float64)
    F = np.asarray(F, dtype=np.float64)
    return pcg(lambda v: kernel_matvec(X, kernel, sigma, v, mu), woodbury_apply(F, mu),
               np.asarray(y, dtype=np.float64), tol, max_iter)
