"""Pins of the oracle's kernel ridge regression (Section 3.2): the PCG
solution solves (A + mu I) beta = y (checked against a dense direct solve),
the Woodbury form of P^{-1} equals a dense solve with F F^* + mu I, an exact
factor (F F^* = A) converges in one iteration, and the preconditioner from
accelerated RPCholesky cuts the iteration count against plain CG."""
import numpy as np

from oracle import PointsAccess, kernel_matvec, pcg, philox_stream, rpc_accel, woodbury_apply
from oracle.kernels import kernel_block
from paper_2410_03969_amd import workloads as W


def problem(N=1500, d=4, seed=0):
    rng = np.random.default_rng(seed)
    X = rng.random((N, d))
    y = np.sin(3 * X).sum(axis=1) + 0.01 * rng.standard_normal(N)
    return X, y, float(np.sqrt(d)), 1e-9 * N


def test_matvec_and_solution_against_dense():
    X, y, sigma, mu = problem(N=800)
    A = kernel_block(X, slice(None), slice(None), W.MATERN52, sigma)
    v = np.random.default_rng(1).standard_normal(X.shape[0])
    assert np.allclose(kernel_matvec(X, W.MATERN52, sigma, v, mu, chunk=333), A @ v + mu * v, rtol=1e-12,
                       atol=1e-10)
    F = rpc_accel(PointsAccess(X, W.MATERN52, sigma), 150, 15, philox_stream(0)).F
    beta, it, rel = pcg(lambda u: A @ u + mu * u, woodbury_apply(F, mu), y, 1e-10, 2000)
    res = np.linalg.norm(A @ beta + mu * beta - y) / np.linalg.norm(y)
    assert rel <= 1e-10 and res <= 1e-9


def test_woodbury_equals_dense_solve():
    rng = np.random.default_rng(2)
    F = rng.standard_normal((300, 40))
    mu = 0.3
    r = rng.standard_normal(300)
    want = np.linalg.solve(F @ F.T + mu * np.eye(300), r)
    assert np.allclose(woodbury_apply(F, mu)(r), want, rtol=1e-10, atol=1e-12)


def test_exact_preconditioner_converges_in_one_iteration():
    X, y, sigma, mu = problem(N=400)
    A = kernel_block(X, slice(None), slice(None), W.MATERN52, sigma)
    F = np.linalg.cholesky(A + 1e-12 * np.eye(400))       # F F^* = A (to 1e-12)
    beta, it, rel = pcg(lambda v: A @ v + mu * v, woodbury_apply(F, mu), y, 1e-6, 50)
    assert it == 1


def test_rpcholesky_preconditioner_beats_plain_cg():
    X, y, sigma, mu = problem(N=800)
    A = kernel_block(X, slice(None), slice(None), W.MATERN52, sigma)
    F = rpc_accel(PointsAccess(X, W.MATERN52, sigma), 150, 15, philox_stream(0)).F
    _, it_p, _ = pcg(lambda u: A @ u + mu * u, woodbury_apply(F, mu), y, 1e-6, 3000)
    _, it_0, rel_0 = pcg(lambda u: A @ u + mu * u, woodbury_apply(np.zeros((800, 0)), mu), y, 1e-6, 5 * it_p)
    assert rel_0 > 1e-6, (it_p, it_0, rel_0)          # plain CG is not done after 5x the iterations
