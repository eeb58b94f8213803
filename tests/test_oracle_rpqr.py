"""Pins of the oracle's accelerated randomly pivoted QR (Alg. 5) against the
QR-Cholesky correspondence (Proposition qr_cholesky): on B it picks the same
pivots as accelerated RPCholesky (pinned on its own) on the Gram matrix
B^* B from the same uniform words, F equals that method's factor, Q is
orthonormal, B_hat = Q F^* satisfies B_hat^* B_hat = F F^*, and u is the
squared column norms of the residual B - B_hat."""
import numpy as np
import pytest

from oracle import DenseAccess, philox_stream, rpc_accel, rpqr_accel


def matrix(M, N, rank, decay, seed):
    rng = np.random.default_rng(seed)
    U = np.linalg.qr(rng.standard_normal((M, rank)))[0]
    V = np.linalg.qr(rng.standard_normal((N, rank)))[0]
    s = decay ** np.arange(rank)
    return (U * s) @ V.T + 1e-3 * rng.standard_normal((M, N))


@pytest.mark.parametrize("M,N,k,b,seed", [(300, 500, 60, 16, 0), (120, 700, 90, 37, 1), (400, 200, 30, 1, 2)])
def test_same_pivots_and_factor_as_cholesky_on_the_gram_matrix(M, N, k, b, seed):
    B = matrix(M, N, 80, 0.93, seed)
    qr = rpqr_accel(B, k, b, philox_stream(seed))
    ch = rpc_accel(DenseAccess(B.T @ B), k, b, philox_stream(seed))
    assert np.array_equal(qr.pivots, ch.pivots)
    assert qr.round_sizes == ch.round_sizes
    scale = np.linalg.norm(B) ** 2
    assert np.max(np.abs(qr.F - ch.F)) <= 1e-9 * np.sqrt(scale)
    assert np.allclose(qr.Q.T @ qr.Q, np.eye(qr.Q.shape[1]), atol=1e-12)
    Bh = qr.Q @ qr.F.T
    assert np.allclose(Bh.T @ Bh, ch.F @ ch.F.T, atol=1e-9 * scale)
    R = B - Bh
    u_direct = np.sum(R * R, axis=0)
    u_direct[qr.pivots] = 0.0
    assert np.allclose(qr.u, np.maximum(u_direct, 0.0), atol=1e-9 * scale)


def test_full_rank_reaches_the_exact_matrix():
    """k = M columns of a generic M x N matrix (M < N): Q spans R^M, so
    B_hat = Q Q^* B = B and the residual norms vanish."""
    rng = np.random.default_rng(5)
    B = rng.standard_normal((30, 200))
    qr = rpqr_accel(B, 30, 8, philox_stream(3))
    assert len(qr.pivots) == 30 and len(set(qr.pivots.tolist())) == 30
    assert np.allclose(qr.Q.T @ qr.Q, np.eye(30), atol=1e-12)
    assert np.allclose(qr.Q @ qr.F.T, B, atol=1e-10 * np.linalg.norm(B))
    assert np.sum(qr.u) <= 1e-12 * np.sum(B * B)


def test_extra_gram_schmidt_keeps_q_orthonormal_on_a_graded_matrix():
    """Singular values from 1 to 1e-12: one Gram-Schmidt pass would lose
    orthogonality (to about 1e-3 at k = 30); with the extra pass of Alg. 5 Q
    stays orthonormal to rounding."""
    rng = np.random.default_rng(0)
    U = np.linalg.qr(rng.standard_normal((300, 60)))[0]
    V = np.linalg.qr(rng.standard_normal((400, 60)))[0]
    B = (U * np.logspace(0, -12, 60)) @ V.T
    qr = rpqr_accel(B, 30, 10, philox_stream(1))
    assert len(qr.pivots) == 30
    assert np.max(np.abs(qr.Q.T @ qr.Q - np.eye(30))) <= 1e-12
