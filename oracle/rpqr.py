"""Accelerated randomly pivoted QR (Alg. 5; Section 5), written plainly in
FP64 numpy.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Readings where the paper leaves a choice:
* Orth (orthonormalize the columns) is the QR factorization with a positive
  diagonal in R, so Q and F are unique and comparable entry by entry.
* The residual column norms of the accepted pivots are set to exactly zero
  after each round (their exact value), as the Cholesky methods do.
* Rounds, uniform words, duplicate and cap rules and stopping are those of
  rpc_accel, with the residual Gram matrix C^* C in place of H.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .rpc import draw_proposals, reject_sample_submatrix


@dataclass
class QRResult:
    Q: np.ndarray          # M x k_out, orthonormal columns
    F: np.ndarray          # N x k_out, F = B^* Q, so B_hat = Q F^*
    pivots: np.ndarray     # acceptance order
    u: np.ndarray          # final residual squared column norms
    rounds: int
    status: str
    round_sizes: list = field(default_factory=list)


def orth(Y: np.ndarray) -> np.ndarray:
    """Q of the QR factorization Y = Q R with diag(R) > 0."""
    Qy, R = np.linalg.qr(Y)
    sgn = np.where(np.diag(R) < 0, -1.0, 1.0)
    return Qy * sgn


def rpqr_accel(B: np.ndarray, k: int, b: int, stream, max_rounds=None) -> QRResult:
    """Alg. 5: propose b columns from the residual squared column norms,
    keep a subset by RejectionSampleSubmatrix (Alg. 1) on C^* C, extend Q by
    the residual columns of the kept pivots (one extra Gram-Schmidt pass,
    then Orth) and F by B^* Q_perp."""
    B = np.asarray(B, dtype=np.float64)
    M, N = B.shape
    u = np.sum(B * B, axis=0)
    Q = np.zeros((M, 0))
    F = np.zeros((N, 0))
    S: list[int] = []
    r = 0
    status = "ok"
    sizes = []
    while len(S) < k and (max_rounds is None or r < max_rounds):
        words = stream(2 * b * r, 2 * b)
        props, T = draw_proposals(u, words[:b]) if np.sum(u) > 0 else (None, 0.0)
        if not T > 0:
            status = "early_stop"
            break
        kr = len(S)
        C = B[:, props] - Q @ F[props, :].T
        Tacc, _ = reject_sample_submatrix(C.T @ C, words[b:], props, cap=k - kr)
        r += 1
        sizes.append(int(Tacc.size))
        if Tacc.size == 0:
            status = "early_stop"
            break
        Si = props[Tacc]
        Qp = B[:, Si] - Q @ F[Si, :].T
        Qp = Qp - Q @ (Q.T @ Qp)
        Qp = orth(Qp)
        G = B.T @ Qp
        Q = np.hstack([Q, Qp])
        F = np.hstack([F, G])
        u = np.maximum(u - np.sum(G * G, axis=1), 0.0)
        u[Si] = 0.0
        S.extend(int(s) for s in Si)
    return QRResult(Q=Q, F=F, pivots=np.array(S, dtype=np.int64), u=u, rounds=r, status=status,
                    round_sizes=sizes)
