"""Randomly pivoted Cholesky variants, written plainly in FP64 numpy.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Every random decision reads the uniform stream of ``oracle.stream``: round r
of a block method uses words 2br..2br+b-1 for its b proposals and words
2br+b..2br+2b-1 for its b acceptance tests; iteration r of simple
RPCholesky uses word 2r (the proposal slot of a block of size one).

Readings of points where the paper is silent (each listed again in the
design notes):

* Proposal draw (Alg. 2 step 1, "sample iid from u"): proposal l is the
  smallest j with cumsum(u)_j > U_l * sum(u); an index with u_j = 0 can never
  be drawn.  If rounding pushes the target past the last partial sum, the last
  j with u_j > 0 is taken.
* Acceptance (Alg. 1): the strict test u_i * V < h_ii, where u is the diagonal
  of H before any elimination and h_ii the current Schur-complement diagonal.
  Two rules are added: a proposal equal to one already accepted in the same
  round is rejected (its exact residual is zero), and no proposal is accepted
  once k pivots are held (the experiments run until k pivots are selected,
  Section 3).
* Residual diagonal (Alg. 2 step 3): after the clamped update, the entries of
  the newly accepted pivots are set to exactly zero, which is their exact
  value; so a pivot is never proposed again.
* Stopping: the run ends early when the residual trace sum(u) is not
  positive, or when a round accepts nothing (then every proposal had a
  non-positive computed residual, i.e. the residual is numerically zero).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from scipy.linalg import cholesky, solve_triangular

from .kernels import kappa, kernel_block


# ---------------------------------------------------------------- access models
class PointsAccess:
    """Submatrix access A(I, J) to a kernel matrix built from points
    (Section 1.1, submatrix access model; Section 1.2, kernel matrices)."""

    def __init__(self, X, kernel: int, sigma: float):
        self.X = np.ascontiguousarray(X, dtype=np.float64)
        self.N = self.X.shape[0]
        self.kernel = int(kernel)
        self.sigma = float(sigma)

    def diag(self) -> np.ndarray:
        return kappa(np.zeros(self.N), self.kernel, self.sigma)

    def block(self, I, J) -> np.ndarray:
        return kernel_block(self.X, I, J, self.kernel, self.sigma)

    def columns(self, J) -> np.ndarray:
        return kernel_block(self.X, slice(None), J, self.kernel, self.sigma)


class ExpandedPointsAccess(PointsAccess):
    """The same kernel matrix as PointsAccess, with squared distances formed as
    |x|^2 + |y|^2 - 2 x.y (Appendix A.1), the dot products by one matrix
    product, clamped at zero; an entry whose row and column are the same point
    index is kappa(0) exactly.  A checker for pivot sets at sizes where direct
    differences take minutes (tens of thousands of rows against thousands of
    pivots at d = 256); its FP64 cancellation error is about
    1e-16 (|x|^2 + |y|^2) per squared distance."""

    def __init__(self, X, kernel: int, sigma: float):
        super().__init__(X, kernel, sigma)
        self.sq = np.einsum("ij,ij->i", self.X, self.X)

    def block(self, I, J) -> np.ndarray:
        I = np.arange(self.N)[I] if isinstance(I, slice) else np.asarray(I, dtype=np.int64)
        J = np.arange(self.N)[J] if isinstance(J, slice) else np.asarray(J, dtype=np.int64)
        r2 = self.sq[I][:, None] + self.sq[J][None, :] - 2.0 * (self.X[I] @ self.X[J].T)
        np.maximum(r2, 0.0, out=r2)
        out = kappa(r2, self.kernel, self.sigma)
        same = I[:, None] == J[None, :]
        out[same] = kappa(np.zeros(1), self.kernel, self.sigma)[0]
        return out

    def columns(self, J) -> np.ndarray:
        return self.block(slice(None), J)


class DenseAccess:
    """Submatrix access to an explicit psd matrix (lets tests use matrices
    whose diagonal is not constant)."""

    def __init__(self, A):
        self.A = np.asarray(A, dtype=np.float64)
        self.N = self.A.shape[0]

    def diag(self) -> np.ndarray:
        return np.diag(self.A).copy()

    def block(self, I, J) -> np.ndarray:
        return self.A[np.ix_(np.asarray(I), np.asarray(J))]

    def columns(self, J) -> np.ndarray:
        return self.A[:, np.asarray(J)]


# ------------------------------------------------------------------- results
@dataclass
class Result:
    F: np.ndarray            # N x k_out, column j belongs to pivots[j]
    pivots: np.ndarray       # int64, acceptance order
    rounds: int
    proposals: int
    status: str              # "ok" or "early_stop"
    trace_A: float
    u: np.ndarray            # final residual diagonal
    round_sizes: list = field(default_factory=list)
    u_history: list = field(default_factory=list)
    # per round: (smallest relative distance of a proposal target U*T to the
    # edges of its CDF interval, smallest |u_i V_i - h_ii| / u_i over the
    # acceptance tests); how close each random decision came to flipping
    margins: list = field(default_factory=list)

    @property
    def k_out(self) -> int:
        return int(self.pivots.size)

    @property
    def trace_error(self) -> float:
        """Relative trace error tr(A - F F^T) / tr(A) (Section 1.4)."""
        return float((self.trace_A - np.sum(self.F * self.F)) / self.trace_A)


# ------------------------------------------------------------ building blocks
def draw_proposals(u: np.ndarray, U: np.ndarray, margin=None):
    """Inverse-CDF draws from the distribution u / sum(u) (Section 2.1 proposal
    step; Alg. 2 step 1).  Returns (indices, total).  If ``margin`` is a list,
    the smallest distance of a target U*T to the edges of its interval
    [C_{s-1}, C_s), relative to the total, is appended to it."""
    C = np.cumsum(u)
    T = C[-1]
    s = np.searchsorted(C, U * T, side="right")
    if np.any(s >= u.size):
        last = np.flatnonzero(u > 0)[-1]
        s = np.where(s >= u.size, last, s)
    if margin is not None:
        t = U * T
        lo = np.where(s > 0, C[np.maximum(s - 1, 0)], 0.0)
        margin.append(float(np.min(np.minimum(np.abs(C[s] - t), np.abs(t - lo))) / T) if T > 0 else 0.0)
    return s.astype(np.int64), T


def reject_sample_submatrix(H: np.ndarray, V: np.ndarray, proposals=None, cap=None, margin=None):
    """RejectionSampleSubmatrix (Alg. 1, Section 2.2).

    H is the b x b residual submatrix at the proposals, V the b acceptance
    uniforms.  Returns (T, L): accepted local indices in order and the lower
    Cholesky factor of the original H(T, T).  If ``margin`` is a list, the
    smallest |u_i V_i - h_ii| / u_i over the tests is appended to it."""
    H = np.array(H, dtype=np.float64, copy=True)
    b = H.shape[0]
    u_loc = np.diag(H).copy()
    L = np.zeros((b, b))
    T: list[int] = []
    m = np.inf
    for i in range(b):
        if u_loc[i] > 0 and (cap is None or len(T) < cap):
            m = min(m, abs(u_loc[i] * V[i] - H[i, i]) / u_loc[i])
        accept = u_loc[i] * V[i] < H[i, i]
        if accept and cap is not None and len(T) >= cap:
            accept = False
        if accept and proposals is not None and T and proposals[i] in proposals[T]:
            accept = False
        if accept:
            T.append(i)
            L[i:, i] = H[i:, i] / np.sqrt(H[i, i])
            H[i + 1:, i + 1:] -= np.outer(L[i + 1:, i], L[i + 1:, i])
    if margin is not None:
        margin.append(float(m))
    T_arr = np.array(T, dtype=np.int64)
    return T_arr, L[np.ix_(T_arr, T_arr)]


# ------------------------------------------------------------------ algorithms
def rpc_accel(access, k: int, b: int, stream, max_rounds=None, record=False) -> Result:
    """Accelerated RPCholesky, standard (full-memory) form (Alg. 2; Section 2.3),
    run until k pivots are held (Section 3) or for max_rounds rounds."""
    N = access.N
    u = access.diag().astype(np.float64)
    trace_A = float(np.sum(u))
    F = np.zeros((N, k), order="F")
    S: list[int] = []
    r = 0
    status = "ok"
    sizes, hist, margins = [], [], []
    while len(S) < k and (max_rounds is None or r < max_rounds):
        words = stream(2 * b * r, 2 * b)
        mp, ma = [], []
        props, T = draw_proposals(u, words[:b], margin=mp) if np.sum(u) > 0 else (None, 0.0)
        if not T > 0:
            status = "early_stop"
            break
        kr = len(S)
        # step 2: residual submatrix at the proposals, then rejection sampling
        Fp = F[props, :kr]
        H = access.block(props, props) - Fp @ Fp.T
        Tacc, L = reject_sample_submatrix(H, words[b:], props, cap=k - kr, margin=ma)
        margins.append((mp[0], ma[0]))
        r += 1
        sizes.append(int(Tacc.size))
        if Tacc.size == 0:
            status = "early_stop"
            break
        Sr = props[Tacc]
        # step 3: new columns G = (A(:,S_r) - F F(S_r,:)^T) L^{-T}
        C = access.columns(Sr) - F[:, :kr] @ F[Sr, :kr].T
        G = solve_triangular(L, C.T, lower=True).T
        F[:, kr:kr + Sr.size] = G
        u = np.maximum(u - np.sum(G * G, axis=1), 0.0)
        u[Sr] = 0.0
        S.extend(int(s) for s in Sr)
        if record:
            hist.append(u.copy())
    k_out = len(S)
    return Result(F=np.asfortranarray(F[:, :k_out]), pivots=np.array(S, dtype=np.int64),
                  rounds=r, proposals=r * b, status=status, trace_A=trace_A, u=u,
                  round_sizes=sizes, u_history=hist, margins=margins)


@dataclass
class LowMemResult:
    pivots: np.ndarray     # acceptance order
    L: np.ndarray          # k_out x k_out lower Cholesky factor of A(S, S)
    u: np.ndarray          # final residual diagonal
    rounds: int
    status: str
    trace_A: float
    round_sizes: list = field(default_factory=list)


def rpc_accel_lowmem(access, k: int, b: int, stream, max_rounds=None) -> LowMemResult:
    """Accelerated RPCholesky, low-memory implementation (Alg. 3; Section 2.4):
    no N x k factor is kept; the pivots S and the Cholesky factor L of
    A(S, S) define the approximation A(:,S) L^{-*} L^{-1} A(S,:), and the
    entries A(R, S) are regenerated whenever a step needs them.  Same
    rounds, uniform words and stopping rules as rpc_accel; the diagonal
    update walks the rows in chunks of b, as printed."""
    N = access.N
    u = access.diag().astype(np.float64)
    trace_A = float(np.sum(u))
    L = np.zeros((0, 0))
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
        Sa = np.array(S, dtype=np.int64)
        # step 2: H = A(S',S') - A(S',S) L^{-*} L^{-1} A(S,S'), through Y = L^{-1} A(S,S')
        if kr:
            Y = solve_triangular(L, access.block(Sa, props), lower=True)
        else:
            Y = np.zeros((0, b))
        H = access.block(props, props) - Y.T @ Y
        Tacc, Li = reject_sample_submatrix(H, words[b:], props, cap=k - kr)
        r += 1
        sizes.append(int(Tacc.size))
        if Tacc.size == 0:
            status = "early_stop"
            break
        Si = props[Tacc]
        # step 3: W = L^{-*} L^{-1} A(S, S_i); for each chunk R of b rows,
        # G = (A(R,S_i) - A(R,S) W) L_i^{-*} and u(R) -= rowsqnorm(G)
        W = solve_triangular(L.T, Y[:, Tacc], lower=False) if kr else np.zeros((0, Tacc.size))
        for r0 in range(0, N, b):
            R = np.arange(r0, min(r0 + b, N))
            C = access.block(R, Si)
            if kr:
                C = C - access.block(R, Sa) @ W
            G = solve_triangular(Li, C.T, lower=True).T
            u[R] -= np.sum(G * G, axis=1)
        # L <- [[L, 0], [A(S_i,S) L^{-*}, L_i]], where A(S_i,S) L^{-*} = Y(:,T)^*
        Ln = np.zeros((kr + Tacc.size, kr + Tacc.size))
        Ln[:kr, :kr] = L
        Ln[kr:, :kr] = Y[:, Tacc].T
        Ln[kr:, kr:] = Li
        L = Ln
        u = np.maximum(u, 0.0)
        u[Si] = 0.0
        S.extend(int(s) for s in Si)
    return LowMemResult(pivots=np.array(S, dtype=np.int64), L=L, u=u, rounds=r, status=status,
                        trace_A=trace_A, round_sizes=sizes)


def rpc_plain(access, k: int, stream) -> Result:
    """Simple RPCholesky, one pivot per iteration (Alg. 6; Section 1.3.1).
    Iteration r reads uniform word 2r."""
    N = access.N
    u = access.diag().astype(np.float64)
    trace_A = float(np.sum(u))
    F = np.zeros((N, k), order="F")
    S: list[int] = []
    status = "ok"
    r = 0
    while len(S) < k:
        if not np.sum(u) > 0:
            status = "early_stop"
            break
        s, _ = draw_proposals(u, stream(2 * r, 1))
        s = int(s[0])
        r += 1
        i = len(S)
        g = access.columns([s])[:, 0] - F[:, :i] @ F[s, :i]
        if not g[s] > 0:
            status = "early_stop"
            break
        F[:, i] = g / np.sqrt(g[s])
        u = np.maximum(u - F[:, i] ** 2, 0.0)
        u[s] = 0.0
        S.append(s)
    return Result(F=np.asfortranarray(F[:, :len(S)]), pivots=np.array(S, dtype=np.int64),
                  rounds=r, proposals=r, status=status, trace_A=trace_A, u=u)


def rpc_block(access, k: int, b: int, stream, max_rounds=None) -> Result:
    """Block RPCholesky (Alg. 7): keep every distinct proposal.  Used only as a
    negative control; the round structure reads the same proposal words as
    the accelerated method."""
    N = access.N
    u = access.diag().astype(np.float64)
    trace_A = float(np.sum(u))
    F = np.zeros((N, k), order="F")
    S: list[int] = []
    r = 0
    status = "ok"
    while len(S) < k and (max_rounds is None or r < max_rounds):
        if not np.sum(u) > 0:
            status = "early_stop"
            break
        props, _ = draw_proposals(u, stream(2 * b * r, b))
        r += 1
        _, first = np.unique(props, return_index=True)
        Sp = props[np.sort(first)][: k - len(S)]
        kr = len(S)
        G = access.columns(Sp) - F[:, :kr] @ F[Sp, :kr].T
        L = cholesky(G[Sp, :], lower=True)
        Gn = solve_triangular(L, G.T, lower=True).T
        F[:, kr:kr + Sp.size] = Gn
        u = np.maximum(u - np.sum(Gn * Gn, axis=1), 0.0)
        u[Sp] = 0.0
        S.extend(int(s) for s in Sp)
    return Result(F=np.asfortranarray(F[:, :len(S)]), pivots=np.array(S, dtype=np.int64),
                  rounds=r, proposals=r * b, status=status, trace_A=trace_A, u=u)


# ------------------------------------------------------------------ checkers
def factor_from_pivots(access, pivots, rows=None) -> np.ndarray:
    """The factor that any pivoted partial Cholesky produces for an ordered
    pivot list: F = A(:,S) chol(A(S,S))^{-T} (Section 1.3.1 update rule,
    composed over the pivots; Section 2.4 implicit form).  ``rows`` selects
    rows of F."""
    S = np.asarray(pivots, dtype=np.int64)
    L = cholesky(access.block(S, S), lower=True)
    cols = access.columns(S) if rows is None else access.block(np.asarray(rows), S)
    return solve_triangular(L, cols.T, lower=True).T


def nystrom_err(access, pivots, rows=None, chunk: int = 8192) -> np.ndarray:
    """Residual diagonal of the Nystrom approximation A(:,S) A(S,S)^{-1} A(S,:)
    (Section 2.4), recomputed from the pivots alone: A_jj - |L^{-1} A(S,j)|^2
    for the selected rows (all rows by default).  Its sum is the trace error
    of the pivot set, independent of any stored factor."""
    S = np.asarray(pivots, dtype=np.int64)
    L = cholesky(access.block(S, S), lower=True)
    idx = np.arange(access.N) if rows is None else np.asarray(rows, dtype=np.int64)
    d = access.diag()[idx]
    out = np.empty(idx.size)
    for a in range(0, idx.size, chunk):
        blk = access.block(idx[a:a + chunk], S)
        W = solve_triangular(L, blk.T, lower=True)
        out[a:a + chunk] = d[a:a + chunk] - np.sum(W * W, axis=0)
    return out
