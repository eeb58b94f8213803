"""Pins for the oracle's RPCholesky algorithms against what the paper and the
mathematics fix: closed forms, invariants, special cases that reduce to
textbook routines, brute-force laws on tiny inputs and the central error bound.
"""
import math

import numpy as np
import pytest
from scipy.linalg import cholesky
from scipy.stats import chisquare

from oracle import (DenseAccess, PointsAccess, array_stream, draw_proposals,
                    factor_from_pivots, nystrom_err, philox_stream, reject_sample_submatrix,
                    rpc_accel, rpc_block, rpc_plain)
from oracle.kernels import GAUSSIAN, LAPLACE_L2, MATERN32
from paper_2410_03969_amd import workloads as W


# ------------------------------------------------------------------ proposals
def test_draw_matches_brute_force_definition():
    """Proposal l is the smallest j whose running sum exceeds U*total."""
    rng = np.random.default_rng(0)
    u = rng.random(37)
    u[[3, 4, 20]] = 0.0
    U = rng.random(200)
    s, T = draw_proposals(u, U)
    for Ul, sl in zip(U, s):
        run, pick = 0.0, None
        for j, w in enumerate(u):
            run += w
            if run > Ul * T:
                pick = j
                break
        assert pick == sl
    assert not np.isin(s, [3, 4, 20]).any()


def test_draw_frequencies_follow_weights():
    """Empirical frequencies of 2e5 draws match u / sum(u) (chi-square)."""
    u = np.array([0.5, 2.0, 0.0, 1.0, 3.5, 0.25, 1.75, 1.0])
    U = philox_stream(11)(0, 200_000)
    s, _ = draw_proposals(u, U)
    counts = np.bincount(s, minlength=u.size)
    assert counts[2] == 0
    nz = u > 0
    assert chisquare(counts[nz], U.size * u[nz] / u.sum()).pvalue > 1e-3


def test_draw_rounding_fallback_picks_last_positive():
    u = np.array([0.3, 0.7, 0.0, 0.0])
    s, _ = draw_proposals(u, np.array([1.0]))   # U = 1 is outside the stream's range
    assert s[0] == 1


# ------------------------------------------------------ rejection sampling step
def _psd(n, r, seed):
    return W.dense_psd(n, r, seed)


def test_reject_sample_L_is_cholesky_of_accepted_block():
    rng = np.random.default_rng(3)
    for trial in range(20):
        H = _psd(9, 9, trial)
        V = rng.random(9)
        T, L = reject_sample_submatrix(H, V)
        assert T[0] == 0                                   # first proposal always accepted
        assert np.allclose(L, np.linalg.cholesky(H[np.ix_(T, T)]), rtol=1e-12, atol=1e-12)


def test_reject_sample_zero_uniforms_accept_every_independent_proposal():
    # with V = 0 the test is h_ii > 0: a full-rank H accepts everything
    H = _psd(6, 6, 1)
    T, L = reject_sample_submatrix(H, np.zeros(6))
    assert list(T) == list(range(6))
    assert np.allclose(L, cholesky(H, lower=True), rtol=1e-12)


def test_reject_sample_rank_deficient_rejects_dependent_proposals():
    # rank-2 H: after two acceptances every residual diagonal is zero up to
    # rounding, far below u_i * V for V = 1e-3
    H = _psd(6, 2, 5)
    T, _ = reject_sample_submatrix(H, np.full(6, 1e-3))
    assert len(T) == 2


def test_reject_sample_duplicate_and_cap_rules():
    H = np.ones((3, 3))                       # three copies of the same index
    T, L = reject_sample_submatrix(H, np.zeros(3), proposals=np.array([4, 4, 4]))
    assert list(T) == [0] and L[0, 0] == 1.0
    T, _ = reject_sample_submatrix(np.eye(4), np.zeros(4), cap=2)
    assert list(T) == [0, 1]


def test_acceptance_probability_is_schur_ratio():
    """Alg. 1 accepts proposal 2 of 2 with probability
    (h22 - h12^2/h11) / h22 (Section 1.3.3, rejection step)."""
    H = np.array([[2.0, 1.2], [1.2, 1.5]])
    p = (1.5 - 1.2 ** 2 / 2.0) / 1.5
    V = np.linspace(0, 1, 2001, endpoint=False)
    acc = [len(reject_sample_submatrix(H, np.array([0.5, v]))[0]) == 2 for v in V]
    assert abs(np.mean(acc) - p) < 1e-3


# ------------------------------------------------------------- residual matrix
def test_H_is_schur_complement():
    """H = A(S',S') - F(S',:) F(S',:)^T equals the Schur complement
    A(S',S') - A(S',S) A(S,S)^{-1} A(S,S') (Alg. 2 step 2)."""
    rng = np.random.default_rng(4)
    X = rng.standard_normal((300, 3))
    acc = PointsAccess(X, GAUSSIAN, 1.0)
    res = rpc_accel(acc, k=25, b=8, stream=philox_stream(1))
    S = res.pivots
    P = rng.integers(0, 300, 10)
    H = acc.block(P, P) - res.F[P] @ res.F[P].T
    schur = acc.block(P, P) - acc.block(P, S) @ np.linalg.solve(acc.block(S, S), acc.block(S, P))
    assert np.allclose(H, schur, atol=1e-10)


@pytest.mark.parametrize("ker", [GAUSSIAN, LAPLACE_L2, MATERN32])
def test_factor_is_function_of_pivots_and_interpolates(ker):
    """F = A(:,S) chol(A(S,S))^{-T} in pivot order, and F F^T reproduces A
    exactly on the pivot rows (Nystrom interpolation, Section 2.4)."""
    rng = np.random.default_rng(5)
    X = rng.standard_normal((500, 4))
    acc = PointsAccess(X, ker, 1.5)
    res = rpc_accel(acc, k=40, b=10, stream=philox_stream(2))
    assert res.k_out == 40
    ref = factor_from_pivots(acc, res.pivots)
    assert np.linalg.norm(res.F - ref) / np.linalg.norm(ref) < 1e-10
    S = res.pivots
    assert np.allclose(res.F[S] @ res.F.T, acc.block(S, np.arange(500)), atol=1e-10)


def test_residual_diagonal_invariants():
    """u is the diagonal of A - F F^T, nonnegative, elementwise nonincreasing,
    and exactly zero at every pivot (Alg. 2 step 3)."""
    rng = np.random.default_rng(6)
    X = rng.standard_normal((400, 2))
    acc = PointsAccess(X, GAUSSIAN, 0.7)
    res = rpc_accel(acc, k=60, b=12, stream=philox_stream(3), record=True)
    prev = acc.diag()
    for u in res.u_history:
        assert np.all(u >= 0) and np.all(u <= prev)
        prev = u
    assert np.allclose(res.u, acc.diag() - np.sum(res.F ** 2, axis=1), atol=1e-12)
    assert np.all(res.u[res.pivots] == 0.0)


def test_trace_error_equals_nystrom_error():
    rng = np.random.default_rng(7)
    X = rng.standard_normal((600, 3))
    acc = PointsAccess(X, LAPLACE_L2, 1.0)
    res = rpc_accel(acc, k=50, b=10, stream=philox_stream(4))
    ny = nystrom_err(acc, res.pivots).sum() / res.trace_A
    assert abs(res.trace_error - ny) < 1e-12


def test_rank_bounds_per_round():
    """t <= k <= b t after t rounds (Section 2.3)."""
    rng = np.random.default_rng(8)
    acc = PointsAccess(rng.standard_normal((500, 5)), GAUSSIAN, 1.0)
    for t in (1, 2, 5):
        res = rpc_accel(acc, k=500, b=7, stream=philox_stream(t), max_rounds=t)
        assert t <= res.k_out <= 7 * t
        assert all(s >= 1 for s in res.round_sizes)


# -------------------------------------------------------------- special cases
def test_block_size_one_is_simple_rpcholesky():
    """With b = 1 the accelerated method is simple RPCholesky (Alg. 6) on the
    same stream: identical pivots, same factor."""
    rng = np.random.default_rng(9)
    acc = PointsAccess(rng.standard_normal((700, 3)), GAUSSIAN, 0.8)
    for seed in range(3):
        a = rpc_accel(acc, k=60, b=1, stream=philox_stream(seed))
        p = rpc_plain(acc, k=60, stream=philox_stream(seed))
        assert np.array_equal(a.pivots, p.pivots)
        assert np.linalg.norm(a.F - p.F) / np.linalg.norm(p.F) < 1e-13


def simulate_identity(N, k, b, stream):
    """A = I: proposals are uniform over the indices not yet pivoted; the
    accepted set is the distinct proposals in order, capped at k."""
    remaining = list(range(N))
    piv = []
    r = 0
    while len(piv) < k and remaining:
        U = stream(2 * b * r, 2 * b)[:b]
        T = float(len(remaining))
        props = [remaining[int(math.floor(x * T))] for x in U]
        for p in props:
            if len(piv) < k and p in remaining:   # duplicates of this round are gone
                piv.append(p)
                remaining.remove(p)
        r += 1
    return piv


@pytest.mark.parametrize("b", [1, 5, 16])
def test_identity_matrix_pivots_exact(b):
    X = W.grid(3)                       # 64 points, Gaussian sigma=1 -> A = I exactly
    acc = PointsAccess(X, GAUSSIAN, 1.0)
    assert np.array_equal(acc.block(np.arange(64), np.arange(64)), np.eye(64))
    res = rpc_accel(acc, k=40, b=b, stream=philox_stream(21))
    assert list(res.pivots) == simulate_identity(64, 40, b, philox_stream(21))
    assert np.array_equal(res.F, np.eye(64)[:, res.pivots])


def test_cluster_matrix_exact_recovery():
    """A block-diagonal all-ones matrix of rank r is recovered exactly with r
    pivots, one per group, and the run stops early (zero residual)."""
    sizes = [50, 7, 130, 1, 22]
    X, labels = W.clusters(sizes, d=3, seed=3)
    acc = PointsAccess(X, GAUSSIAN, 1.0)
    res = rpc_accel(acc, k=20, b=6, stream=philox_stream(5))
    assert res.status == "early_stop" and res.k_out == len(sizes)
    assert sorted(labels[res.pivots]) == list(range(len(sizes)))
    A = acc.block(np.arange(len(X)), np.arange(len(X)))
    assert np.array_equal(res.F @ res.F.T, A)
    assert res.trace_error == 0.0 and np.all(res.u == 0.0)


# ---------------------------------------------------------------- random laws
def test_first_pivot_law():
    """P{s_1 = j} = A_jj / tr A (Section 1.3.1, first-step law), checked on a
    matrix with an uneven diagonal over 20000 seeded runs."""
    A = W.dense_psd(5, 5, seed=1)
    acc = DenseAccess(A)
    M = 20000
    counts = np.zeros(5)
    for seed in range(M):
        counts[rpc_accel(acc, k=1, b=3, stream=philox_stream(seed)).pivots[0]] += 1
    p = np.diag(A) / np.trace(A)
    assert chisquare(counts, M * p).pvalue > 1e-3


def rpc_sequence_law(A, m):
    """Exact law of the first m pivots of simple RPCholesky: the product of
    residual-diagonal ratios (Section 1.3.1), with residuals formed by the
    Schur complement through numpy.linalg.solve."""
    N = A.shape[0]
    law = {}

    def rec(seq, prob):
        if len(seq) == m:
            law[tuple(seq)] = prob
            return
        if seq:
            S = np.array(seq)
            R = A - A[:, S] @ np.linalg.solve(A[np.ix_(S, S)], A[S, :])
        else:
            R = A
        d = np.clip(np.diag(R), 0, None)
        d[seq] = 0
        for j in range(N):
            if d[j] > 1e-14 * d.sum():
                rec(seq + [j], prob * d[j] / d.sum())

    rec([], 1.0)
    return law


def _chi2_against(law, samples):
    keys = list(law)
    idx = {k: i for i, k in enumerate(keys)}
    obs = np.zeros(len(keys))
    other = 0
    for s in samples:
        if s in idx:
            obs[idx[s]] += 1
        else:
            other += 1
    exp = np.array([law[k] for k in keys]) * len(samples)
    big = exp >= 5
    o = np.append(obs[big], obs[~big].sum() + other)
    e = np.append(exp[big], exp[~big].sum() + 1e-12)
    if e[-1] < 5:
        o[-2] += o[-1]
        e[-2] += e[-1]
        o, e = o[:-1], e[:-1]
    return chisquare(o, e * o.sum() / e.sum()).pvalue


def _near_duplicate_matrix():
    X = np.array([[0.0, 0.0], [0.05, 0.0], [1.3, 0.2], [0.4, 1.1], [2.0, 1.5], [0.9, 0.7]])
    return PointsAccess(X, GAUSSIAN, 1.0).block(np.arange(6), np.arange(6))


@pytest.mark.parametrize("b", [2, 3, 5])
def test_accepted_sequence_has_rpcholesky_law(b):
    """Accepted pivots of the accelerated method follow the simple
    RPCholesky law (Section 2.2, last paragraph): ordered triples on N = 6,
    exact law by enumeration, 12000 seeded runs."""
    A = _near_duplicate_matrix()
    acc = DenseAccess(A)
    law = rpc_sequence_law(A, 3)
    samples = [tuple(rpc_accel(acc, k=3, b=b, stream=philox_stream(s)).pivots)
               for s in range(12000)]
    assert _chi2_against(law, samples) > 1e-3


def test_block_rpcholesky_fails_the_law():
    """Negative control: keeping every proposal (Alg. 7) does not produce the
    RPCholesky law on a matrix with two nearly equal columns."""
    A = _near_duplicate_matrix()
    acc = DenseAccess(A)
    law = rpc_sequence_law(A, 2)
    samples = [tuple(rpc_block(acc, k=2, b=2, stream=philox_stream(s)).pivots)
               for s in range(6000)]
    samples = [s for s in samples if len(s) == 2]
    assert _chi2_against(law, samples) < 1e-6


def test_expected_residual_identity():
    """Averaging the one-pivot residual over the first-pivot law gives
    A - A^2 / tr A (Section 4.1, expected residual function)."""
    A = W.dense_psd(6, 6, seed=2)
    acc = DenseAccess(A)
    d = np.diag(A)
    C = np.cumsum(d)
    avg = np.zeros_like(A)
    for j in range(6):
        # a uniform that lands inside index j's interval of the CDF
        lo = C[j - 1] if j else 0.0
        U = np.array([(lo + 0.5 * d[j]) / C[-1], 0.0])
        res = rpc_accel(acc, k=1, b=1, stream=array_stream(U))
        assert res.pivots[0] == j
        avg += d[j] / np.trace(A) * (A - res.F @ res.F.T)
    assert np.allclose(avg, A - A @ A / np.trace(A), atol=1e-12)


def test_central_error_bound():
    """Mean residual trace after t full rounds is at most tr Phi_b^(t)(A),
    the scalar map x -> x - x^2/alpha applied b times per round to the
    eigenvalues with alpha the trace at the round start (Section 4, central
    error bound)."""
    rng = np.random.default_rng(10)
    Q, _ = np.linalg.qr(rng.standard_normal((40, 40)))
    lam = 0.7 ** np.arange(40)
    A = (Q * lam) @ Q.T
    A = (A + A.T) / 2
    b, t = 4, 3
    x = lam.copy()
    for _ in range(t):
        alpha = x.sum()
        for _ in range(b):
            x = x - x * x / alpha
    bound = x.sum()
    acc = DenseAccess(A)
    M = 1500
    tr = np.array([np.trace(A) - np.sum(rpc_accel(acc, k=40, b=b, stream=philox_stream(s),
                                                   max_rounds=t).F ** 2) for s in range(M)])
    assert tr.mean() <= bound + 3 * tr.std() / np.sqrt(M)
    # a run that rejected everything after the first pivot of each round would
    # sit far above the bound; the accelerated method is well inside it
    assert tr.mean() < bound


# --------------------------------------------------- checkers used at scale
@pytest.mark.parametrize("ker,d", [(GAUSSIAN, 8), (LAPLACE_L2, 20), (MATERN32, 256)])
def test_expanded_access_equals_direct_differences(ker, d):
    """The expansion |x|^2 + |y|^2 - 2 x.y gives the direct-difference kernel
    block to FP64 cancellation accuracy, with exact kappa(0) on repeated
    indices; the Nystrom error of a pivot set agrees to 1e-9 relative."""
    from oracle import ExpandedPointsAccess
    rng = np.random.default_rng(d)
    if d == 256:
        X = np.where(rng.random((3000, d)) < 0.1, rng.standard_normal((3000, d)), 0.0)
        sigma = 4.0
    else:
        X = rng.standard_normal((3000, d))
        sigma = 2.0
    a, e = PointsAccess(X, ker, sigma), ExpandedPointsAccess(X, ker, sigma)
    I = rng.choice(3000, 400, replace=False)
    J = np.concatenate([I[:50], rng.choice(3000, 150, replace=False)])
    Bd, Be = a.block(I, J), e.block(I, J)
    assert np.max(np.abs(Bd - Be)) < 1e-6 if ker != GAUSSIAN else np.max(np.abs(Bd - Be)) < 1e-12
    assert np.all(Be[np.arange(50), np.arange(50)] == 1.0)
    res = rpc_accel(a, k=150, b=30, stream=philox_stream(1))
    rows = rng.choice(3000, 1000, replace=False)
    nd = nystrom_err(a, res.pivots, rows=rows).sum()
    ne = nystrom_err(e, res.pivots, rows=rows).sum()
    assert abs(nd - ne) <= 1e-9 * nd


def test_decision_margins():
    """The proposal margin is the distance of U*T to the nearest edge of the
    drawn index's CDF interval over T; the acceptance margin is
    |u_i V_i - h_ii| / u_i, smallest over the round's tests."""
    u = np.array([1.0, 2.0, 1.0])                    # C = 1, 3, 4; T = 4
    m = []
    draw_proposals(u, np.array([0.5, 0.24]), margin=m)  # targets 2.0 (in [1,3)), 0.96 (in [0,1))
    assert m[0] == pytest.approx(min(1.0, 1.0, 0.04, 0.96) / 4.0)
    H = np.array([[2.0, 1.0], [1.0, 2.0]])
    ma = []
    T, _ = reject_sample_submatrix(H, np.array([0.25, 0.5]), margin=ma)
    # test 0: |2*0.25 - 2| / 2 = 0.75; test 1 after the update: h = 1.5, |2*0.5 - 1.5| / 2 = 0.25
    assert list(T) == [0, 1] and ma[0] == pytest.approx(0.25)
    res = rpc_accel(PointsAccess(np.random.default_rng(0).random((200, 2)), GAUSSIAN, 0.3), k=20, b=5,
                    stream=philox_stream(0))
    assert len(res.margins) == res.rounds and all(p >= 0 and a >= 0 for p, a in res.margins)
