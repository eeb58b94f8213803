"""GPU runs of the two baselines the accelerated method is measured against,
through the C ABI, in FP64 against the oracle:
- block RPCholesky (Alg. 7, method ARPC_BLOCK): identical pivots and factor;
- simple RPCholesky (Alg. 6): the accelerated method with b = 1;
and the failure that motivates rejection sampling: on clusters of
near-duplicate points, block RPCholesky spends columns on duplicates of
clusters it already covers and leaves others uncovered."""
import numpy as np
import pytest

from oracle import PointsAccess, philox_stream, rpc_accel, rpc_block, rpc_plain
from paper_2410_03969_amd import workloads as W
from test_gpu_parity import FTOL, assert_parity, gpu_factor, oracle_run

pytestmark = pytest.mark.gpu


def oracle_block(X, prob):
    return rpc_block(PointsAccess(X, prob.kernel, prob.sigma), prob.k, prob.b, philox_stream(prob.seed))


@pytest.mark.parametrize("b", [37, 300, 600])
def test_block_method_matches_oracle(b):
    """b = 37 (register-resident tiles), 300 (tiles in L2), 600 (one proposal
    at a time): every distinct proposal kept, as in the oracle."""
    rng = np.random.default_rng(b)
    X = rng.standard_normal((5003, 5))
    prob = W.Problem(N=5003, d=5, k=2 * b + 13, b=b, kernel=W.LAPLACE_L2, sigma=1.5, seed=b,
                     method=W.BLOCK)
    F, piv, out = gpu_factor(X, prob)
    assert_parity(F, piv, out, oracle_block(X, prob))


def test_block_size_one_is_simple_rpcholesky():
    rng = np.random.default_rng(7)
    X = rng.random((3000, 3))
    prob = W.Problem(N=3000, d=3, k=60, b=1, kernel=W.MATERN52, sigma=0.4, seed=7)
    F, piv, out = gpu_factor(X, prob)
    ref = rpc_plain(PointsAccess(X, prob.kernel, prob.sigma), prob.k, philox_stream(prob.seed))
    assert np.array_equal(piv, ref.pivots)
    err = np.linalg.norm(F - ref.F) / np.linalg.norm(ref.F)
    assert err <= FTOL, err


def clustered(nc=40, m=100, eps=0.05, d=5, seed=1):
    rng = np.random.default_rng(seed)
    centers = 20.0 * rng.standard_normal((nc, d))
    labels = rng.integers(0, nc, size=nc * m)
    return centers[labels] + eps * rng.standard_normal((nc * m, d)), labels


def test_block_method_wastes_columns_on_near_duplicates():
    X, labels = clustered()
    base = W.Problem(N=X.shape[0], d=5, k=60, b=40, kernel=W.GAUSSIAN, sigma=1.0, seed=1)
    Fa, pa, oa = gpu_factor(X, base)
    assert_parity(Fa, pa, oa, oracle_run(X, base))
    blk = base.with_(method=W.BLOCK)
    Fb, pb, ob = gpu_factor(X, blk)
    assert_parity(Fb, pb, ob, oracle_block(X, blk))
    trA = oa["stats"]["trace_A"]
    te_a = (trA - np.sum(Fa ** 2)) / trA
    te_b = (trA - np.sum(Fb ** 2)) / trA
    cov_a, cov_b = len(set(labels[pa].tolist())), len(set(labels[pb].tolist()))
    print(f"clusters covered: accelerated {cov_a}, block {cov_b}; trace error {te_a:.4e} vs {te_b:.4e}")
    assert cov_a == 40 and cov_b < 40
    assert te_b > 3 * te_a


@pytest.mark.parametrize("b,method", [(1, W.ACCEL), (50, W.BLOCK)])
def test_bf16_round_kernel_baselines(b, method):
    """The BF16 one-kernel round with one proposal per round (simple
    RPCholesky) and with block RPCholesky: the factor equals the FP64 factor
    of the pivots chosen, to BF16 accuracy."""
    from oracle import factor_from_pivots
    rng = np.random.default_rng(100 + b)
    N = 6151
    X = rng.uniform(0.0, 1.0, size=(N, 3))
    prob = W.Problem(N=N, d=3, k=120, b=b, kernel=W.LAPLACE_L2, sigma=0.5, seed=b, prec=W.BF16, method=method)
    F, piv, out = gpu_factor(X, prob)
    assert out["stats"]["fused"] == 1
    k_out = out["stats"]["k_out"]
    assert k_out == prob.k and len(set(piv.tolist())) == k_out
    rows = np.concatenate([rng.choice(N, 150, replace=False), np.arange(N - 20, N)])
    ref = factor_from_pivots(PointsAccess(X, prob.kernel, prob.sigma), piv, rows=rows)
    err = np.linalg.norm(F[rows] - ref) / np.linalg.norm(ref)
    print(f"bf16 b={b} method={method}: relF {err:.3e}")
    assert err < 5e-2, err
