"""GPU parity of accelerated randomly pivoted QR (Alg. 5) through the C ABI
against the FP64 oracle: identical pivots, Q and F entry by entry (Orth is
the QR factorization with a positive diagonal in R on both sides; the GPU
forms it by Cholesky QR, the oracle by Householder QR), Q orthonormal."""
import sys

import numpy as np
import pytest

from oracle import philox_stream, rpqr_accel

pytestmark = pytest.mark.gpu


def matrix(M, N, rank, decay, seed, noise=1e-3):
    rng = np.random.default_rng(seed)
    U = np.linalg.qr(rng.standard_normal((M, rank)))[0]
    V = np.linalg.qr(rng.standard_normal((N, rank)))[0]
    return (U * decay ** np.arange(rank)) @ V.T + noise * rng.standard_normal((M, N))


def graded(M, N, seed):
    rng = np.random.default_rng(seed)
    U = np.linalg.qr(rng.standard_normal((M, 60)))[0]
    V = np.linalg.qr(rng.standard_normal((N, 60)))[0]
    return (U * np.logspace(0, -12, 60)) @ V.T


def run(B, k, b, seed, max_rounds=0):
    from paper_2410_03969_amd import binding
    print(f"[gpu rpqr] M={B.shape[0]} N={B.shape[1]} k={k} b={b} seed={seed}", flush=True)
    sys.stdout.flush()
    out = binding.qr_factor(B, k, b, seed=seed, max_rounds=max_rounds)
    k_out = out["stats"]["k_out"]
    return (out["Q"].cpu().numpy()[:, :k_out], out["F"].cpu().numpy()[:, :k_out], out["pivots"].cpu().numpy(), out)


CASES = [
    ("lowrank_noise", lambda: matrix(300, 500, 80, 0.93, 0), 60, 16, 0),
    ("wide_ragged", lambda: matrix(120, 700, 80, 0.93, 1), 90, 37, 1),
    ("tall_b1", lambda: matrix(400, 200, 80, 0.93, 2), 30, 1, 2),
    ("graded", lambda: graded(300, 400, 0), 30, 10, 1),
    ("full_rank", lambda: np.random.default_rng(5).standard_normal((30, 200)), 30, 8, 3),
    ("larger", lambda: matrix(1000, 3000, 400, 0.99, 4), 300, 100, 4),
]


@pytest.mark.parametrize("name,make,k,b,seed", CASES)
def test_rpqr_against_oracle(name, make, k, b, seed):
    B = make()
    Q, F, piv, out = run(B, k, b, seed)
    ref = rpqr_accel(B, k, b, philox_stream(seed))
    k_out = out["stats"]["k_out"]
    assert k_out == len(ref.pivots)
    assert np.array_equal(piv[:k_out], ref.pivots)
    assert np.all(piv[k_out:] == -1)
    eq = np.linalg.norm(Q - ref.Q) / np.linalg.norm(ref.Q)
    ef = np.linalg.norm(F - ref.F) / np.linalg.norm(ref.F)
    orth = np.max(np.abs(Q.T @ Q - np.eye(k_out)))
    print(f"{name}: relQ={eq:.2e} relF={ef:.2e} orth={orth:.2e} rounds={out['stats']['rounds']}")
    assert eq <= 1e-8 and ef <= 1e-8 and orth <= 1e-10
    st = out["stats"]
    assert abs(st["trace_A"] - np.sum(B * B)) <= 1e-12 * np.sum(B * B)
    assert abs(st["trace_resid"] - np.sum(ref.u)) <= 1e-9 * st["trace_A"]


def test_rpqr_exhausted_columns_stop_early():
    """Five nonzero columns: after them every residual norm is exactly zero."""
    rng = np.random.default_rng(9)
    B = np.zeros((50, 400))
    cols = rng.choice(400, 5, replace=False)
    B[:, cols] = rng.standard_normal((50, 5))
    Q, F, piv, out = run(B, 20, 4, 7)
    assert out["status"] == 1 and out["stats"]["k_out"] == 5
    assert sorted(piv[:5].tolist()) == sorted(cols.tolist()) and np.all(piv[5:] == -1)
    assert np.allclose(Q @ F.T, B, atol=1e-12 * np.linalg.norm(B))
