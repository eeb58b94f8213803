"""GPU kernel ridge regression (Section 3.2) through the C ABI against the
FP64 oracle: the solution's true residual |(A + mu I) beta - y| / |y| (dense
A on the host), PCG iteration counts equal to the oracle's run with the same
F, the factor from arpc_factor in FP64 and in the BF16 mode (FP32 storage),
and plain CG (k = 0) taking many times more iterations."""
import sys

import numpy as np
import pytest

from oracle import pcg, woodbury_apply
from oracle.kernels import kernel_block
from paper_2410_03969_amd import workloads as W

pytestmark = pytest.mark.gpu


def problem(N=3000, d=4, seed=0):
    rng = np.random.default_rng(seed)
    X = rng.random((N, d))
    y = np.sin(3 * X).sum(axis=1) + 0.01 * rng.standard_normal(N)
    return X, y, float(np.sqrt(d)), 1e-9 * N


@pytest.mark.parametrize("prec", [W.FP64, W.FP32])
def test_krr_pcg_with_rpcholesky_preconditioner(prec):
    from paper_2410_03969_amd import binding
    X, y, sigma, mu = problem()
    N = X.shape[0]
    prob = W.Problem(N=N, d=X.shape[1], k=300, b=30, kernel=W.MATERN52, sigma=sigma, seed=1, prec=prec)
    print(f"[gpu krr] N={N} prec={prec}", flush=True)
    sys.stdout.flush()
    fac = binding.factor(X, prob)
    F = fac["F"][:, : fac["stats"]["k_out"]]
    tol = 1e-8
    out = binding.krr_pcg(X, y, F, W.MATERN52, sigma, mu, tol=tol, max_iter=3000)
    beta = out["beta"].cpu().numpy()
    st = out["stats"]
    A = kernel_block(X, slice(None), slice(None), W.MATERN52, sigma)
    res = np.linalg.norm(A @ beta + mu * beta - y) / np.linalg.norm(y)
    Fh = F.to(dtype=__import__("torch").float64).cpu().numpy()
    _, it_ref, _ = pcg(lambda v: A @ v + mu * v, woodbury_apply(Fh, mu), y, tol, 3000)
    print(f"prec={prec}: iterations {st['iterations']} (oracle {it_ref}), true residual {res:.2e}, "
          f"ms {st['ms_total']:.1f}")
    assert out["status"] == 0 and st["rel_residual"] <= tol
    assert res <= 1e-6
    assert abs(st["iterations"] - it_ref) <= max(3, it_ref // 10)


def test_krr_high_dimension_and_ragged_partitions():
    """d = 40 (coordinates read from memory in the product with A, not held in
    registers) and N = 4133, whose column partitions end in a short one: the
    true residual and the oracle's PCG iteration count on the same F."""
    from paper_2410_03969_amd import binding
    X, y, sigma, mu = problem(N=4133, d=40, seed=5)
    N = X.shape[0]
    prob = W.Problem(N=N, d=40, k=250, b=25, kernel=W.MATERN52, sigma=sigma, seed=4, prec=W.FP64)
    print(f"[gpu krr] N={N} d=40", flush=True)
    sys.stdout.flush()
    fac = binding.factor(X, prob)
    F = fac["F"][:, : fac["stats"]["k_out"]]
    tol = 1e-8
    out = binding.krr_pcg(X, y, F, W.MATERN52, sigma, mu, tol=tol, max_iter=3000)
    beta = out["beta"].cpu().numpy()
    st = out["stats"]
    A = kernel_block(X, slice(None), slice(None), W.MATERN52, sigma)
    res = np.linalg.norm(A @ beta + mu * beta - y) / np.linalg.norm(y)
    _, it_ref, _ = pcg(lambda v: A @ v + mu * v, woodbury_apply(F.cpu().numpy(), mu), y, tol, 3000)
    print(f"d=40: iterations {st['iterations']} (oracle {it_ref}), true residual {res:.2e}")
    assert out["status"] == 0 and st["rel_residual"] <= tol
    assert res <= 1e-6
    assert abs(st["iterations"] - it_ref) <= max(3, it_ref // 10)


def test_krr_plain_cg_needs_many_more_iterations():
    from paper_2410_03969_amd import binding
    X, y, sigma, mu = problem(N=2000, seed=3)
    prob = W.Problem(N=2000, d=4, k=200, b=20, kernel=W.MATERN52, sigma=sigma, seed=2, prec=W.FP64)
    fac = binding.factor(X, prob)
    pre = binding.krr_pcg(X, y, fac["F"], W.MATERN52, sigma, mu, tol=1e-6, max_iter=4000)
    plain = binding.krr_pcg(X, y, None, W.MATERN52, sigma, mu, tol=1e-6, max_iter=5 * pre["stats"]["iterations"])
    print(f"preconditioned {pre['stats']['iterations']}, plain {plain['stats']['iterations']} "
          f"(residual {plain['stats']['rel_residual']:.2e})")
    assert pre["status"] == 0
    assert plain["status"] == 1 and plain["stats"]["rel_residual"] > 1e-6


def test_krr_matvec_exact_on_one_iteration():
    """With F F^* = A exactly reproduced by k = N pivots the preconditioner is
    A + mu I and PCG stops after one iteration (exact kernel products)."""
    from paper_2410_03969_amd import binding
    X, y, sigma, mu = problem(N=300, seed=4)
    mu = 1e-2
    prob = W.Problem(N=300, d=4, k=300, b=30, kernel=W.MATERN52, sigma=sigma, seed=3, prec=W.FP64)
    fac = binding.factor(X, prob)
    out = binding.krr_pcg(X, y, fac["F"], W.MATERN52, sigma, mu, tol=1e-6, max_iter=10)
    assert out["stats"]["iterations"] <= 2
    A = kernel_block(X, slice(None), slice(None), W.MATERN52, sigma)
    beta = out["beta"].cpu().numpy()
    assert np.linalg.norm(A @ beta + mu * beta - y) / np.linalg.norm(y) <= 1e-6
