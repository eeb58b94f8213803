"""Pins for oracle.kernels: distances against scipy's cdist, special values of
each kernel's formula, symmetry and positive semidefiniteness."""
import numpy as np
import pytest
from scipy.spatial.distance import cdist

from oracle.kernels import GAUSSIAN, LAPLACE_L2, MATERN32, MATERN52, kappa, kernel_block

E = np.exp(-1.0)


def test_special_values():
    s = 1.7
    # each kernel is 1 at distance 0
    for ker in (GAUSSIAN, LAPLACE_L2, MATERN32, MATERN52):
        assert kappa(np.array([0.0]), ker, s)[0] == 1.0
    # Gaussian at |x-y|^2 = 2 sigma^2 is e^-1 (Section 1.2, Gaussian kernel)
    assert np.isclose(kappa(np.array([2 * s * s]), GAUSSIAN, s)[0], E, rtol=1e-15)
    # Laplace at |x-y| = sigma is e^-1
    assert np.isclose(kappa(np.array([s * s]), LAPLACE_L2, s)[0], E, rtol=1e-15)
    # Matern-3/2 at r = l/sqrt3 is 2/e
    assert np.isclose(kappa(np.array([s * s / 3]), MATERN32, s)[0], 2 * E, rtol=1e-15)
    # Matern-5/2 (Section 3.2) at r = sigma/sqrt5 is (1 + 1 + 1/3)/e
    assert np.isclose(kappa(np.array([s * s / 5]), MATERN52, s)[0], (7 / 3) * E, rtol=1e-15)


def test_matern_smoothness_at_zero():
    # Matern-3/2 and -5/2 are flat at r = 0 (no linear term), the Laplace
    # kernel falls with slope -1/sigma: a dropped term in either formula shows here
    h = 1e-6
    assert abs((1 - kappa(np.array([h * h]), LAPLACE_L2, 1.0)[0]) / h - 1.0) < 1e-5
    for ker in (MATERN32, MATERN52):
        assert (1 - kappa(np.array([h * h]), ker, 1.0)[0]) / h < 1e-5


@pytest.mark.parametrize("ker", [GAUSSIAN, LAPLACE_L2, MATERN32, MATERN52])
def test_block_matches_cdist(ker):
    rng = np.random.default_rng(1)
    X = rng.standard_normal((60, 5))
    I = rng.integers(0, 60, 17)
    J = rng.integers(0, 60, 11)
    r2 = cdist(X[I], X[J], "sqeuclidean")
    got = kernel_block(X, I, J, ker, 1.3, chunk=7)
    assert np.allclose(got, kappa(r2, ker, 1.3), rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("ker", [GAUSSIAN, LAPLACE_L2, MATERN32, MATERN52])
def test_kernel_matrix_symmetric_psd_unit_diag(ker):
    rng = np.random.default_rng(2)
    X = rng.standard_normal((80, 3))
    A = kernel_block(X, slice(None), slice(None), ker, 0.9)
    assert np.array_equal(A, A.T)
    assert np.all(np.diag(A) == 1.0)
    assert np.linalg.eigvalsh(A).min() > -1e-10
