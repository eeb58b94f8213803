"""Kernel functions, evaluated by direct differences in FP64.

Section 1.2 defines the Gaussian kernel exp(-|x-y|^2 / (2 sigma^2)).  The
Laplace kernel here uses the l2 distance, exp(-|x-y| / sigma) (the paper's
printed Laplace kernel sums absolute coordinate differences; the l2 form is
the one that a squared-distance evaluation supports).  The Matern-5/2 kernel
is the one printed in Section 3.2; the Matern-3/2 kernel, named in Section 3.1
without a formula, is taken in its standard form (1 + sqrt3 r/l) exp(-sqrt3 r/l).

Distances are formed by subtracting coordinates and summing squares, the way
the paper's block-RPCholesky experiments compute them (Appendix A.1), so a
point paired with itself gives distance exactly 0 and kernel value exactly 1.
"""
from __future__ import annotations

import numpy as np

GAUSSIAN, LAPLACE_L2, MATERN32, MATERN52 = 0, 1, 2, 3


def kappa(r2: np.ndarray, kernel: int, sigma: float) -> np.ndarray:
    """Kernel value as a function of the squared distance r2."""
    r2 = np.asarray(r2, dtype=np.float64)
    if kernel == GAUSSIAN:
        return np.exp(-r2 / (2.0 * sigma * sigma))
    r = np.sqrt(r2)
    if kernel == LAPLACE_L2:
        return np.exp(-r / sigma)
    if kernel == MATERN32:
        t = np.sqrt(3.0) * r / sigma
        return (1.0 + t) * np.exp(-t)
    if kernel == MATERN52:
        t = np.sqrt(5.0) * r / sigma
        return (1.0 + t + (5.0 / 3.0) * r2 / (sigma * sigma)) * np.exp(-t)
    raise ValueError(f"unknown kernel {kernel}")


def kernel_block(X: np.ndarray, I, J, kernel: int, sigma: float,
                 chunk: int = 4096) -> np.ndarray:
    """A(I, J) = [kappa(x_i, x_j)] for rows I and columns J (index arrays or
    slices), by direct differences, row chunk by row chunk."""
    XI = X[I]
    XJ = X[J]
    out = np.empty((XI.shape[0], XJ.shape[0]), dtype=np.float64)
    for a in range(0, XI.shape[0], chunk):
        diff = XI[a:a + chunk, None, :] - XJ[None, :, :]
        r2 = np.einsum("ijk,ijk->ij", diff, diff)
        out[a:a + chunk] = kappa(r2, kernel, sigma)
    return out
