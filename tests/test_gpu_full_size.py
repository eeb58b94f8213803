"""GPU runs at the full sizes of the mixture workload (N = 1e6, d = 8, k = 2000,
b = 200, the configuration bench.py times) and of the sparse high-dimensional
workload (N = 2e5, d = 256, k = 4000, b = 400), through the C ABI.

At these sizes the factor stays on the device.  Checks:
- valid, distinct pivots and the full rank k;
- sampled rows of F against the FP64 oracle's factor of the same pivots
  (F = A(:,S) chol(A(S,S))^{-T}, computed one row at a time on the host);
- properties that hold at any size: |F|_F^2 <= tr A, and the trace error of a
  reduced-precision run within 1.05x of the FP64 run's (mixture workload);
- the FP8 mode against the oracle's factor of the e4m3-rounded points.
"""
import sys

import numpy as np
import pytest

from oracle import PointsAccess, factor_from_pivots, round_e4m3
from paper_2410_03969_amd import workloads as W

pytestmark = pytest.mark.gpu


def _run(X, prob):
    from paper_2410_03969_amd import binding
    print(f"[gpu full size] N={prob.N} d={prob.d} k={prob.k} b={prob.b} kernel={prob.kernel} "
          f"prec={prob.prec}", flush=True)
    sys.stdout.flush()
    return binding.factor(X, prob)


def _norm2(F, k_out, chunk=256):
    """|F(:, :k_out)|_F^2 in FP64, a block of columns at a time."""
    import torch
    tot = 0.0
    for j in range(0, k_out, chunk):
        tot += float((F[:, j:j + chunk].to(torch.float64) ** 2).sum().item())
    return tot


def _check(X, prob, out, rows, ncols, tol):
    """prob: the problem of the run (its precision is printed)."""
    k_out = out["stats"]["k_out"]
    piv = out["pivots"].cpu().numpy()
    assert out["status"] == 0 and k_out == prob.k
    assert np.all((piv >= 0) & (piv < prob.N)) and len(set(piv.tolist())) == prob.k
    trA = out["stats"]["trace_A"]
    n2 = _norm2(out["F"], k_out)
    assert n2 <= trA * (1 + 1e-3)
    import torch
    Fs = out["F"][torch.as_tensor(rows, device=out["F"].device), :ncols].to(torch.float64).cpu().numpy()
    ref = factor_from_pivots(PointsAccess(X, prob.kernel, prob.sigma), piv[:ncols], rows=rows)
    err = np.linalg.norm(Fs - ref) / np.linalg.norm(ref)
    te = (trA - n2) / trA
    print(f"  prec={prob.prec} sampled relF={err:.3e} trace error={te:.6e}", flush=True)
    assert err < tol, err
    return te


def _rows(N, seed):
    return np.concatenate([np.random.default_rng(seed).choice(N, 200, replace=False), np.arange(N - 8, N)])


def test_mixture_full_size_bf16_against_fp64():
    X, prob = W.mixture()
    rows = _rows(prob.N, 1)
    out = _run(X, prob.with_(prec=W.BF16))
    assert out["stats"]["fused"] == 1            # the round kernel bench.py times
    te = _check(X, prob.with_(prec=W.BF16), out, rows, 2 * prob.b, 5e-2)
    del out
    out64 = _run(X, prob.with_(prec=W.FP64))
    te64 = _check(X, prob.with_(prec=W.FP64), out64, rows, 2 * prob.b, 1e-9)
    print(f"  trace error ratio bf16 / fp64 = {te / te64:.5f}", flush=True)
    assert te <= 1.05 * te64


def test_sparse_high_dim_full_size():
    X, prob = W.sparse_hd()
    rows = _rows(prob.N, 2)
    out64 = _run(X, prob.with_(prec=W.FP64))
    te64 = _check(X, prob.with_(prec=W.FP64), out64, rows, 2 * prob.b, 1e-9)
    del out64
    out = _run(X, prob.with_(prec=W.BF16X3))
    te = _check(X, prob.with_(prec=W.BF16X3), out, rows, 2 * prob.b, 2e-3)
    print(f"  trace error ratio bf16x3 / fp64 = {te / te64:.5f}", flush=True)
    del out
    # FP8 mode: the factor of the e4m3-rounded points (its own oracle), and the
    # trace error that rounding costs against the FP64 run
    out8 = _run(X, prob.with_(prec=W.FP8))
    te8 = _check(round_e4m3(X), prob.with_(prec=W.FP8), out8, rows, 2 * prob.b, 5e-2)
    print(f"  trace error ratio fp8 / fp64 = {te8 / te64:.5f}", flush=True)
