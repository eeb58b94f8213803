"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs and the same uniform stream.

Bar: in FP64 mode the pivot sequence is identical and
|F_gpu - F_oracle|_F / |F_oracle|_F <= 1e-10.  The identity and cluster
matrices are exact in every precision, so they are compared bit for bit.
"""
import math
import sys

import numpy as np
import pytest

from oracle import (PointsAccess, array_stream, factor_from_pivots, philox_stream,
                    round_e4m3, rpc_accel)
from paper_2410_03969_amd import workloads as W

pytestmark = pytest.mark.gpu

FTOL = 1e-10


def gpu_factor(X, prob, U=None):
    from paper_2410_03969_amd import binding
    print(f"[gpu] N={prob.N} d={prob.d} k={prob.k} b={prob.b} kernel={prob.kernel} "
          f"prec={prob.prec} seed={prob.seed} max_rounds={prob.max_rounds}",
          flush=True)
    sys.stdout.flush()
    out = binding.factor(X, prob, U=U)
    k_out = out["stats"]["k_out"]
    F = out["F"].cpu().numpy()[:, :k_out].astype(np.float64)
    piv = out["pivots"].cpu().numpy()
    return F, piv, out


def oracle_run(X, prob, max_rounds=None, U=None):
    stream = philox_stream(prob.seed) if U is None else array_stream(U)
    return rpc_accel(PointsAccess(X, prob.kernel, prob.sigma), prob.k, prob.b, stream,
                     max_rounds=max_rounds)


TIE = 1e-12   # a decision this close to its threshold may flip on rounding alone


def assert_parity(F, piv, out, ref, ftol=FTOL):
    """Identical pivots and F within ftol (relative Frobenius).  Prints the
    oracle's decision margins (how close each round's draws and acceptance
    tests came to flipping) and the largest column-wise relative error; a
    pivot mismatch in a round whose margin is below TIE is reported as a tie."""
    k = ref.k_out
    assert out["stats"]["k_out"] == k
    mp = min((m[0] for m in ref.margins), default=np.inf)
    ma = min((m[1] for m in ref.margins), default=np.inf)
    first_diff = np.flatnonzero(piv[:k] != ref.pivots)
    if first_diff.size:
        j = int(first_diff[0])
        rnd = int(np.searchsorted(np.cumsum(ref.round_sizes), j, side="right"))
        m = ref.margins[min(rnd, len(ref.margins) - 1)]
        kind = "TIE (margin below 1e-12)" if min(m) < TIE else "not a tie"
        raise AssertionError(f"pivots differ first at {j} (round {rnd}, margins {m[0]:.2e} / {m[1]:.2e}: {kind})")
    assert np.all(piv[k:] == -1)
    nref = np.linalg.norm(ref.F, axis=0)
    colerr = np.linalg.norm(F - ref.F, axis=0) / np.maximum(nref, 1e-300)
    err = np.linalg.norm(F - ref.F) / max(np.linalg.norm(ref.F), 1e-300)
    print(f"  parity: relF {err:.3e}, worst column {colerr.max() if colerr.size else 0:.3e}, "
          f"decision margins: proposals {mp:.2e}, tests {ma:.2e}", flush=True)
    assert err <= ftol, f"relative F error {err:.3e}"
    assert out["stats"]["rounds"] == ref.rounds
    return err


def test_small_workload_fp64():
    X, prob = W.small()
    F, piv, out = gpu_factor(X, prob)
    ref = oracle_run(X, prob)
    err = assert_parity(F, piv, out, ref)
    st = out["stats"]
    assert abs(st["trace_A"] - ref.trace_A) < 1e-9
    assert abs(st["trace_resid"] - np.sum(ref.u)) < 1e-9 * ref.trace_A
    print(f"relF={err:.2e} rounds={st['rounds']}")


def test_more_chunks_than_the_one_launch_proposal_form():
    """N = 4.3e6 gives 4200 chunk sums, past the 4096 that the one-launch
    proposal kernel stages in LDS, so the proposals take the two-launch form
    (prefix in global memory); FP64 parity as everywhere else."""
    rng = np.random.default_rng(11)
    N = 4_300_000
    X = rng.random((N, 3))
    prob = W.Problem(N=N, d=3, k=16, b=8, kernel=W.GAUSSIAN, sigma=0.5, seed=5)
    F, piv, out = gpu_factor(X, prob)
    assert_parity(F, piv, out, oracle_run(X, prob))


def test_block_size_one():
    rng = np.random.default_rng(1)
    X = rng.random((1500, 2))
    prob = W.Problem(N=1500, d=2, k=40, b=1, kernel=W.GAUSSIAN, sigma=0.3, seed=3)
    F, piv, out = gpu_factor(X, prob)
    assert_parity(F, piv, out, oracle_run(X, prob))


@pytest.mark.parametrize("kernel", [W.GAUSSIAN, W.LAPLACE_L2, W.MATERN32, W.MATERN52])
def test_kernels_ragged_shapes(kernel):
    """N not a multiple of the 64-row tile nor of the 1024-row chunk, b not a
    multiple of the 64-column tile."""
    rng = np.random.default_rng(kernel + 10)
    X = rng.standard_normal((5003, 5))
    prob = W.Problem(N=5003, d=5, k=150, b=37, kernel=kernel, sigma=1.5, seed=kernel)
    F, piv, out = gpu_factor(X, prob)
    assert_parity(F, piv, out, oracle_run(X, prob))


@pytest.mark.parametrize("kernel", [W.GAUSSIAN, W.MATERN32])
def test_high_dimension_fp64(kernel):
    """d = 70: kernel columns from the matrix-core distance kernel (two
    contraction chunks, the second ragged) and H from the LDS-tiled gather
    (a ragged second chunk of 64 dims); b = 150 leaves a ragged 16 x 16 block."""
    rng = np.random.default_rng(70 + kernel)
    X = rng.standard_normal((3001, 70))
    prob = W.Problem(N=3001, d=70, k=400, b=150, kernel=kernel, sigma=6.0, seed=kernel)
    F, piv, out = gpu_factor(X, prob)
    assert_parity(F, piv, out, oracle_run(X, prob))


def test_large_block_global_rejection_path():
    """b above the LDS-resident limit runs RejectionSampleSubmatrix on a
    global-memory matrix."""
    rng = np.random.default_rng(2)
    X = rng.standard_normal((4000, 6))
    prob = W.Problem(N=4000, d=6, k=500, b=260, kernel=W.GAUSSIAN, sigma=2.0, seed=5)
    F, piv, out = gpu_factor(X, prob)
    assert_parity(F, piv, out, oracle_run(X, prob))


@pytest.mark.parametrize("b", [400, 512, 513])
def test_large_blocks_two_rounds(b):
    """b = 400 and 512: trailing tiles in global memory (ragged and full last
    block column); b = 513: the one-proposal-at-a-time global kernel.  Two
    full rounds and a partial third (the pivot cap)."""
    rng = np.random.default_rng(b)
    X = rng.standard_normal((5000, 6))
    prob = W.Problem(N=5000, d=6, k=2 * b + 11, b=b, kernel=W.MATERN32, sigma=1.5, seed=b)
    F, piv, out = gpu_factor(X, prob)
    assert_parity(F, piv, out, oracle_run(X, prob))


@pytest.mark.parametrize("b", [300, 520])
def test_identity_matrix_exact_large_block(b):
    """A = I with blocks above the register-resident limit: repeated proposals
    of one point inside a block must be rejected exactly as in sampling
    without replacement."""
    X = W.grid(5, levels=5)
    N = X.shape[0]
    prob = W.Problem(N=N, d=5, k=1500, b=b, kernel=W.GAUSSIAN, sigma=1.0, seed=13)
    F, piv, out = gpu_factor(X, prob)
    want = simulate_identity(N, prob.k, prob.b, philox_stream(prob.seed))
    assert list(piv) == want
    assert np.array_equal(F, np.eye(N)[:, want])


@pytest.mark.parametrize("b", [200, 256])
def test_identity_matrix_exact_register_block(b):
    """A = I on 512 points with blocks of the register-resident form: most
    rounds propose some point twice inside one 16-proposal block and across
    blocks, and the last rounds draw from a few remaining points, so the
    duplicate search sees long runs of repeats."""
    X = W.grid(3, levels=8)
    N = X.shape[0]
    prob = W.Problem(N=N, d=3, k=480, b=b, kernel=W.GAUSSIAN, sigma=1.0, seed=17)
    F, piv, out = gpu_factor(X, prob)
    want = simulate_identity(N, prob.k, prob.b, philox_stream(prob.seed))
    assert list(piv) == want
    assert np.array_equal(F, np.eye(N)[:, want])


def test_lds_limit_block_size():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((3000, 4))
    prob = W.Problem(N=3000, d=4, k=420, b=200, kernel=W.MATERN32, sigma=1.0, seed=9)
    F, piv, out = gpu_factor(X, prob)
    assert_parity(F, piv, out, oracle_run(X, prob))


def simulate_identity(N, k, b, stream):
    remaining = list(range(N))
    piv = []
    r = 0
    while len(piv) < k and remaining:
        U = stream(2 * b * r, 2 * b)[:b]
        T = float(len(remaining))
        props = [remaining[int(math.floor(x * T))] for x in U]
        for p in props:
            if len(piv) < k and p in remaining:
                piv.append(p)
                remaining.remove(p)
        r += 1
    return piv


ALL_PRECS = [W.FP64, W.FP32, W.BF16X3, W.BF16, W.FP8]


@pytest.mark.parametrize("prec", ALL_PRECS)
def test_identity_matrix_exact(prec):
    """Grid points 64 apart with a unit Gaussian: A = I exactly in any format,
    so pivots follow sampling without replacement and F is exact."""
    X = W.grid(5, levels=5)        # 3125 points: ragged against tiles and chunks
    N = X.shape[0]
    prob = W.Problem(N=N, d=5, k=700, b=64, kernel=W.GAUSSIAN, sigma=1.0, seed=11, prec=prec)
    F, piv, out = gpu_factor(X, prob)
    want = simulate_identity(N, prob.k, prob.b, philox_stream(prob.seed))
    assert list(piv) == want
    assert np.array_equal(F, np.eye(N)[:, want])


@pytest.mark.parametrize("prec", ALL_PRECS)
def test_cluster_matrix_exact(prec):
    sizes = [500, 70, 1300, 1, 220, 9, 3000]
    X, labels = W.clusters(sizes, d=3, seed=4)
    prob = W.Problem(N=X.shape[0], d=3, k=30, b=8, kernel=W.GAUSSIAN, sigma=1.0, seed=2, prec=prec)
    F, piv, out = gpu_factor(X, prob)
    assert out["status"] == 1 and out["stats"]["k_out"] == len(sizes)
    ref = oracle_run(X, prob)
    assert np.array_equal(piv[:len(sizes)], ref.pivots)
    assert np.all(piv[len(sizes):] == -1)
    assert np.array_equal(F, ref.F)
    assert out["stats"]["trace_resid"] == 0.0


def test_explicit_uniform_stream_equals_seeded_stream():
    X, prob = W.small()
    U = philox_stream(prob.seed)(0, 2 * prob.b * 40)
    F1, piv1, _ = gpu_factor(X, prob, U=U)
    F2, piv2, _ = gpu_factor(X, prob)
    assert np.array_equal(piv1, piv2) and np.array_equal(F1, F2)


def test_adversarial_uniforms():
    """Uniforms at the ends of [0,1): draws at the CDF extremes and acceptance
    tests with V = 0 (accept every positive residual)."""
    rng = np.random.default_rng(5)
    X = rng.random((2500, 3))
    prob = W.Problem(N=2500, d=3, k=90, b=12, kernel=W.LAPLACE_L2, sigma=0.4, seed=0)
    U = np.tile(np.concatenate([np.r_[0.0, 1 - 2.0 ** -53, 0.5, 2.0 ** -53], rng.random(8),
                                np.zeros(12)]), 40)
    F, piv, out = gpu_factor(X, prob, U=U)
    assert_parity(F, piv, out, oracle_run(X, prob, U=U))


def test_exhausted_uniform_stream_is_an_error():
    from paper_2410_03969_amd import binding
    X, prob = W.small()
    with pytest.raises(RuntimeError):
        binding.factor(X, prob, U=np.full(2 * prob.b * 2, 0.5))


def test_round_limit():
    X, prob = W.small()
    prob = prob.with_(k=100, b=7)
    F, piv, out = gpu_factor(X, prob.with_(max_rounds=3))
    ref = oracle_run(X, prob, max_rounds=3)
    assert out["stats"]["rounds"] == 3 and out["status"] == 0
    assert_parity(F, piv, out, ref)


def test_rank_equals_size():
    X = W.grid(3)
    prob = W.Problem(N=64, d=3, k=64, b=10, kernel=W.GAUSSIAN, sigma=1.0, seed=1)
    F, piv, out = gpu_factor(X, prob)
    assert sorted(piv) == list(range(64)) and out["status"] == 0


def test_nonfinite_points_rejected():
    from paper_2410_03969_amd import binding
    X, prob = W.small()
    X = X.copy()
    X[1234, 1] = np.nan
    with pytest.raises(RuntimeError, match="non-finite"):
        binding.factor(X, prob)


@pytest.mark.parametrize("d,bad", [(8, np.nan), (8, np.inf), (3, -np.inf)])
def test_nonfinite_points_rejected_fp8(d, bad):
    """The FP8 mode flags non-finite coordinates while it rounds the points
    (d % 4 == 0: in the same pass that packs the codes; else in the
    initialisation's scan of the rounded copy)."""
    from paper_2410_03969_amd import binding
    rng = np.random.default_rng(21)
    X = rng.random((3000, d))
    X[2999, d - 1] = bad
    prob = W.Problem(N=3000, d=d, k=40, b=10, kernel=W.GAUSSIAN, sigma=0.5, seed=2, prec=W.FP8)
    with pytest.raises(RuntimeError, match="non-finite"):
        binding.factor(X, prob)


def test_fp32_mode_factor_consistent_with_its_pivots():
    """FP32 storage: the factor equals the exact FP64 factor of the pivots it
    chose, to FP32 accuracy, on sampled rows."""
    X, prob = W.small()
    prob = prob.with_(prec=W.FP32)
    F, piv, out = gpu_factor(X, prob)
    acc = PointsAccess(X, prob.kernel, prob.sigma)
    assert len(set(piv.tolist())) == prob.k
    rows = np.random.default_rng(0).choice(prob.N, 200, replace=False)
    ref = factor_from_pivots(acc, piv[:40], rows=rows)
    err = np.linalg.norm(F[rows, :40] - ref) / np.linalg.norm(ref)
    assert err < 1e-4, err


@pytest.mark.parametrize("d", [40, 70])
def test_high_dimension_fp32_ragged_rows(d):
    """d > 16 in FP32: kernel columns from the FP32 matrix-core distance
    kernel, stored through its per-wavefront window; N = 3001 leaves a last
    row tile whose 16-byte runs stop short of N, and rows not a multiple of
    four.  The factor equals the FP64 factor of its own pivots to FP32
    accuracy, the last rows included."""
    rng = np.random.default_rng(d)
    N = 3001
    X = rng.standard_normal((N, d))
    prob = W.Problem(N=N, d=d, k=300, b=100, kernel=W.MATERN32, sigma=4.0, seed=d, prec=W.FP32)
    F, piv, out = gpu_factor(X, prob)
    assert out["stats"]["fused"] == 0
    assert out["stats"]["k_out"] == prob.k and len(set(piv.tolist())) == prob.k
    rows = np.concatenate([np.random.default_rng(1).choice(N - 8, 200, replace=False), np.arange(N - 8, N)])
    ref = factor_from_pivots(PointsAccess(X, prob.kernel, prob.sigma), piv[:150], rows=rows)
    err = np.linalg.norm(F[rows, :150] - ref) / np.linalg.norm(ref)
    print(f"fp32 d={d}: relF {err:.3e}")
    assert err < 1e-4, err


def test_laplace_workload_full_size_fp64():
    """The N = 1e5, d = 20, k = 1000, b = 120 Laplace workload at full size."""
    X, prob = W.laplace()
    F, piv, out = gpu_factor(X, prob)
    ref = oracle_run(X, prob)
    err = assert_parity(F, piv, out, ref)
    print(f"laplace relF={err:.2e} rounds={ref.rounds} trace_err={ref.trace_error:.4e}")


def test_vector_unit_gemm_cross_check(monkeypatch):
    """The register-tiled vector kernels (kept as a cross-check of the matrix
    cores) reproduce the oracle too."""
    monkeypatch.setenv("ARPC_GEMM", "valu")
    X, prob = W.small()
    F, piv, out = gpu_factor(X, prob)
    assert_parity(F, piv, out, oracle_run(X, prob))


# (b, d): one case per compiled column-block count of the one-kernel round
# product (2, 4, 8, 13, 16 blocks of 16 columns) and both coordinate widths.
FUSED_CASES = [(20, 3), (50, 8), (120, 12), (200, 8), (250, 16)]
# Relative Frobenius error of the first columns against the FP64 factor of the
# same pivots: three-product BF16 carries about 2^-17 relative error per
# product (FP32-class); one BF16 product about 2^-9 per operand.
FUSED_TOL = {W.BF16X3: 2e-4, W.BF16: 5e-2}


def assert_elementwise(F, ref, prec, label):
    """Every sampled entry within 4 FUSED_TOL of the largest one.  A localized
    mistake (one tile, one lane group, one store window) shifts a Frobenius
    norm over many rows only a little, but moves its own entries by about
    their size, and every entry is at most 1 here (|F(i,:)|^2 <= A_ii = 1)."""
    emax = float(np.max(np.abs(F - ref)))
    scale = float(np.max(np.abs(ref)))
    print(f"  {label}: max entry error {emax:.3e} ({emax / scale:.3e} of the largest entry)")
    assert emax <= 4 * FUSED_TOL[prec] * scale, (emax, scale)


@pytest.mark.parametrize("prec", [W.BF16X3, W.BF16])
@pytest.mark.parametrize("b,d", FUSED_CASES)
def test_fused_round_factor_consistent_with_its_pivots(prec, b, d):
    """The BF16 modes run the update GEMM, the solve and the stores as one
    kernel: its factor equals the FP64 factor of the pivots it chose, on
    sampled rows, over row counts that leave a ragged last tile and panel."""
    rng = np.random.default_rng(1000 + b)
    N = 6151
    X = rng.uniform(0.0, 1.0, size=(N, d))
    # Laplace kernel: a slowly decaying spectrum, so the rank stays far above k
    prob = W.Problem(N=N, d=d, k=min(3 * b, 600), b=b, kernel=W.LAPLACE_L2, sigma=0.5,
                     seed=11, prec=prec)
    F, piv, out = gpu_factor(X, prob)
    assert out["stats"]["fused"] == 1
    k_out = out["stats"]["k_out"]
    assert k_out == prob.k and len(set(piv[:k_out].tolist())) == k_out
    acc = PointsAccess(X, prob.kernel, prob.sigma)
    rows = np.concatenate([np.random.default_rng(0).choice(N, 150, replace=False), np.arange(N - 40, N)])
    ncols = min(k_out, 2 * b)
    ref = factor_from_pivots(acc, piv[:ncols], rows=rows)
    err = np.linalg.norm(F[rows, :ncols] - ref) / np.linalg.norm(ref)
    print(f"fused prec={prec} b={b} d={d} cols={ncols} relF={err:.3e}")
    assert err < FUSED_TOL[prec], err
    assert_elementwise(F[rows, :ncols], ref, prec, f"fused prec={prec} b={b} d={d}")
    # the residual trace from the factor stays a valid bound
    trA = out["stats"]["trace_A"]
    assert np.sum(F ** 2) <= trA * (1 + 1e-3)


@pytest.mark.parametrize("prec", [W.FP32, W.BF16X3, W.BF16])
def test_product_term_rows_unaligned_k(prec):
    """Where F is stored in FP32, H's product term F(S',:) F(S',:)^T reads the
    proposals' rows from an FP32 copy whose leading dimension is k rounded up
    to a multiple of four, four columns per 16-byte load.  k = 301 leaves
    three pad columns per row, the contraction splits into two partitions
    (k > 256), and k_r ends inside a 16-column chunk in most rounds; the
    first 2b columns (k_r up to 300, into the second partition) equal the
    FP64 factor of the same pivots."""
    rng = np.random.default_rng(301)
    N, b, d = 5003, 150, 8
    X = rng.uniform(0.0, 1.0, size=(N, d))
    prob = W.Problem(N=N, d=d, k=301, b=b, kernel=W.LAPLACE_L2, sigma=0.5, seed=13, prec=prec)
    print(f"[gpu parity] product term rows, prec={prec} N={N} k=301 b={b}", flush=True)
    F, piv, out = gpu_factor(X, prob)
    k_out = out["stats"]["k_out"]
    assert k_out == prob.k and len(set(piv[:k_out].tolist())) == k_out
    acc = PointsAccess(X, prob.kernel, prob.sigma)
    rows = np.concatenate([np.random.default_rng(3).choice(N, 150, replace=False), np.arange(N - 40, N)])
    ncols = 2 * b
    ref = factor_from_pivots(acc, piv[:ncols], rows=rows)
    err = np.linalg.norm(F[rows, :ncols] - ref) / np.linalg.norm(ref)
    tol = {W.FP32: 1e-4, **FUSED_TOL}[prec]
    print(f"product term rows prec={prec}: relF={err:.3e} (tol {tol:g})")
    assert err < tol, err
    if prec != W.FP32:
        assert_elementwise(F[rows, :ncols], ref, prec, f"product term rows prec={prec}")


@pytest.mark.parametrize("prec,b,d", [(W.BF16, 20, 17), (W.BF16, 60, 24), (W.BF16, 120, 32), (W.BF16, 200, 32)])
def test_fused_round_wide_points(prec, b, d):
    """The one-product BF16 mode also runs one kernel per round for
    16 < d <= 32 when b <= 208 (13 column blocks): the factor equals the FP64
    factor of its pivots on sampled rows, as for d <= 16."""
    rng = np.random.default_rng(2000 + b + d)
    N = 5003
    X = rng.uniform(0.0, 1.0, size=(N, d))
    prob = W.Problem(N=N, d=d, k=min(3 * b, 600), b=b, kernel=W.LAPLACE_L2, sigma=0.5, seed=12, prec=prec)
    F, piv, out = gpu_factor(X, prob)
    assert out["stats"]["fused"] == 1
    k_out = out["stats"]["k_out"]
    assert k_out == prob.k and len(set(piv[:k_out].tolist())) == k_out
    acc = PointsAccess(X, prob.kernel, prob.sigma)
    rows = np.concatenate([np.random.default_rng(1).choice(N, 150, replace=False), np.arange(N - 40, N)])
    ncols = min(k_out, 2 * b)
    ref = factor_from_pivots(acc, piv[:ncols], rows=rows)
    err = np.linalg.norm(F[rows, :ncols] - ref) / np.linalg.norm(ref)
    print(f"fused wide prec={prec} b={b} d={d} cols={ncols} relF={err:.3e}")
    assert err < FUSED_TOL[prec], err
    assert_elementwise(F[rows, :ncols], ref, prec, f"fused wide prec={prec} b={b} d={d}")
    assert np.sum(F ** 2) <= out["stats"]["trace_A"] * (1 + 1e-3)


@pytest.mark.parametrize("prec,b,d", [(W.BF16X3, 60, 17), (W.BF16, 240, 32), (W.BF16, 60, 33)])
def test_wide_points_outside_the_one_kernel_form(prec, b, d):
    """Three products at d > 16, one product with 14 or more column blocks
    at d > 16, and d > 32 keep the two-kernel round product (where the
    expanded distances fall back to direct differences as they cancel)."""
    rng = np.random.default_rng(3000 + b + d)
    X = rng.uniform(0.0, 1.0, size=(3001, d))
    prob = W.Problem(N=3001, d=d, k=2 * b, b=b, kernel=W.LAPLACE_L2, sigma=0.5, seed=13, prec=prec)
    F, piv, out = gpu_factor(X, prob)
    assert out["stats"]["fused"] == 0
    k_out = out["stats"]["k_out"]
    assert k_out == prob.k and len(set(piv[:k_out].tolist())) == k_out
    # the factor against the FP64 factor of its pivots, as for the one-kernel form
    acc = PointsAccess(X, prob.kernel, prob.sigma)
    rows = np.concatenate([np.random.default_rng(2).choice(3001, 150, replace=False), np.arange(3001 - 40, 3001)])
    ncols = min(k_out, 2 * b)
    ref = factor_from_pivots(acc, piv[:ncols], rows=rows)
    err = np.linalg.norm(F[rows, :ncols] - ref) / np.linalg.norm(ref)
    print(f"two-kernel prec={prec} b={b} d={d} cols={ncols} relF={err:.3e}")
    assert err < FUSED_TOL[prec], err
    assert_elementwise(F[rows, :ncols], ref, prec, f"two-kernel prec={prec} b={b} d={d}")


def test_fused_and_two_kernel_paths_agree_on_exact_matrix(monkeypatch):
    """On the exact cluster matrix both BF16 round products recover the same
    rank and pivots (a round-off independent answer)."""
    X, labels = W.clusters([40] * 30, d=6, spacing=50.0, seed=5)
    prob = W.Problem(N=X.shape[0], d=6, k=30, b=16, kernel=W.GAUSSIAN, sigma=0.5, seed=3, prec=W.BF16)
    F1, piv1, out1 = gpu_factor(X, prob)
    monkeypatch.setenv("ARPC_FUSED", "0")
    F2, piv2, out2 = gpu_factor(X, prob)
    assert out1["stats"]["fused"] == 1 and out2["stats"]["fused"] == 0
    assert np.array_equal(piv1, piv2)
    assert sorted(labels[piv1[:30]].tolist()) == list(range(30))


@pytest.mark.parametrize("prec", [W.FP32, W.BF16X3, W.BF16])
def test_reduced_precision_trace_error(prec):
    """Reduced-precision modes keep the trace error within 1.05x of the FP64
    run, both from the factor (tr A - |F|^2) and from the pivots alone
    (Nystrom residual recomputed in FP64 by the oracle)."""
    from oracle import nystrom_err
    X, prob = W.laplace(N=20_000)
    prob = prob.with_(k=400, b=50)
    F64, piv64, out64 = gpu_factor(X, prob)
    Fm, pivm, outm = gpu_factor(X, prob.with_(prec=prec))
    trA = out64["stats"]["trace_A"]
    te64 = (trA - np.sum(F64 ** 2)) / trA
    tem = (trA - np.sum(Fm ** 2)) / trA
    acc = PointsAccess(X, prob.kernel, prob.sigma)
    ny64 = nystrom_err(acc, piv64[:out64["stats"]["k_out"]]).sum() / trA
    nym = nystrom_err(acc, pivm[:outm["stats"]["k_out"]]).sum() / trA
    print(f"prec={prec} trace err F: {tem:.6e} vs fp64 {te64:.6e}; nystrom {nym:.6e} vs {ny64:.6e}")
    assert tem <= 1.05 * te64 and nym <= 1.05 * ny64


@pytest.mark.parametrize("d", [24, 30, 40, 32, 48, 256])
def test_fp8_mode_factors_the_rounded_points(d):
    """The FP8 mode factors the kernel matrix of the points rounded to e4m3:
    its factor matches the FP64 factor of its pivots on round_e4m3(X) to the
    BF16 update's accuracy, and is clearly further from that of the unrounded
    points.  Coordinates reach (240, 448] (OCP e4m3 only) and beyond 448
    (saturation); d = 24 and 40 leave a ragged 32-wide contraction step (packed
    e4m3 rows, kernel columns stored by the distance kernel), d = 30 takes the
    unpacked path (d not a multiple of 4); d = 32, 48 and 256 form the kernel
    columns in the update GEMM's epilogue (d % 16 == 0, d <= 256; 48 leaves a
    ragged step there).  N = 4001 at d = 24 and 48: the last tile is ragged."""
    rng = np.random.default_rng(d)
    N = 4001 if d in (24, 48) else 4000
    X = 100.0 * rng.standard_normal((N, d))
    X[0, 0], X[1, 1], X[2, 2] = 1000.0, -460.0, 300.0
    prob = W.Problem(N=N, d=d, k=300, b=60, kernel=W.GAUSSIAN, sigma=60.0 * np.sqrt(d), seed=d, prec=W.FP8)
    F, piv, out = gpu_factor(X, prob)
    k_out = out["stats"]["k_out"]
    assert out["stats"]["fused"] == 0
    assert k_out == prob.k and len(set(piv.tolist())) == k_out
    rows = np.concatenate([np.arange(8), rng.choice(N, 200, replace=False), np.arange(N - 8, N)])
    ncols = 120
    Xq = round_e4m3(X)
    assert np.count_nonzero(np.abs(Xq) > 240) > 50
    ref_q = factor_from_pivots(PointsAccess(Xq, prob.kernel, prob.sigma), piv[:ncols], rows=rows)
    ref_x = factor_from_pivots(PointsAccess(X, prob.kernel, prob.sigma), piv[:ncols], rows=rows)
    err_q = np.linalg.norm(F[rows, :ncols] - ref_q) / np.linalg.norm(ref_q)
    err_x = np.linalg.norm(F[rows, :ncols] - ref_x) / np.linalg.norm(ref_x)
    print(f"fp8 d={d}: relF vs rounded points {err_q:.3e}, vs unrounded {err_x:.3e}")
    assert err_q < 2e-2 and err_q < 0.25 * err_x
    # every entry, as in assert_elementwise (FP8 mode: 4 x 2e-2 of the largest entry)
    emax = float(np.max(np.abs(F[rows, :ncols] - ref_q)))
    print(f"  fp8 d={d}: max entry error {emax:.3e}")
    assert emax <= 4 * 2e-2 * float(np.max(np.abs(ref_q)))
