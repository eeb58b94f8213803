"""GPU serving tests (continuous batching through the C ABI).

Each job's result must be the same alone (arpc_factor) and in the mix
(submitted with other jobs to a serving context whose budget forces queueing
and whose slots let rounds of different jobs overlap): the kernels, launch
shapes and data of a job do not depend on the other jobs, so the comparison is
bit for bit.
"""
import sys
import time

import numpy as np
import pytest

from paper_2410_03969_amd import workloads as W

pytestmark = pytest.mark.gpu


def _jobs():
    """Twelve jobs shaped like the serving stream (points uniform on [0,1]^d,
    Gaussian kernel with bandwidth sqrt(d), b = k/10), small enough for a test,
    over every precision mode (FP8 included), both round-product paths and
    both pivot rules (jobs 5 and 11 run block RPCholesky)."""
    rng = np.random.default_rng(4)
    precs = [W.BF16X3, W.BF16, W.FP64, W.FP32, W.FP8]
    out = []
    for j in range(12):
        N = int(round(10 ** rng.uniform(3.3, 4.3)))
        d = int(rng.choice([3, 8, 32]))
        k = int(rng.integers(40, 300))
        b = max(1, k // 10)
        X = np.random.default_rng(1000 + j).random((N, d))
        prob = W.Problem(N=N, d=d, k=k, b=b, kernel=W.GAUSSIAN, sigma=float(np.sqrt(d)), seed=j,
                         prec=precs[j % len(precs)], method=W.BLOCK if j % 6 == 5 else W.ACCEL)
        out.append((X, prob))
    return out


def _alone(X, prob):
    from paper_2410_03969_amd import binding
    out = binding.factor(X, prob)
    return out["F"].cpu().numpy().copy(), out["pivots"].cpu().numpy().copy(), out["status"]


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


MODES = {"ticks": ("1", "1"), "graphs": ("0", "1"), "plain": ("0", "0")}   # (ARPC_SERVE_TICKS, ARPC_SERVE_GRAPHS)


@pytest.mark.parametrize("mode", list(MODES))
def test_results_same_alone_and_in_the_mix(monkeypatch, mode):
    """Ticks: the BF16-mode jobs with d <= 16 advance together (one launch per
    round step over a table of jobs); graphs / plain: every job on its own
    slot stream, with or without graph replay."""
    from paper_2410_03969_amd import binding
    ticks, graphs = MODES[mode]
    monkeypatch.setenv("ARPC_SERVE_TICKS", ticks)
    monkeypatch.setenv("ARPC_SERVE_GRAPHS", graphs)
    jobs = _jobs()
    alone = []
    for X, prob in jobs:
        _log(f"[serving alone] N={prob.N} d={prob.d} k={prob.k} b={prob.b} prec={prob.prec} method={prob.method}")
        alone.append(_alone(X, prob))
    ws = [binding.arpc_workspace_size(binding.make_problem(p)) for _, p in jobs]
    budget = int(2.5 * max(ws))   # a few jobs at a time: the rest wait for memory
    _log(f"[serving mix] budget={budget} slots=4 mode={mode}")
    srv = binding.Server(budget, max_slots=4)
    try:
        handles = [srv.submit(X, prob) for X, prob in jobs]
        results = [srv.wait(h) for h in handles]
        info = srv.info()
    finally:
        srv.close()
    for (F0, p0, s0), r, (X, prob) in zip(alone, results, jobs):
        assert r["status"] == s0
        assert np.array_equal(r["pivots"].cpu().numpy(), p0), f"pivots differ for job {prob}"
        assert np.array_equal(r["F"].cpu().numpy(), F0), f"F differs for job {prob}"
        assert r["stats"]["ms_total"] > 0
    assert info["completed"] == len(jobs) and info["active"] == 0 and info["queued"] == 0
    assert info["peak_bytes"] <= budget
    assert info["peak_active"] >= 2, info     # jobs did overlap
    n_tickable = sum(1 for _, p in jobs if (p.prec in (W.BF16, W.BF16X3) and p.d <= 16)
                     or (p.prec == W.BF16 and p.d <= 32 and p.b <= 208))
    if mode == "ticks":
        assert info["ticked_jobs"] == n_tickable and info["ticks"] > 0, info
    else:
        assert info["ticked_jobs"] == 0 and info["ticks"] == 0, info


def test_ticked_jobs_share_launches():
    """Sixteen small BF16-mode jobs of three column-block shapes, all
    submitted at once with room for all of them: fewer ticks than the jobs'
    rounds added up (each tick ran a round of several jobs), and every result
    equals the job's result alone."""
    from paper_2410_03969_amd import binding
    rng = np.random.default_rng(11)
    jobs = []
    for j in range(16):
        N = int(rng.integers(3000, 9000))
        d = int(rng.choice([3, 8, 16]))
        k = int(rng.choice([60, 300, 1000]))
        X = np.random.default_rng(2000 + j).random((N, d))
        jobs.append((X, W.Problem(N=N, d=d, k=k, b=k // 10, kernel=W.GAUSSIAN, sigma=0.3, seed=j,
                                  prec=W.BF16 if j % 3 else W.BF16X3)))
    alone = [_alone(X, p) for X, p in jobs]
    budget = sum(binding.arpc_workspace_size(binding.make_problem(p)) for _, p in jobs) + (1 << 24)
    _log(f"[serving ticks] 16 jobs budget={budget}")
    srv = binding.Server(budget, max_slots=16)
    try:
        hs = [srv.submit(X, p) for X, p in jobs]
        res = [srv.wait(h) for h in hs]
        info = srv.info()
    finally:
        srv.close()
    rounds = 0
    for (F0, p0, s0), r in zip(alone, res):
        assert r["status"] == s0
        assert np.array_equal(r["pivots"].cpu().numpy(), p0)
        assert np.array_equal(r["F"].cpu().numpy(), F0)
        rounds += r["stats"]["rounds"]
    print(f"ticks {info['ticks']} for {rounds} job rounds, peak active {info['peak_active']}")
    assert info["ticked_jobs"] == 16
    assert info["ticks"] < rounds


def test_served_fp64_jobs_match_the_oracle():
    """Eight jobs of the serving stream's shape (the first eight with
    N <= 20000: points uniform on [0,1]^d, Gaussian sigma = sqrt(d),
    b = k / 10), served together in FP64, against the FP64 oracle on the same
    uniform stream.  Pivots are compared over the rounds that start with a
    residual trace above 1e-8 tr A; F over the same columns within 1e-10.
    Jobs with d = 3 or 8 reach numerical rank before k: past that point the
    residual diagonal is rounding noise on both sides, and their decisions
    differ as ties do; there both runs must end with a residual trace at
    that level."""
    from oracle import PointsAccess, philox_stream, rpc_accel
    from paper_2410_03969_amd import binding
    stream = W.serving_stream(n_jobs=512, rate=1.0, prec=W.FP64, materialize=False)
    picked = [j for j in stream if j.problem.N <= 20000][:8]
    jobs = [(np.random.default_rng(1000 + j.job_id).random((j.problem.N, j.problem.d)), j.problem) for j in picked]
    budget = sum(binding.arpc_workspace_size(binding.make_problem(p)) for _, p in jobs) + (1 << 24)
    _log(f"[serving fp64] jobs {[j.job_id for j in picked]}")
    srv = binding.Server(budget, max_slots=8)
    try:
        hs = [srv.submit(X, p) for X, p in jobs]
        res = [srv.wait(h) for h in hs]
    finally:
        srv.close()
    for (X, p), r in zip(jobs, res):
        ref = rpc_accel(PointsAccess(X, p.kernel, p.sigma), p.k, p.b, philox_stream(p.seed), record=True)
        starts = [ref.trace_A] + [float(h.sum()) for h in ref.u_history]
        r_ok = next((i for i, t in enumerate(starts) if t <= 1e-8 * ref.trace_A), len(ref.round_sizes))
        r_ok = min(r_ok, len(ref.round_sizes))
        m = int(sum(ref.round_sizes[:r_ok]))
        st = r["stats"]
        k_out = st["k_out"]
        piv = r["pivots"].cpu().numpy()
        assert k_out >= m, (p, k_out, m)
        assert np.array_equal(piv[:m], ref.pivots[:m]), p
        # F: the columns of rounds that start above 1e-6 tr A within 1e-10
        # (Frobenius).  The later compared columns belong to pivots whose
        # residuals h went down to 1e-8 of the diagonal (kappa(0) = 1): a
        # column of the factor is as accurate as the condition of A(S,S) so
        # far allows, about 1 / min h, so column c is held to 1e-13 / min h
        # over the columns up to c (h of column c = F(s_c, c)^2).
        r_f = next((i for i, t in enumerate(starts) if t <= 1e-6 * ref.trace_A), len(ref.round_sizes))
        mf = int(sum(ref.round_sizes[:min(r_f, r_ok)]))
        F = r["F"].cpu().numpy()[:, :m]
        err = np.linalg.norm(F[:, :mf] - ref.F[:, :mf]) / np.linalg.norm(ref.F[:, :mf])
        hmin = np.minimum.accumulate(ref.F[ref.pivots[:m], np.arange(m)] ** 2)
        col = np.linalg.norm(F - ref.F[:, :m], axis=0) / np.linalg.norm(ref.F[:, :m], axis=0)
        ratio = (col * hmin / 1e-13)[mf:]
        print(f"N={p.N} d={p.d} k={p.k}: k_out={k_out} (oracle {ref.k_out}), compared {m} pivots "
              f"over {r_ok} rounds, relF={err:.2e} over {mf} columns; later columns: worst error "
              f"{col[mf:].max() if m > mf else 0:.2e}, worst error / (1e-13 / min h) "
              f"{ratio.max() if m > mf else 0:.2e}")
        assert err <= 1e-10
        assert m == mf or ratio.max() <= 1.0
        if ref.k_out == p.k and r_ok == len(ref.round_sizes):
            assert k_out == p.k and np.array_equal(piv, ref.pivots)
        else:
            assert st["trace_resid"] <= 1e-8 * st["trace_A"], st
            assert float(np.sum(ref.u)) <= 1e-8 * ref.trace_A


def test_admission_respects_budget():
    from paper_2410_03969_amd import binding
    X = np.random.default_rng(0).random((20000, 8))
    prob = W.Problem(N=20000, d=8, k=200, b=20, kernel=W.GAUSSIAN, sigma=1.0, seed=1, prec=W.BF16X3)
    ws = binding.arpc_workspace_size(binding.make_problem(prob))
    budget = 2 * ws + ws // 2                 # two jobs fit, three do not
    _log(f"[serving budget] ws={ws} budget={budget}")
    srv = binding.Server(budget, max_slots=8)
    try:
        hs = [srv.submit(X, prob.with_(seed=s)) for s in range(6)]
        res = [srv.wait(h) for h in hs]
        info = srv.info()
    finally:
        srv.close()
    assert all(r["status"] == 0 for r in res)
    assert info["peak_bytes"] <= budget
    assert info["peak_active"] <= 2
    # the same job alone gives the same pivots
    _, p0, _ = _alone(X, prob.with_(seed=3))
    assert np.array_equal(res[3]["pivots"].cpu().numpy(), p0)


def test_cancel_errors_and_destroy():
    from paper_2410_03969_amd import binding
    rng = np.random.default_rng(2)
    X = rng.random((50000, 3))
    big = W.Problem(N=50000, d=3, k=1500, b=15, kernel=W.GAUSSIAN, sigma=0.05, seed=0, prec=W.BF16)
    small = W.Problem(N=5000, d=3, k=50, b=5, kernel=W.GAUSSIAN, sigma=0.5, seed=1, prec=W.BF16)
    ws_big = binding.arpc_workspace_size(binding.make_problem(big))
    _log(f"[serving cancel] ws_big={ws_big}")
    srv = binding.Server(ws_big + (1 << 20), max_slots=1)
    try:
        # too large for the whole budget
        import torch
        Xd = torch.from_numpy(X).cuda()
        F = torch.empty((4000, 50000), dtype=torch.float32, device="cuda")
        piv = torch.empty(4000, dtype=torch.int64, device="cuda")
        st, _ = binding.arpc_submit(srv.ctx, binding.make_problem(big.with_(k=4000, b=40)), Xd.data_ptr(),
                                    F.data_ptr(), piv.data_ptr())
        assert st == binding.ARPC_ENOMEM
        st, _ = binding.arpc_submit(srv.ctx, binding.make_problem(big.with_(b=0)), Xd.data_ptr(),
                                    F.data_ptr(), piv.data_ptr())
        assert st == binding.ARPC_EINVAL
        # one slot: the second job waits in the queue and is cancelled there
        h1 = srv.submit(X, big)
        h2 = srv.submit(X[:5000], small)
        assert srv.cancel(h2) == 0
        r2 = srv.wait(h2)
        assert r2["status"] == binding.ARPC_ECANCELED
        # the active job is cancelled between batches of rounds (or has finished)
        assert srv.cancel(h1) == 0
        r1 = srv.wait(h1)
        assert r1["status"] in (binding.ARPC_ECANCELED, binding.ARPC_OK)
        # the context still serves
        h3 = srv.submit(X[:5000], small)
        r3 = srv.wait(h3)
        assert r3["status"] == 0
        _, p0, _ = _alone(X[:5000], small)
        assert np.array_equal(r3["pivots"].cpu().numpy(), p0)
        info = srv.info()
        assert info["cancelled"] >= 1
        # destroy with work still queued and active
        srv.submit(X, big)
        srv.submit(X[:5000], small)
        time.sleep(0.01)
    finally:
        srv.close()
