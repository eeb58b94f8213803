"""Asynchronous factorization through the C ABI (arpc_factor_async,
arpc_factor_continue, arpc_factor_query): the same result as the blocking
arpc_factor, bit for bit, with other work on the same stream between the
call and the synchronisation; a round limit that ends the run early, then
more rounds; an early stop on an exact low-rank matrix; and the serving
context's outstanding-job limit (ARPC_EBUSY)."""
import sys

import numpy as np
import pytest

from paper_2410_03969_amd import binding as B
from paper_2410_03969_amd import workloads as W

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _buffers(prob):
    import torch
    dev = torch.device("cuda:0")
    fdt = torch.float64 if prob.prec == W.FP64 else torch.float32
    Ft = torch.full((prob.k, prob.N), 5.0, dtype=fdt, device=dev)
    piv = torch.full((prob.k,), 7, dtype=torch.int64, device=dev)
    nb = B.arpc_workspace_size(B.make_problem(prob))
    ws = torch.empty(nb, dtype=torch.uint8, device=dev)
    return Ft, piv, ws, nb


def _blocking(X, prob):
    out = B.factor(X, prob)
    return out["F"].cpu().numpy().copy(), out["pivots"].cpu().numpy().copy(), out["status"], out["stats"]


def _with(gen, **kw):
    X, prob = gen()
    return X, prob.with_(**kw)


CASES = {
    "small_fp64": W.small,
    "mixture_bf16": lambda: _with(lambda: W.mixture(N=200_000), k=1000, b=100, prec=W.BF16),
    "laplace_fp32": lambda: _with(lambda: W.laplace(N=20_000), k=400, b=60, prec=W.FP32),
}


@pytest.mark.parametrize("name", list(CASES))
def test_async_equals_blocking(name):
    import torch
    X, prob = CASES[name]()
    _log(f"[async] {name} N={prob.N} d={prob.d} k={prob.k} b={prob.b} prec={prob.prec}")
    F0, p0, s0, st0 = _blocking(X, prob)
    Xd = torch.from_numpy(X).cuda()
    Ft, piv, ws, nb = _buffers(prob)
    pr = B.make_problem(prob)
    s = torch.cuda.current_stream()
    torch.cuda.synchronize()
    st = B.arpc_factor_async(pr, Xd.data_ptr(), Ft.data_ptr(), piv.data_ptr(), ws.data_ptr(), nb, s.cuda_stream)
    assert st == B.ARPC_OK
    pending = not s.query()
    # unrelated work on the same stream, ordered after the factorization
    Z = torch.arange(1 << 20, dtype=torch.float64, device="cuda")
    Z.mul_(2.0).add_(1.0)
    s.synchronize()
    assert float(Z[12345].item()) == 2.0 * 12345 + 1.0
    st, stats = B.arpc_factor_query(pr, ws.data_ptr(), nb)
    assert st == s0, (st, s0)
    assert stats.k_out == st0["k_out"] and stats.rounds == st0["rounds"]
    assert stats.trace_resid == st0["trace_resid"] and stats.trace_A == st0["trace_A"]
    assert stats.flops_colgemm == st0["flops_colgemm"]
    assert np.array_equal(piv.cpu().numpy(), p0)
    assert np.array_equal(Ft.t().cpu().numpy(), F0)
    _log(f"[async] {name}: stream busy right after the call: {pending}")
    if name == "mixture_bf16":
        assert pending   # a few milliseconds of device work: the call did not wait for it


def test_round_limit_then_continue():
    import torch
    X, prob = W.small()
    prob = prob.with_(k=300, b=20)
    F0, p0, s0, _ = _blocking(X, prob)
    Xd = torch.from_numpy(X).cuda()
    Ft, piv, ws, nb = _buffers(prob)
    pr = B.make_problem(prob)
    s = torch.cuda.current_stream()
    assert B.arpc_factor_async(pr, Xd.data_ptr(), Ft.data_ptr(), piv.data_ptr(), ws.data_ptr(), nb,
                               s.cuda_stream, 3) == B.ARPC_OK
    s.synchronize()
    st, stats = B.arpc_factor_query(pr, ws.data_ptr(), nb)
    assert st == B.ARPC_INCOMPLETE and stats.rounds == 3 and 0 < stats.k_out < prob.k
    k3 = stats.k_out
    assert np.array_equal(piv.cpu().numpy()[:k3], p0[:k3])
    assert np.all(piv.cpu().numpy()[k3:] == -1) and np.all(Ft.t().cpu().numpy()[:, k3:] == 0.0)
    # more rounds than needed: the surplus ones exit on the device
    assert B.arpc_factor_continue(pr, Xd.data_ptr(), Ft.data_ptr(), piv.data_ptr(), ws.data_ptr(), nb,
                                  s.cuda_stream, prob.k) == B.ARPC_OK
    s.synchronize()
    st, stats = B.arpc_factor_query(pr, ws.data_ptr(), nb)
    assert st == s0 == B.ARPC_OK and stats.k_out == prob.k
    assert np.array_equal(piv.cpu().numpy(), p0)
    assert np.array_equal(Ft.t().cpu().numpy(), F0)


def test_async_early_stop_on_exact_low_rank():
    import torch
    X, _ = W.clusters([50] * 12, d=4, spacing=64.0, seed=2)
    prob = W.Problem(N=X.shape[0], d=4, k=40, b=8, kernel=W.GAUSSIAN, sigma=1.0, seed=5, prec=W.BF16)
    Xd = torch.from_numpy(X).cuda()
    Ft, piv, ws, nb = _buffers(prob)
    pr = B.make_problem(prob)
    s = torch.cuda.current_stream()
    assert B.arpc_factor_async(pr, Xd.data_ptr(), Ft.data_ptr(), piv.data_ptr(), ws.data_ptr(), nb,
                               s.cuda_stream, 0) == B.ARPC_OK
    s.synchronize()
    st, stats = B.arpc_factor_query(pr, ws.data_ptr(), nb)
    assert st == B.ARPC_EARLY_STOP and stats.k_out == 12 and stats.trace_resid == 0.0
    p = piv.cpu().numpy()
    assert np.all(p[12:] == -1) and np.all(Ft.t().cpu().numpy()[:, 12:] == 0.0)


def test_serving_outstanding_limit_gives_ebusy():
    rng = np.random.default_rng(8)
    X = rng.random((60000, 3))
    big = W.Problem(N=60000, d=3, k=1500, b=15, kernel=W.GAUSSIAN, sigma=0.05, seed=0, prec=W.BF16)
    small = W.Problem(N=4000, d=3, k=40, b=8, kernel=W.GAUSSIAN, sigma=0.5, seed=1, prec=W.BF16)
    ws = B.arpc_workspace_size(B.make_problem(big))
    srv = B.Server(2 * ws, max_slots=1)
    try:
        assert B.arpc_serving_set_limit(srv.ctx, 0) == B.ARPC_EINVAL
        assert B.arpc_serving_set_limit(srv.ctx, 2) == B.ARPC_OK
        h1 = srv.submit(X, big)          # active (one slot)
        h2 = srv.submit(X[:4000], small)  # queued behind it
        with pytest.raises(RuntimeError, match="busy"):
            srv.submit(X[:4000], small.with_(seed=2))
        r1, r2 = srv.wait(h1), srv.wait(h2)
        assert r1["status"] == 0 and r2["status"] == 0
        h3 = srv.submit(X[:4000], small.with_(seed=2))   # room again
        assert srv.wait(h3)["status"] == 0
    finally:
        srv.close()
