"""Thin ctypes binding of libarpc.so (argument marshalling only).

Names mirror the C ABI in include/arpc.h.  Every computation runs in the HIP
library; PyTorch is used only to allocate device memory and to obtain the
current HIP stream.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libarpc.so")

ARPC_OK, ARPC_EARLY_STOP, ARPC_INCOMPLETE = 0, 1, 2
ARPC_EINVAL, ARPC_ENOMEM, ARPC_EBUSY, ARPC_EDEVICE, ARPC_ENUMERIC, ARPC_ECANCELED = -1, -2, -3, -4, -5, -6
KERNEL_CLASSES = ["init", "propose", "gather", "reject", "prep", "colgemm", "trsm", "diag", "finish"]
NUM_KC = len(KERNEL_CLASSES)

EXPORTS = ["arpc_status_str", "arpc_version", "arpc_workspace_size", "arpc_factor",
           "arpc_factor_uniforms", "arpc_stream_uniforms_host", "arpc_set_profiling",
           "arpc_set_profiling_classes", "arpc_lowmem_workspace_size", "arpc_factor_lowmem",
           "arpc_qr_workspace_size", "arpc_qr_factor", "arpc_krr_workspace_size", "arpc_krr_pcg",
           "arpc_create", "arpc_destroy", "arpc_submit", "arpc_poll", "arpc_wait", "arpc_cancel",
           "arpc_serving_info", "arpc_factor_async", "arpc_factor_continue", "arpc_factor_query",
           "arpc_serving_set_limit"]


class ArpcProblem(C.Structure):
    _fields_ = [("N", C.c_int64), ("d", C.c_int64), ("k", C.c_int64), ("b", C.c_int64),
                ("kernel", C.c_int32), ("prec", C.c_int32), ("bandwidth", C.c_double),
                ("seed", C.c_uint64), ("max_rounds", C.c_int64), ("method", C.c_int32),
                ("reserved", C.c_int32)]


class ArpcKrrStats(C.Structure):
    _fields_ = [("iterations", C.c_int64), ("rel_residual", C.c_double), ("ms_total", C.c_double),
                ("ms_setup", C.c_double), ("ms_matvec", C.c_double), ("ms_precond", C.c_double),
                ("status", C.c_int32), ("reserved", C.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


class ArpcStats(C.Structure):
    _fields_ = [("k_out", C.c_int64), ("rounds", C.c_int64), ("proposals", C.c_int64),
                ("status", C.c_int32), ("fused", C.c_int32), ("trace_A", C.c_double),
                ("trace_resid", C.c_double), ("ms_total", C.c_double),
                ("ms_kernel", C.c_double * NUM_KC), ("launches", C.c_int64 * NUM_KC),
                ("flops_colgemm", C.c_double), ("flops_trsm", C.c_double),
                ("bytes_colgemm", C.c_double), ("bytes_trsm", C.c_double), ("bytes_blocked", C.c_double)]

    def as_dict(self) -> dict:
        d = {f: getattr(self, f) for f, _ in self._fields_ if f not in ("ms_kernel", "launches")}
        d["ms_kernel"] = dict(zip(KERNEL_CLASSES, list(self.ms_kernel)))
        d["launches"] = dict(zip(KERNEL_CLASSES, list(self.launches)))
        return d


class ArpcServingStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("cancelled", C.c_int64),
                ("active", C.c_int64), ("queued", C.c_int64), ("peak_active", C.c_int64),
                ("bytes_in_use", C.c_int64), ("peak_bytes", C.c_int64), ("budget_bytes", C.c_int64),
                ("slots", C.c_int64), ("ticks", C.c_int64), ("ticked_jobs", C.c_int64)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def lib():
    """Load libarpc.so (raises if it is missing: there is no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing; build it with "
                              "`python -m paper_2410_03969_amd.build`")
        L = C.CDLL(LIB_PATH)
        L.arpc_status_str.restype = C.c_char_p
        L.arpc_status_str.argtypes = [C.c_int]
        L.arpc_version.restype = C.c_char_p
        L.arpc_workspace_size.restype = C.c_int
        L.arpc_workspace_size.argtypes = [C.POINTER(ArpcProblem), C.POINTER(C.c_size_t)]
        L.arpc_factor.restype = C.c_int
        L.arpc_factor.argtypes = [C.POINTER(ArpcProblem), C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.c_void_p, C.c_size_t, C.c_void_p, C.POINTER(ArpcStats)]
        L.arpc_factor_uniforms.restype = C.c_int
        L.arpc_factor_uniforms.argtypes = [C.POINTER(ArpcProblem), C.c_void_p, C.c_void_p, C.c_void_p,
                                           C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p, C.c_int64,
                                           C.POINTER(ArpcStats)]
        for name in ("arpc_factor_async", "arpc_factor_continue"):
            fn = getattr(L, name)
            fn.restype = C.c_int
            fn.argtypes = [C.POINTER(ArpcProblem), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t,
                           C.c_void_p, C.c_int64]
        L.arpc_factor_query.restype = C.c_int
        L.arpc_factor_query.argtypes = [C.POINTER(ArpcProblem), C.c_void_p, C.c_size_t, C.POINTER(ArpcStats)]
        L.arpc_serving_set_limit.restype = C.c_int
        L.arpc_serving_set_limit.argtypes = [C.c_void_p, C.c_int64]
        L.arpc_stream_uniforms_host.restype = C.c_int
        L.arpc_lowmem_workspace_size.restype = C.c_int
        L.arpc_lowmem_workspace_size.argtypes = [C.POINTER(ArpcProblem), C.POINTER(C.c_size_t)]
        L.arpc_factor_lowmem.restype = C.c_int
        L.arpc_factor_lowmem.argtypes = [C.POINTER(ArpcProblem), C.c_void_p, C.c_void_p, C.c_void_p,
                                         C.c_void_p, C.c_size_t, C.c_void_p, C.POINTER(ArpcStats)]
        L.arpc_qr_workspace_size.restype = C.c_int
        L.arpc_qr_workspace_size.argtypes = [C.c_int64, C.c_int64, C.c_int64, C.c_int64, C.POINTER(C.c_size_t)]
        L.arpc_qr_factor.restype = C.c_int
        L.arpc_qr_factor.argtypes = [C.c_int64, C.c_int64, C.c_int64, C.c_int64, C.c_uint64, C.c_int64,
                                     C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t,
                                     C.c_void_p, C.POINTER(ArpcStats)]
        L.arpc_krr_workspace_size.restype = C.c_int
        L.arpc_krr_workspace_size.argtypes = [C.c_int64, C.c_int64, C.c_int64, C.c_int32, C.POINTER(C.c_size_t)]
        L.arpc_krr_pcg.restype = C.c_int
        L.arpc_krr_pcg.argtypes = [C.c_int64, C.c_int64, C.c_int32, C.c_double, C.c_double, C.c_void_p, C.c_void_p,
                                   C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_int64, C.c_void_p, C.c_void_p,
                                   C.c_size_t, C.c_void_p, C.POINTER(ArpcKrrStats)]
        L.arpc_stream_uniforms_host.argtypes = [C.c_uint64, C.c_int64, C.c_int64, C.c_void_p]
        L.arpc_set_profiling.restype = None
        L.arpc_set_profiling.argtypes = [C.c_int]
        L.arpc_set_profiling_classes.restype = None
        L.arpc_set_profiling_classes.argtypes = [C.c_uint]
        L.arpc_create.restype = C.c_int
        L.arpc_create.argtypes = [C.c_int, C.c_size_t, C.c_int, C.POINTER(C.c_void_p)]
        L.arpc_destroy.restype = C.c_int
        L.arpc_destroy.argtypes = [C.c_void_p]
        L.arpc_submit.restype = C.c_int
        L.arpc_submit.argtypes = [C.c_void_p, C.POINTER(ArpcProblem), C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.POINTER(C.c_uint64)]
        L.arpc_poll.restype = C.c_int
        L.arpc_poll.argtypes = [C.c_void_p, C.c_uint64, C.POINTER(C.c_int), C.POINTER(ArpcStats)]
        L.arpc_wait.restype = C.c_int
        L.arpc_wait.argtypes = [C.c_void_p, C.c_uint64, C.POINTER(ArpcStats)]
        L.arpc_cancel.restype = C.c_int
        L.arpc_cancel.argtypes = [C.c_void_p, C.c_uint64]
        L.arpc_serving_info.restype = C.c_int
        L.arpc_serving_info.argtypes = [C.c_void_p, C.POINTER(ArpcServingStats)]
        _lib = L
    return _lib


def make_problem(p) -> ArpcProblem:
    """From a workloads.Problem (or any object with the same fields)."""
    return ArpcProblem(N=p.N, d=p.d, k=p.k, b=p.b, kernel=p.kernel, prec=p.prec,
                       bandwidth=float(p.sigma), seed=int(p.seed),
                       max_rounds=int(getattr(p, "max_rounds", 0) or 0),
                       method=int(getattr(p, "method", 0) or 0), reserved=0)


def arpc_status_str(status: int) -> str:
    return lib().arpc_status_str(int(status)).decode()


def arpc_version() -> str:
    return lib().arpc_version().decode()


def arpc_workspace_size(problem: ArpcProblem) -> int:
    n = C.c_size_t(0)
    st = lib().arpc_workspace_size(C.byref(problem), C.byref(n))
    if st != ARPC_OK:
        raise ValueError(f"arpc_workspace_size: {arpc_status_str(st)}")
    return int(n.value)


def arpc_factor(problem: ArpcProblem, X_ptr: int, F_ptr: int, piv_ptr: int, ws_ptr: int,
                ws_bytes: int, stream: int):
    stats = ArpcStats()
    st = lib().arpc_factor(C.byref(problem), C.c_void_p(X_ptr), C.c_void_p(F_ptr), C.c_void_p(piv_ptr),
                           C.c_void_p(ws_ptr), C.c_size_t(ws_bytes), C.c_void_p(stream), C.byref(stats))
    return st, stats


def arpc_factor_async(problem: ArpcProblem, X_ptr: int, F_ptr: int, piv_ptr: int, ws_ptr: int, ws_bytes: int,
                      stream: int, rounds: int = 0) -> int:
    return lib().arpc_factor_async(C.byref(problem), C.c_void_p(X_ptr), C.c_void_p(F_ptr), C.c_void_p(piv_ptr),
                                   C.c_void_p(ws_ptr), C.c_size_t(ws_bytes), C.c_void_p(stream), C.c_int64(rounds))


def arpc_factor_continue(problem: ArpcProblem, X_ptr: int, F_ptr: int, piv_ptr: int, ws_ptr: int, ws_bytes: int,
                         stream: int, rounds: int) -> int:
    return lib().arpc_factor_continue(C.byref(problem), C.c_void_p(X_ptr), C.c_void_p(F_ptr), C.c_void_p(piv_ptr),
                                      C.c_void_p(ws_ptr), C.c_size_t(ws_bytes), C.c_void_p(stream),
                                      C.c_int64(rounds))


def arpc_factor_query(problem: ArpcProblem, ws_ptr: int, ws_bytes: int):
    stats = ArpcStats()
    st = lib().arpc_factor_query(C.byref(problem), C.c_void_p(ws_ptr), C.c_size_t(ws_bytes), C.byref(stats))
    return st, stats


def arpc_factor_uniforms(problem: ArpcProblem, X_ptr: int, F_ptr: int, piv_ptr: int, ws_ptr: int,
                         ws_bytes: int, stream: int, U_ptr: int, nU: int):
    stats = ArpcStats()
    st = lib().arpc_factor_uniforms(C.byref(problem), C.c_void_p(X_ptr), C.c_void_p(F_ptr),
                                    C.c_void_p(piv_ptr), C.c_void_p(ws_ptr), C.c_size_t(ws_bytes),
                                    C.c_void_p(stream), C.c_void_p(U_ptr), C.c_int64(nU), C.byref(stats))
    return st, stats


def arpc_lowmem_workspace_size(problem: ArpcProblem) -> int:
    n = C.c_size_t(0)
    st = lib().arpc_lowmem_workspace_size(C.byref(problem), C.byref(n))
    if st != ARPC_OK:
        raise ValueError(f"arpc_lowmem_workspace_size: {arpc_status_str(st)}")
    return int(n.value)


def arpc_factor_lowmem(problem: ArpcProblem, X_ptr: int, L_ptr: int, piv_ptr: int, ws_ptr: int,
                       ws_bytes: int, stream: int):
    stats = ArpcStats()
    st = lib().arpc_factor_lowmem(C.byref(problem), C.c_void_p(X_ptr), C.c_void_p(L_ptr), C.c_void_p(piv_ptr),
                                  C.c_void_p(ws_ptr), C.c_size_t(ws_bytes), C.c_void_p(stream), C.byref(stats))
    return st, stats


def arpc_qr_workspace_size(M: int, N: int, k: int, b: int) -> int:
    n = C.c_size_t(0)
    st = lib().arpc_qr_workspace_size(int(M), int(N), int(k), int(b), C.byref(n))
    if st != ARPC_OK:
        raise ValueError(f"arpc_qr_workspace_size: {arpc_status_str(st)}")
    return int(n.value)


def arpc_stream_uniforms_host(seed: int, start: int, n: int) -> np.ndarray:
    out = np.empty(n, dtype=np.float64)
    st = lib().arpc_stream_uniforms_host(C.c_uint64(seed), C.c_int64(start), C.c_int64(n),
                                         out.ctypes.data_as(C.c_void_p))
    if st != ARPC_OK:
        raise ValueError(arpc_status_str(st))
    return out


def arpc_set_profiling(on: bool) -> None:
    lib().arpc_set_profiling(1 if on else 0)


def arpc_set_profiling_classes(classes) -> None:
    """Time only the named kernel classes (names from KERNEL_CLASSES)."""
    mask = 0
    for c in classes:
        mask |= 1 << KERNEL_CLASSES.index(c)
    lib().arpc_set_profiling_classes(mask)


# ------------------------------------------------------------ torch convenience
def factor(X, problem, U=None, device: str = "cuda", stream=None, workspace=None):
    """Run the factorization on the GPU.  X: numpy (N x d) or a device tensor.
    Returns a dict with the device tensors F (N x k, column j = F[:, j]),
    pivots, and the status and stats.  Allocation only: all arithmetic runs in
    libarpc.so."""
    import torch

    if not torch.cuda.is_available():
        raise RuntimeError("the HIP library needs a GPU")
    pr = make_problem(problem)
    if isinstance(X, np.ndarray):
        Xd = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float64)).to(device)
    else:
        Xd = X.contiguous()
    fdt = torch.float64 if problem.prec == 0 else torch.float32
    # column-major N x k == row-major k x N
    Ft = torch.empty((problem.k, problem.N), dtype=fdt, device=device)
    piv = torch.empty(problem.k, dtype=torch.int64, device=device)
    nbytes = arpc_workspace_size(pr)
    ws = workspace if workspace is not None else torch.empty(nbytes, dtype=torch.uint8, device=device)
    s = stream if stream is not None else torch.cuda.current_stream()
    if U is None:
        status, stats = arpc_factor(pr, Xd.data_ptr(), Ft.data_ptr(), piv.data_ptr(), ws.data_ptr(),
                                    nbytes, s.cuda_stream)
    else:
        Ud = torch.as_tensor(np.asarray(U, dtype=np.float64)).to(device)
        status, stats = arpc_factor_uniforms(pr, Xd.data_ptr(), Ft.data_ptr(), piv.data_ptr(),
                                             ws.data_ptr(), nbytes, s.cuda_stream, Ud.data_ptr(),
                                             Ud.numel())
    if status < 0:
        raise RuntimeError(f"arpc_factor failed: {arpc_status_str(status)}")
    return {"F": Ft.t(), "pivots": piv, "status": status, "stats": stats.as_dict()}


def factor_lowmem(X, problem, device: str = "cuda", stream=None):
    """The low-memory implementation on the GPU.  Returns a dict with the
    device tensors L (k x k lower factor of A(S,S)) and pivots, the status and
    the stats.  Allocation only: all arithmetic runs in libarpc.so."""
    import torch

    if not torch.cuda.is_available():
        raise RuntimeError("the HIP library needs a GPU")
    pr = make_problem(problem)
    if isinstance(X, np.ndarray):
        Xd = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float64)).to(device)
    else:
        Xd = X.contiguous()
    # column-major k x k == row-major k x k transposed
    Lt = torch.empty((problem.k, problem.k), dtype=torch.float64, device=device)
    piv = torch.empty(problem.k, dtype=torch.int64, device=device)
    nbytes = arpc_lowmem_workspace_size(pr)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
    s = stream if stream is not None else torch.cuda.current_stream()
    status, stats = arpc_factor_lowmem(pr, Xd.data_ptr(), Lt.data_ptr(), piv.data_ptr(), ws.data_ptr(), nbytes,
                                       s.cuda_stream)
    if status < 0:
        raise RuntimeError(f"arpc_factor_lowmem failed: {arpc_status_str(status)}")
    return {"L": Lt.t(), "pivots": piv, "status": status, "stats": stats.as_dict()}


def qr_factor(B, k: int, b: int, seed: int = 0, max_rounds: int = 0, device: str = "cuda", stream=None):
    """Accelerated randomly pivoted QR on the GPU.  B: numpy (M x N) or a
    device tensor laid out column-major (the transpose of a contiguous N x M
    tensor).  Returns a dict with the device tensors Q (M x k), F (N x k),
    pivots, the status and the stats.  Allocation only."""
    import torch

    if not torch.cuda.is_available():
        raise RuntimeError("the HIP library needs a GPU")
    if isinstance(B, np.ndarray):
        M, N = B.shape
        Bt = torch.from_numpy(np.ascontiguousarray(np.asarray(B, dtype=np.float64).T)).to(device)   # N x M rows
    else:
        Bt = B.t().contiguous()
        N, M = Bt.shape
    Qt = torch.empty((k, M), dtype=torch.float64, device=device)
    Ft = torch.empty((k, N), dtype=torch.float64, device=device)
    piv = torch.empty(k, dtype=torch.int64, device=device)
    nbytes = arpc_qr_workspace_size(M, N, k, b)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
    s = stream if stream is not None else torch.cuda.current_stream()
    stats = ArpcStats()
    status = lib().arpc_qr_factor(int(M), int(N), int(k), int(b), C.c_uint64(seed), int(max_rounds),
                                  C.c_void_p(Bt.data_ptr()), C.c_void_p(Qt.data_ptr()), C.c_void_p(Ft.data_ptr()),
                                  C.c_void_p(piv.data_ptr()), C.c_void_p(ws.data_ptr()), C.c_size_t(nbytes),
                                  C.c_void_p(s.cuda_stream), C.byref(stats))
    if status < 0:
        raise RuntimeError(f"arpc_qr_factor failed: {arpc_status_str(status)}")
    return {"Q": Qt.t(), "F": Ft.t(), "pivots": piv, "status": status, "stats": stats.as_dict()}


def krr_pcg(X, y, F, kernel: int, sigma: float, mu: float, tol: float = 1e-8, max_iter: int = 1000,
            device: str = "cuda", stream=None):
    """(A + mu I) beta = y by PCG with P = F F^* + mu I on the GPU.  X, y:
    numpy or device tensors; F: a device tensor N x k (FP64 or FP32, column
    j = F[:, j], as factor() returns it) or None.  Returns a dict with the
    device tensor beta, the status and the stats.  Allocation only."""
    import torch

    if not torch.cuda.is_available():
        raise RuntimeError("the HIP library needs a GPU")
    Xd = torch.as_tensor(np.ascontiguousarray(X, dtype=np.float64) if isinstance(X, np.ndarray) else X,
                         device=device).contiguous()
    yd = torch.as_tensor(np.ascontiguousarray(y, dtype=np.float64) if isinstance(y, np.ndarray) else y,
                         device=device).contiguous()
    N, d = Xd.shape
    if F is None:
        k, f_prec, Fp = 0, 0, 0
    else:
        k = F.shape[1]
        Ft = F.t().contiguous()          # column-major N x k
        f_prec = 0 if Ft.dtype == torch.float64 else 1
        Fp = Ft.data_ptr()
    n = C.c_size_t(0)
    st = lib().arpc_krr_workspace_size(int(N), int(d), int(k), int(f_prec), C.byref(n))
    if st != ARPC_OK:
        raise ValueError(f"arpc_krr_workspace_size: {arpc_status_str(st)}")
    ws = torch.empty(int(n.value), dtype=torch.uint8, device=device)
    beta = torch.empty(N, dtype=torch.float64, device=device)
    s = stream if stream is not None else torch.cuda.current_stream()
    stats = ArpcKrrStats()
    status = lib().arpc_krr_pcg(int(N), int(d), int(kernel), float(sigma), float(mu), C.c_void_p(Xd.data_ptr()),
                                C.c_void_p(yd.data_ptr()), C.c_void_p(Fp), int(f_prec), int(k), float(tol),
                                int(max_iter), C.c_void_p(beta.data_ptr()), C.c_void_p(ws.data_ptr()), n,
                                C.c_void_p(s.cuda_stream), C.byref(stats))
    if status < 0:
        raise RuntimeError(f"arpc_krr_pcg failed: {arpc_status_str(status)}")
    return {"beta": beta, "status": status, "stats": stats.as_dict()}


# ------------------------------------------------------------------- serving
def arpc_create(device: int, budget_bytes: int, max_slots: int):
    ctx = C.c_void_p()
    st = lib().arpc_create(int(device), C.c_size_t(int(budget_bytes)), int(max_slots), C.byref(ctx))
    return st, ctx


def arpc_destroy(ctx) -> int:
    return lib().arpc_destroy(ctx)


def arpc_submit(ctx, problem: ArpcProblem, X_ptr: int, F_ptr: int, piv_ptr: int):
    job = C.c_uint64(0)
    st = lib().arpc_submit(ctx, C.byref(problem), C.c_void_p(X_ptr), C.c_void_p(F_ptr), C.c_void_p(piv_ptr),
                           C.byref(job))
    return st, job.value


def arpc_poll(ctx, job: int):
    done = C.c_int(0)
    stats = ArpcStats()
    st = lib().arpc_poll(ctx, C.c_uint64(job), C.byref(done), C.byref(stats))
    return st, bool(done.value), stats


def arpc_wait(ctx, job: int):
    stats = ArpcStats()
    st = lib().arpc_wait(ctx, C.c_uint64(job), C.byref(stats))
    return st, stats


def arpc_cancel(ctx, job: int) -> int:
    return lib().arpc_cancel(ctx, C.c_uint64(job))


def arpc_serving_set_limit(ctx, max_outstanding: int) -> int:
    return lib().arpc_serving_set_limit(ctx, C.c_int64(max_outstanding))


def arpc_serving_info(ctx) -> dict:
    out = ArpcServingStats()
    st = lib().arpc_serving_info(ctx, C.byref(out))
    if st != ARPC_OK:
        raise ValueError(arpc_status_str(st))
    return out.as_dict()


class Server:
    """A serving context plus the device buffers of its jobs (allocation and
    argument marshalling only; the scheduling runs in libarpc.so)."""

    def __init__(self, budget_bytes: int, max_slots: int = 8, device: int = 0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the HIP library needs a GPU")
        st, self.ctx = arpc_create(device, budget_bytes, max_slots)
        if st != ARPC_OK:
            raise RuntimeError(f"arpc_create failed: {arpc_status_str(st)}")
        self.device = torch.device("cuda", device)
        self.bufs = {}

    def submit(self, X, problem) -> int:
        """Queue a job on points X (numpy or device tensor); returns the handle."""
        import torch
        pr = make_problem(problem)
        if isinstance(X, np.ndarray):
            Xd = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float64)).to(self.device)
        else:
            Xd = X.contiguous()
        fdt = torch.float64 if problem.prec == 0 else torch.float32
        Ft = torch.empty((problem.k, problem.N), dtype=fdt, device=self.device)
        piv = torch.empty(problem.k, dtype=torch.int64, device=self.device)
        # inputs resident before the scheduler's streams read them (torch's own
        # stream only: a device-wide sync would also wait for running jobs)
        torch.cuda.current_stream(self.device).synchronize()
        st, job = arpc_submit(self.ctx, pr, Xd.data_ptr(), Ft.data_ptr(), piv.data_ptr())
        if st != ARPC_OK:
            raise RuntimeError(f"arpc_submit failed: {arpc_status_str(st)}")
        self.bufs[job] = (Xd, Ft, piv)
        return job

    def wait(self, job: int) -> dict:
        st, stats = arpc_wait(self.ctx, job)
        Xd, Ft, piv = self.bufs.pop(job)
        return {"F": Ft.t(), "pivots": piv, "status": st, "stats": stats.as_dict()}

    def poll(self, job: int):
        st, done, stats = arpc_poll(self.ctx, job)
        if not done:
            return None
        Xd, Ft, piv = self.bufs.pop(job)
        return {"F": Ft.t(), "pivots": piv, "status": st, "stats": stats.as_dict()}

    def cancel(self, job: int) -> int:
        return arpc_cancel(self.ctx, job)

    def info(self) -> dict:
        return arpc_serving_info(self.ctx)

    def close(self) -> None:
        if self.ctx is not None:
            arpc_destroy(self.ctx)
            self.ctx = None
