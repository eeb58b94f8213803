"""Host-side checks of the C ABI: the library loads, exports every function
that include/arpc.h declares, validates arguments, and its host copy of the
uniform stream equals the oracle's.  No GPU compute is launched here."""
import os
import re

import numpy as np
import pytest

from oracle import philox_stream
from paper_2410_03969_amd import binding as B
from paper_2410_03969_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "arpc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(arpc_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    lib = B.lib()
    names = declared_functions()
    assert len(names) >= 7
    for n in names:
        assert hasattr(lib, n), n
    assert set(B.EXPORTS) <= set(names)


def test_version_and_status_strings():
    assert B.arpc_version().startswith("arpc")
    assert B.arpc_status_str(0) == "ok"
    assert "invalid" in B.arpc_status_str(-1)
    assert B.arpc_status_str(12345) == "unknown status"


def test_struct_layout_matches_header(tmp_path):
    """Sizes and field offsets of the binding's structs equal what a C
    compiler makes of include/arpc.h."""
    import ctypes
    import subprocess
    fields = {"arpc_problem": [f for f, _ in B.ArpcProblem._fields_],
              "arpc_stats": [f for f, _ in B.ArpcStats._fields_],
              "arpc_serving_stats": [f for f, _ in B.ArpcServingStats._fields_],
              "arpc_krr_stats": [f for f, _ in B.ArpcKrrStats._fields_]}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "arpc.h"', 'int main(void){']
    for st, fs in fields.items():
        lines.append(f'printf("%zu\\n", sizeof({st}));')
        lines += [f'printf("%zu\\n", offsetof({st}, {f}));' for f in fs]
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I" + os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    want = []
    for cls in (B.ArpcProblem, B.ArpcStats, B.ArpcServingStats, B.ArpcKrrStats):
        want.append(ctypes.sizeof(cls))
        want += [getattr(cls, f).offset for f, _ in cls._fields_]
    assert got == want


def test_host_stream_matches_oracle_stream():
    for seed in (0, 1, 99, 2**63 + 5):
        for start in (0, 3, 4, 1001):
            assert np.array_equal(B.arpc_stream_uniforms_host(seed, start, 17),
                                  philox_stream(seed)(start, 17))


def _prob(**kw):
    base = dict(N=1000, d=3, k=50, b=10, kernel=W.GAUSSIAN, sigma=1.0, seed=0, prec=W.FP64)
    base.update(kw)
    return B.make_problem(W.Problem(**base))


def test_workspace_size_grows_with_problem():
    a = B.arpc_workspace_size(_prob())
    b = B.arpc_workspace_size(_prob(N=10_000))
    c = B.arpc_workspace_size(_prob(prec=W.FP32))
    assert 0 < a < b and c < a


@pytest.mark.parametrize("bad", [dict(N=0), dict(d=0), dict(k=0), dict(k=1001), dict(b=0),
                                 dict(b=1025), dict(sigma=0.0), dict(sigma=float("nan")),
                                 dict(sigma=float("inf")), dict(kernel=7), dict(prec=9), dict(prec=5),
                                 dict(method=2), dict(method=-1)])
def test_invalid_problems_rejected(bad):
    with pytest.raises(ValueError):
        B.arpc_workspace_size(_prob(**bad))


def test_reserved_field_must_be_zero():
    p = _prob()
    p.reserved = 1
    with pytest.raises(ValueError):
        B.arpc_workspace_size(p)


def test_fp8_workspace_holds_the_rounded_points():
    extra = B.arpc_workspace_size(_prob(prec=W.FP8, d=24)) - B.arpc_workspace_size(_prob(prec=W.BF16, d=24))
    assert extra >= 8 * 1000 * 24


def test_lowmem_rejects_unsupported_problems():
    good = dict(N=5000, d=3, k=100, b=20, kernel=W.GAUSSIAN, sigma=0.5, seed=0, prec=W.FP64)
    assert B.arpc_lowmem_workspace_size(B.make_problem(W.Problem(**good))) > 0
    for bad in (dict(prec=W.FP32), dict(method=W.BLOCK), dict(k=4097), dict(b=513, k=1000), dict(d=257)):
        with pytest.raises(ValueError):
            B.arpc_lowmem_workspace_size(B.make_problem(W.Problem(**{**good, **bad})))


def test_lowmem_workspace_is_far_below_the_factor():
    p = B.make_problem(W.Problem(N=1_000_000, d=8, k=2000, b=200, kernel=W.GAUSSIAN, sigma=2.0, prec=W.FP64))
    assert B.arpc_lowmem_workspace_size(p) < B.arpc_workspace_size(p) / 20


def test_factor_rejects_null_pointers_without_gpu_work():
    st, _ = B.arpc_factor(_prob(), 0, 0, 0, 0, 0, 0)
    assert st == B.ARPC_EINVAL
    st, _ = B.arpc_factor(_prob(), 8, 8, 8, 256, 10, 0)   # workspace too small
    assert st == B.ARPC_EINVAL
    st, _ = B.arpc_factor(_prob(), 8, 8, 8, 100, 1 << 40, 0)   # misaligned workspace
    assert st == B.ARPC_EINVAL


def test_serving_calls_validate_without_gpu():
    """Serving entry points reject bad arguments before touching a device; on a
    machine without a GPU, creating a context reports a device error."""
    lib = B.lib()
    import ctypes as C
    assert lib.arpc_create(0, 1 << 20, 0, C.byref(C.c_void_p())) == B.ARPC_EINVAL
    assert lib.arpc_create(0, 1 << 20, 65, C.byref(C.c_void_p())) == B.ARPC_EINVAL
    assert lib.arpc_create(0, 16, 4, C.byref(C.c_void_p())) == B.ARPC_EINVAL
    assert lib.arpc_destroy(None) == B.ARPC_EINVAL
    assert lib.arpc_submit(None, C.byref(_prob()), None, None, None, C.byref(C.c_uint64())) == B.ARPC_EINVAL
    assert lib.arpc_wait(None, 1, None) == B.ARPC_EINVAL
    assert lib.arpc_cancel(None, 1) == B.ARPC_EINVAL
    assert lib.arpc_serving_info(None, None) == B.ARPC_EINVAL
    try:
        import torch
        has_gpu = torch.cuda.is_available()
    except Exception:
        has_gpu = False
    if not has_gpu:
        st, ctx = B.arpc_create(0, 1 << 20, 4)
        assert st == B.ARPC_EDEVICE and not ctx.value
