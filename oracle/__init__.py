"""Plain, slow FP64 CPU oracle for accelerated randomly pivoted Cholesky.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The GPU library shares
no code with it: no kernels, no headers, no helpers, no constants.

Contents (each function cites the passage of Epperly, Tropp & Webber,
"Embrace rejection: kernel matrix approximation by accelerated randomly
pivoted Cholesky", arXiv 2410.03969, that it follows):

* ``stream``  - the uniform stream that replaces the paper's ``Rand()``
* ``kernels`` - kernel functions evaluated by direct differences
* ``fp8``     - rounding to FP8 e4m3 (the point set of the FP8 mode)
* ``rpqr``    - accelerated randomly pivoted QR (Alg. 5)
* ``krr``     - kernel ridge regression by PCG with P = F F^* + mu I (Section 3.2)
* ``rpc``     - simple RPCholesky (Alg. 6), block RPCholesky (Alg. 7),
                RejectionSampleSubmatrix (Alg. 1), accelerated
                RPCholesky (Alg. 2) and its low-memory implementation
                (Alg. 3), plus Nystrom/closed-form checkers.
"""
from .stream import philox_stream, array_stream  # noqa: F401
from .kernels import kappa, kernel_block  # noqa: F401
from .fp8 import round_e4m3  # noqa: F401
from .rpqr import orth, rpqr_accel  # noqa: F401
from .krr import kernel_matvec, krr_pcg, pcg, woodbury_apply  # noqa: F401
from .rpc import (PointsAccess, ExpandedPointsAccess, DenseAccess, rpc_accel, rpc_accel_lowmem, rpc_plain, rpc_block,  # noqa: F401
                  reject_sample_submatrix, factor_from_pivots, nystrom_err,
                  draw_proposals)
