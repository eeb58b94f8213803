"""The uniform stream that drives every random decision.

The paper only writes ``Rand()`` (Alg. 1, acceptance test) and "sample iid
from u" (Alg. 2, step 1).  Reading fixed here: word p of the stream is the
p-th 64-bit output of numpy's ``Philox(key=seed)`` (Philox4x64 with 10
rounds, Salmon et al., SC'11), and its uniform is ``(word >> 11) * 2**-53``,
which lies in [0, 1).  Round r of the block algorithm consumes exactly 2b
words: proposal l uses word 2br + l, acceptance test i uses word 2br + b + i.
"""
from __future__ import annotations

import numpy as np


def philox_stream(seed: int):
    """Return ``f(start, n) -> float64[n]``: uniforms for words start..start+n-1."""
    seed = int(seed)

    def words(start: int, n: int) -> np.ndarray:
        start = int(start)
        # numpy's generator with counter c emits block c+1 first; block q holds
        # words 4q..4q+3.
        g = np.random.Philox(key=seed, counter=start // 4)
        raw = g.random_raw(n + start % 4)[start % 4:]
        return (raw >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)

    return words


def array_stream(U):
    """A stream backed by an explicit array of uniforms (adversarial tests)."""
    U = np.asarray(U, dtype=np.float64)

    def words(start: int, n: int) -> np.ndarray:
        if start + n > U.size:
            raise IndexError("explicit uniform stream exhausted")
        return U[start:start + n].copy()

    return words
