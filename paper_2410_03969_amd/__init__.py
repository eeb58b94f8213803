"""Accelerated randomly pivoted Cholesky on MI355X (gfx950).

The computation lives in the HIP library ``libarpc.so`` (C ABI in
``include/arpc.h``); ``binding`` marshals arguments to it, ``workloads``
draws the seeded synthetic inputs, ``build`` compiles the library.
"""
__all__ = ["binding", "workloads", "build"]
