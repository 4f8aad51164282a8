"""Batched SPHINCS+ (SLH-DSA, SHA2 "simple") signing on MI355X (gfx950).

The GPU library ``libslh.so`` (built from ``csrc/``) does all hashing; the
Python module ``slh`` only marshals arguments to its C ABI (declared in
``include/slh.h``), with PyTorch providing device memory and streams.
Importing this package imports nothing heavy; use ``from
paper_2512_23969_amd import slh``.
"""
