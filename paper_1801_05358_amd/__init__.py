"""Dual messenger Wiener filter for CMB (I, Q, U) maps on the sphere, on
AMD MI355X (gfx950).

The compute path is the C-ABI library ``libdmwf.so`` built from ``csrc/``
(hand-written HIP kernels); ``dmwf`` is its thin ctypes binding.  ``inputs``
holds the seeded synthetic workload recipes.  Submodules are imported
explicitly so that reading the recipes never loads the GPU library.
"""
__all__ = ["dmwf", "inputs"]
