"""Sparse wavefunction UCC circuit solver for MI355X (HIP, gfx950).

The solver itself lives in the HIP shared library ``libswc.so`` behind the C
ABI declared in ``include/swc.h``; ``paper_2301_05726_amd.swc`` is its thin
Python binding.  Importing this package does not load the library, so the
input generator (``synth``) is usable on machines without a GPU.
"""
__all__ = ["synth", "swc"]
