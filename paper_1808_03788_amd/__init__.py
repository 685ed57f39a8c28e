"""ADER-DG hot path for MI355X (gfx950).

The compute path is the HIP library ``libader.so`` behind the C ABI declared
in ``include/ader.h``; ``paper_1808_03788_amd.ader`` is its thin ctypes
binding.  ``paper_1808_03788_amd.inputs`` holds the seeded synthetic inputs
(problem descriptions and initial data) and none of the method's arithmetic.

Importing this package loads nothing; the binding loads the library on first
use and raises if it is missing.
"""
__all__ = ["inputs", "ader"]
