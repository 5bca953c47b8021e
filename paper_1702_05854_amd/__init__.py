"""HSAW-based spread interdiction (eSIA / nSIA, arXiv 1702.05854) on MI355X.

The compute path is the HIP library ``libsia.so`` (kernels for gfx950 behind a
C ABI declared in ``include/sia.h``); ``paper_1702_05854_amd.sia`` is the thin
ctypes binding over it.  ``paper_1702_05854_amd.workloads`` holds the seeded
synthetic input generators.  Importing the package loads nothing native; the
binding loads the library on first use and raises if it is missing.
"""
