"""CPU oracle for the eSIA / nSIA hot path (arXiv 1702.05854).

TEST INFRASTRUCTURE ONLY: the test suite, the package smoke check and the
benchmark's CPU-baseline leg are the only callers.  Nothing here imports the
product package's kernels or binding, and the product never imports this.

* ``oracle.cpu``   -- ctypes binding of the plain single-threaded C oracle
  (``sia_oracle.c``): Philox, thresholds, sampler, counts, greedy, estimates.
* ``oracle.exact`` -- exact rational enumeration on tiny graphs (live-edge
  graphs, HSAW path sums, the sampler's walk tree).
"""
