"""FP64 CPU oracle of the VEGAS hot path — TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check of the entry module and the CPU-baseline
leg of the benchmark may import anything from this package.  The product path
(the HIP library and its Python binding) never calls it and must fail loudly
when its compiled extension is missing.

The oracle is plain, slow and written to be checked against the thesis by
eye: each function cites the passage it follows.  It shares no code with the
GPU path; both consume the seeded inputs of the ``synth`` package and each
implements the Philox generator from its published definition.

Modules
  philox     counter-based generator (published method, not in the thesis)
  vegas      map, estimator, combination, refinement (thesis Sec. "Adaptive
             Monte Carlo: VEGAS algorithm", importance-sampling equations)
  integrands Gaussian product and Genz families (test integrands)
  pdf        log-bicubic / bilinear interpolation on subgrids (thesis Sec.
             on LHAPDF interpolation and the PDFFlow design)
  ttbar      LO pp -> t tbar integrand from the master formula
  flow       piecewise-linear coupling flow, its variance loss, gradients and
             the Adam update (thesis Sec. on optimisers, Adam equations)

Parity status of every function is listed in its module header; a function
with no independent pin says "parity unpinned".
"""
