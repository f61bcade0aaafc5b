"""CPU oracle for the tensor-train finite-volume SWE solver (Danis et al., arXiv 2408.03483).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package: only the
tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` use it.
It shares no code, table or helper with the GPU library.

Modules
  stencils  exact reconstruction weights (Section 2.3), derived from cell-average moments
  fv_grid   plain full-grid finite-volume solver (Sections 2.2-2.4): Upwind3/Upwind5/WENO5
            reconstruction, Gauss-Legendre face quadrature, local Lax-Friedrichs flux, SSP-RK3
  tt        plain 2-core tensor-train algebra (Section 3): rounding, sums, Hadamard products,
            norms, the Taylor reciprocal (Algorithm 1), maxvol and cross interpolation
  tt_fv     the TT finite-volume step (Section 4) as the fixed sequence of TT operations

All arithmetic is float64 (numpy / LAPACK).
"""
