"""CPU FP64 oracle for the quasi-periodic Dirichlet scattering solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
anything here; only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may use it.  It shares no code with the GPU library.

What it computes is the *defining dense problem*, not the fast method: the
Nystrom matrix A = I/2 + D - i omega S of the isolated obstacle (Sec. 2.2, its
discretization in Sec. 2.3), the periodizing blocks B, C, Q (Eqs. 2.16-2.18,
Sec. 2.3), the bordered system (Eq. 2.19 / 2.21) solved by dense LU, and the
outputs (Bragg amplitudes, Remarks 2.2/2.3; flux error, Remark 6.1).  The
hierarchical (HBS) inverse of Sec. 4 is an approximation to tolerance, so the GPU
path is judged against this exact dense solve.

Modules:
  quadrature  Kapur-Rokhlin 6th-order end corrections (derived, Sec. 2.3) and the
              Kress spectral log-split weights.
  nystrom     curve discretization, kernel, dense A, neighbour images A_j, fields.
  periodic    Sommerfeld contour, B, C, Q, bordered solve, Bragg amplitudes, flux.
  transmission  the transmission problem of Sec. 5: the interlaced 2 x 2 Mueller-type
              operator at wavenumbers omega and n omega, its B, C, Bragg amplitudes.

Each function names the passage of the paper it follows.  Readings of passages
that are silent or misprinted are listed in the module docstrings.
"""
