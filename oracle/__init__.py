"""Plain FP64 CPU oracle for the all-at-once Stokes/Oseen optimal-control solver.

TEST INFRASTRUCTURE ONLY.  This package exists so that the HIP path can be
checked against a slow, obviously correct implementation written directly from
the paper (Heinzelreiter & Pearson, "Diagonalization-Based Parallel-in-Time
Preconditioners for Instationary Fluid Flow Control Problems").  Only the test
suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py``
may import it.  The product path (``paper_2405_18964_amd``) never imports,
links or calls anything here, and this package imports nothing from the product
path.  The only code both sides share is the seeded input generator in
``workloads``, which holds none of the method's arithmetic.

Modules
-------
fem        Q2-Q1 finite-element matrices on the uniform unit-square grid
           (section 2.2), assembled element by element with 3x3 Gauss, plus an
           independent Kronecker-product route used to pin the assembly.
kkt        the all-at-once matrix of eq. (FinalA), its right-hand side, a sparse
           direct solve and the sequential time-stepping (reduced-gradient)
           check of the optimality system (section 2.1/2.2).
circulant  the circulant perturbation P_C, its FFT diagonalisation and the
           per-frequency blocks G_j (section 3.1, eq. SubBlockG).
smoothers  multicolour SOR over whole grids (the reading of section 3.4), the
           tiled variant a GPU may run (tile sizes passed in by the caller),
           Chebyshev semi-iteration (section 3.4).
mg         geometric multigrid V-cycles (section 3.4), and exact solves that
           stand in for them in the pins of the block compositions.
precond    the Stokes preconditioners of section 3.2-3.4 (Algorithms 1 and 2)
           and the Oseen preconditioner of section 4 (Algorithm 3).
krylov     right-preconditioned GMRES and flexible GMRES.

Parity status: every function is pinned by a ``-m "not gpu"`` test.  The
multigrid V-cycle is pinned to the textbook two-/three-grid error propagation
operator assembled from dense smoother, transfer and coarse matrices; its
contraction rate is a property of that operator (no closed form) and is only
checked for being a contraction.  The block compositions of section 3.2 and
section 4 (P~_j^{-1}, the Uzawa Schur block, the pressure Schur step and the
second step of Algorithm 3) are pinned, with exact inner inverses, to dense
evaluations of the paper's product forms, and planted mistakes each fail.
"""
