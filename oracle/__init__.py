"""Plain CPU reference (the oracle) for the sketch / Gram / row-norm /
least-squares path of "pylspack: Parallel algorithms and data structures for
sketching, column subset selection, regression and leverage scores"
(Sobczyk & Gallopoulos, arXiv 2203.02798).

TEST INFRASTRUCTURE ONLY.  It is deliberately slow and obvious: NumPy/SciPy in
FP64, written from the paper's definitions, sharing no code with the device
library.  Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` may import it; the product path never routes through it.

Modules
-------
philox   Philox4x32-10 counter-based generator (Salmon et al., SC'11).
sketch   CountSketch hash, explicit S, S*A, Gaussian G, G*S*A (Def. 3,
         Alg. ``bcs_multiply`` / ``countgauss_multiply``), quantisers for the
         reduced-precision Gaussian GEMM.
gram     Gram matrix and squared row norms (Alg. ``gram_serial``, ``gram``,
         ``squared_row_norms``).
leverage QR of the sketch, R^{-1}, sketched and exact leverage scores
         (Alg. ``ls_approximate_drineas`` with QR instead of SVD).
lsq      Least squares: LAPACK ground truth and sketch-and-precondition LSQR
         (Alg. ``least_squares_precondition``).
osnap    OSNAP with s > 1 non-zeros per column (the generalisation of
         CountSketch of Section 2's introduction), its S*A and G*S*A.
css      Column subset selection by the pivoted QR of a sketch.

Parity status: every function is pinned by a ``-m "not gpu"`` test in
``tests/test_oracle_*.py`` against something other than itself (published
Philox answers and rocRAND's Philox, the paper's worked CountSketch example,
closed forms, invariants, brute force on tiny inputs).
"""
