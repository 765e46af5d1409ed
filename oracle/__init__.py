"""CPU oracle for PLSS (Brust & Saunders, "PLSS: A Projected Linear Systems
Solver", arXiv:2207.07615).

TEST INFRASTRUCTURE ONLY.  Nothing in the solver library may import, call or
link anything in this package; only the tests, the smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the GPU path.

Contents (plain, slow, obviously correct; float64 unless stated):

* ``sparse``  CSR validation, CSR product, stable CSR -> CSC transpose.
* ``plss``    Algorithm 1 (residual sketch, optional diagonal W) and the
              general one-column sketch step (identity / mixed / residual
              sketches, Sections 2.5-2.6 and 7).
* ``blocks``  PLSS with a sketch grown by a block of columns per step (block
              identity, or residual plus identity columns), by the block form
              of the triangular update of Section 2.4.
* ``randproj`` The paper's randomized-projection comparison (eq. pkLong with
              a fresh standard normal sketch each iteration), with
              Philox4x32-10 and Box-Muller written from their published
              definitions so the GPU can draw the same sketches.
* ``exact``   The same iterations in rational arithmetic
              (``fractions.Fraction``) on small integer systems, plus a
              rational minimum-norm solve.
* ``pins``    Independent routines the oracle is checked against: a dense
              brute-force evaluation of eq. (pkLong), Craig's method via
              Golub-Kahan bidiagonalisation (Section 6), the textbook
              Kaczmarz sweep (Section 7) and the dense minimum-norm solution.

Readings of points where the paper is silent or inconsistent are stated at
the functions that take them.
"""
