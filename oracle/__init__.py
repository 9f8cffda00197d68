"""Plain FP64 CPU oracle for tree-level QCD |M|^2 (test infrastructure only).

This package is test infrastructure.  Only the test-suite, the smoke check and
the CPU-baseline leg of the benchmark may import it; the product library never
does, and the two share no code.

What it computes is the plain definition of the colour- and helicity-summed,
spin- and colour-averaged squared matrix element of the paper (section 2.1,
eqs. matrix-element, color-amplitude, color-matrix, color-averaged-amplitude):

    |M|^2 = 1/4 * sum_lambda  sum_{alpha,beta} J_alpha N_{alpha beta} J_beta^*
    J_alpha = sum_d c_{d alpha} A_d

* every tree Feynman diagram is enumerated independently (no shared currents)
  and evaluated with explicit 4x4 Dirac matrices and textbook QCD Feynman rules
  (covariant derivative D = d - i g A^a t^a, Feynman gauge);
* colour factors are explicit tensors built from the Gell-Mann matrices
  (t = lambda/2) and f^{abc}; the colour basis is the one the paper describes
  (single traces for gluons, chains for one quark line, chain pairs with one
  shared adjoint index for two quark lines); the decomposition coefficients
  c_{d alpha} are obtained by solving C_d(c) = sum_alpha c_{d alpha} T_alpha(c)
  numerically and the colour matrix is the literal sum over all colour
  assignments, divided by n_a n_b.

Everything is float64 / complex128 numpy, vectorised over events and helicity
configurations, written for reading rather than speed.
"""
from .process import OracleProcess, parse_process  # noqa: F401
from .me2 import oracle_me2, oracle_amplitudes  # noqa: F401
