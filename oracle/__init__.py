"""FP64 CPU oracle for the Galerkin boundary-integral Poisson-Boltzmann operator.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plainly written reference
that the GPU library is checked against.  Only the test-suite, the smoke check
and the CPU-baseline leg of the benchmark may import it; the product path never
does, and it shares no code with the HIP library.

Everything follows the paper (Cartesian FMM Galerkin BIE for linearised PB):
  * geometry, quadrature and kernels: Sec. 2.2-2.3 (Galerkin discretisation,
    Eq. for the kernels K1..K4 and the source terms S1, S2);
  * singular panel pairs: the Sauter-Schwab relative-coordinate idea (Sec. 2.3,
    last paragraph) rebuilt from its mathematics (see ``pairs``);
  * the FMM: Sec. 2.4 (moments, MtM, MtL, LtL, LtP and the six-step driver);
  * the block-diagonal preconditioner: Sec. 2.6;
  * the solvation energy: Eq. for E_sol in Sec. 2.3 and the unit factor of
    Sec. 3;
  * the Kirkwood reference: Sec. 3.1 (sphere with interior charges);
  * the continuous piecewise-linear space S^1_h of Sec. 2.3 (vertex hat
    functions as test and trial functions; see ``p1``).

Functions with no independent pin say "parity unpinned" in their docstring.
"""
