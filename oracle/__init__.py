"""Plain CPU oracle for the per-contingency screening loop.

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously-correct
reference that the GPU path is checked against.  Only the test-suite, the
smoke check and the CPU-baseline leg of the benchmark may import it; the
product library never calls it.  It shares no code with the HIP path.

Everything is float64 NumPy/SciPy, one scenario at a time, following the
paper's steps in order:
  Section II.A   enumeration (N-1, N-2)                 -> screen.py
  Section II.B.3 islanding by graph search              -> islanding.py
  Section II.B.1 AC OPF feasibility and limits          -> opf.py
  Section II.B.2 linearised state matrix, eigenvalues   -> dynamics.py, eigen.py
  Section II.C   frequencies and Risk Index, eq. (1)-(3) -> risk.py
"""
