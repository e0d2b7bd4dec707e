"""FP64 CPU oracle for the planewave Dirac-Kohn-Sham eigenproblem and LOBPCG-F.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the GPU library and its
Python binding) may import, call, link or execute anything under ``oracle/``;
only the test suite, the smoke check and the CPU baseline leg of the benchmark
do.  The oracle shares no code with the GPU path: it consumes the seeded
physical inputs of ``sysgen`` and nothing else.

Everything here is plain numpy/scipy in float64/complex128, written to be read
against the paper:

* ``dks``      -- the planewave basis, the discretised DKS operator of Eq. (DKS)
                  with the local and separable spin-orbit parts of Eq. (HGH),
                  built densely and applied matrix-free through FFTs;
* ``lobpcgf``  -- the filter of Eq. (filter), Algorithm 1 (LOBPCG-F, and
                  plain LOBPCG when the filter is switched off), the filter
                  inside a block Davidson iteration, and the dense definition
                  of the answer: the lowest n eigenpairs of the positive
                  energy band;
* ``scf``      -- the self-consistent field loop around it: Eq. (density),
                  the Hartree and LDA parts of V_hxc, Fermi occupations and
                  Anderson mixing with the Kerker preconditioner (Sec. 4).

Every function names the passage it follows.  No function here is
"parity unpinned": each is checked in ``tests/test_oracle_*.py`` against
closed forms, invariants or brute force.
"""
from . import dks, lobpcgf, scf  # noqa: F401
