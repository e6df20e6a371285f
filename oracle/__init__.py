"""FP64 CPU oracle for the linear FDPB Jacobi-PCG solve.

TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package. The GPU library path
never imports, calls or links it, and it shares no code with that path.

Modules:
  fdpb  - setup (classification, edge dielectrics, salt term, trilinear
          charges, Debye-Hueckel boundary), the matrix-free operator of Eq. 3,
          the energy and a dense assembly for tiny grids.
  pcg   - the preconditioned CG listing of section 2.2 with the Jacobi
          preconditioner of section 2.4, and FP64 iterative refinement.
  solvation - the solvation energy from a solvent and a uniform reference
          solve on the same grid (the energies of section 3.1).
  periodic - the periodic-boundary setup, operator and energy (section 2.7's
          alternative boundary), with an exact FFT solver for uniform media.
  multigrid - geometric-multigrid-preconditioned CG on the same operator.
"""
from . import fdpb, multigrid, pcg, periodic, solvation  # noqa: F401
