"""CPU oracle for the matrix-free HHG Stokes multigrid (Kohl & Ruede, "Textbook
efficiency: massively parallel matrix-free multigrid for the Stokes system").

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package: only the test-suite, the smoke check and the
benchmark's ``cpu_baseline`` leg use it.  It shares no code with the HIP
library (no kernels, headers, tables or constant generators); the only common
module is ``paper_2010_13513_amd/workloads.py``, which holds problem data and seeded random draws and none
of the method's arithmetic.

Everything here is plain float64 numpy/scipy written from the paper's
definitions:

* ``mesh``      -- macro mesh of the unit cube, Bey refinement, the uniformly
                   refined lattice, unknown counts (Sec. 2, 2.1, 2.2,
                   eq. num-unknowns-tet, Tab. unknown-count).
* ``fe``        -- P1 / P2 element matrices by exact barycentric integration and
                   global assembly of A, B, C, M (eq. stokes-discrete, eq. pspg).
* ``stokes``    -- the discrete saddle-point operator, right-hand sides,
                   boundary data, mean-zero projection.
* ``smoother``  -- multicolour ordering and the inexact Uzawa relaxation
                   (eq. uzawa-iteration / uzawa-velocity / uzawa-pressure) and
                   the omega estimate (eq. omega-eigenvalue-problem).
* ``transfer``  -- linear / quadratic prolongation and its transpose (Sec. 3.3).
* ``coarse``    -- dense pseudo-inverse coarse solve.
* ``multigrid`` -- variable V-cycle and FMG (Alg. fmg), error metrics
                   (eq. error, eq. gamma, eq. relative-error).
* ``workunits`` -- the work-unit cost model (Sec. 4).
* ``mlp``       -- float64 forward/backward of the coarse-grid MLP.

Pins (tests/test_oracle_*.py) tie each part to something other than itself:
closed forms, printed values of the paper, textbook identities, library
routines, brute force.
"""
