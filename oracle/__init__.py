"""CPU oracle for the all-slabs-at-once space-time multigrid V-cycle.

TEST INFRASTRUCTURE ONLY. This package is a plain, slow, FP64 NumPy/SciPy
statement of what the GPU library computes, written from the paper
("A parallel space-time multigrid method for the eddy-current equation",
Neumueller & Schwalsberger, 2019). It shares no code with the library; only
the test suite, the smoke check and the benchmark's CPU-baseline leg may
import it. The library must never route through it.

Modules
-------
mesh       topology: edges, faces, boundary, discrete gradient G, discrete curl C
fem        lowest-order Nedelec (Whitney) mass and curl-curl matrices, P1 sigma-stiffness
dgtime     upwind DG-in-time matrices for degree 0 (implicit Euler, eq. (1)) and 1
hierarchy  space-time levels with the coarsening rule (eq. (3)), transfers, Galerkin operators
vcycle     residual, block-Jacobi smoother (eq. (2)), nodal correction (eq. (8)),
           SAS V-cycle, outer solve and power-iteration rate
manufactured  the manufactured-solution right-hand side and initial value

Parity status (each pin lives in tests/test_oracle_*.py):
  * topology, assembly, DG-in-time, transfers, smoother, nodal correction,
    V-cycle fixed point: pinned (integer identities, closed forms, brute force,
    direct sparse solve of the whole space-time system).
  * absolute cycle counts / convergence rates: parity unpinned against the
    paper (the paper's meshes, boundary conditions and spatial solvers differ);
    only qualitative bounds from the paper are checked.
"""
