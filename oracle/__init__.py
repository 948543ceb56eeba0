"""CPU float64 oracle for the eigenfunction-segregation time step.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow reference that the
GPU library is checked against.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the product path never does, and
it shares no code with the HIP library (the two meet only in the seeded input
generators of the ``workloads`` package).

What it computes follows Elliott & Ranner, "A computational approach to an
optimal partition problem on surfaces" (arXiv 1408.2355):

* ``fem``     consistent P1 mass and stiffness matrices on a triangulated
              surface (Section 2.1, the finite element spaces S_h);
* ``flow``    one step of the operator-splitting scheme, Algorithm 2.2 (the
              implicit-Euler heat step, the exact per-node ODE solution of the
              practical step 2 written as its defining sum over j != i, the
              L2 renormalisation), the random start of Section 2.2, and the
              run loop with the energy cadence and stopping rule of Section
              2.2;
* ``energy``  the Rayleigh-quotient eigenvalue estimates (Section 3.2: mean
              H1-seminorm of unit-L2 components), the regularisation energy
              S_eps of equation (Seps-u) integrated exactly per triangle, and
              E = sum_i lambda_i + S_eps;
* ``labels``  the partition read off v_i = u_i - sum_{j != i} u_j
              (equation (vi)).

All arithmetic is float64.  The heat step is solved directly (sparse LU):
the oracle computes the exact solution of the linear system the paper
defines, not an iteration towards it.
"""
from . import fem, flow, energy, labels  # noqa: F401
