"""CPU oracle for block Krylov time stepping (arXiv 2504.02117).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) imports, links or runs anything here; only the tests, the smoke
check and the benchmark's CPU-baseline leg do.

The oracle is plain, slow and FP64 throughout.  It computes what the paper's
method converges to, by the plain definitions:

* ``fv``           cell-centred finite-volume operators (linear and nonlinear)
                   for the semi-discrete problem ``M y' + K y = b`` and
                   ``M y' + f(t, y) = 0`` (Sec. 1, eq. problem; Sec. 2.2).
* ``timecoupling`` Butcher tableaux and the all-at-once time-stepping matrices
                   ``A1``, ``A2``, ``B0`` (Sec. 2.1, eq. general-system-time-steps,
                   eq. time-stepping-matrices-multiple-parallel-time-steps,
                   Example 2) and their pipelined windows (Sec. 2.2,
                   eq. matrix-equation-pipelining).
* ``allatonce``    the Kronecker all-at-once system, its matrix-equation
                   residual and the splitting fixed point (Sec. 2.1,
                   eq. matrix-splitting, eq. matrix-fixed-point-equation).
* ``stepping``     sequential stiffly accurate DIRK time stepping with a direct
                   or simple iterative per-stage solve (Sec. 2,
                   eq. stiffly-accurate-DIRK) -- the result the all-at-once
                   method must reproduce.
* ``richards``     Richards' equation with the van Genuchten closure on an FV grid
                   (Sec. 4.3, eq. RelationshipsThetaK), its exact Jacobian, the
                   window residual with a split mass term and sequential implicit
                   Euler with Newton and direct solves.
* ``cstep``        the same sequential implicit Euler with Jacobi-PCG in plain C
                   (``seqstep.c``, OpenMP), for full-size checks and the
                   all-core CPU baseline.
* ``multigrid``    the geometric V-cycle that defines this library's own
                   multigrid preconditioner (the paper uses AMG without details).
* ``blockops``     plain definitions of the block kernels (block operator,
                   Gram matrices, block solves) used for kernel parity.

It shares no code with the HIP path.  The only module both sides import is
``paper_2504_02117_amd.inputs``, which generates seeded input data and holds
none of the method's arithmetic.

Every function here is pinned by ``tests/test_oracle_*.py`` against facts the
paper or the mathematics fix (worked example, closed-form eigen-decay,
brute-force dense solves, triangular structure, conservation, finite
differences); none is "parity unpinned".
"""
